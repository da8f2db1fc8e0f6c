"""Thin ctypes binding of libmlcc.so (the C ABI in include/mlcc.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Arrays may be NumPy arrays (host) or torch CUDA tensors (device);
torch is used only for device memory and streams.  The library must be built
(``python -m paper_2006_05226_amd.build``); importing this module without it
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlcc.so")

OK, PENDING = 0, 1
E_ARG, E_OOM, E_NOCONV, E_NUMERIC, E_DEVICE, E_BUSY, E_STATE = -1, -2, -3, -4, -5, -6, -7
CCS, MLCC2, MLCCSD, MLCCSD3 = 0, 1, 2, 3
FP64, FP32 = 0, 1
MODEL = {"ccs": CCS, "mlcc2": MLCC2, "mlccsd": MLCCSD, "mlccsd3": MLCCSD3}
BF16X3, BF16 = 2, 3
PREC = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "bf16": BF16}

_STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "E_ARG", -2: "E_OOM", -3: "E_NOCONV",
                 -4: "E_NUMERIC", -5: "E_DEVICE", -6: "E_BUSY", -7: "E_STATE"}


class ProblemDesc(C.Structure):
    _fields_ = [("n_occ", C.c_int32), ("n_vir", C.c_int32), ("n_chol", C.c_int32),
                ("n_occ_act", C.c_int32), ("n_vir_act", C.c_int32), ("model", C.c_int32),
                ("precision", C.c_int32), ("L", C.c_void_p), ("eps", C.c_void_p),
                ("flags", C.c_uint32), ("seed", C.c_uint64), ("fock", C.c_void_p),
                ("n_occ_ccsd", C.c_int32), ("n_vir_ccsd", C.c_int32)]


SYNTH_L = 1
INPUT_ON_DEVICE = 2
DETERMINISTIC = 4


class SolverOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("diis_dim", C.c_int32),
                ("max_subspace", C.c_int32), ("n_guess", C.c_int32), ("effective", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double),
                ("energy", C.c_double), ("complex_roots", C.c_int32), ("transforms", C.c_int32)]


class ServerOpts(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_queue", C.c_int32), ("hbm_budget", C.c_uint64),
                ("host_budget", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("n_roots", C.c_int32), ("omega", C.c_double * 16),
                ("e_corr", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("gs_iterations", C.c_int32),
                ("es_iterations", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("ms", C.c_double),
                ("flops", C.c_double)]


EXPORTS = ["mlcc_context_create", "mlcc_context_destroy", "mlcc_last_error", "mlcc_context_bytes",
           "mlcc_problem_create", "mlcc_problem_destroy", "mlcc_problem_dims",
           "mlcc_set_amplitudes", "mlcc_residual", "mlcc_ground_state",
           "mlcc_jacobian_transform", "mlcc_jacobian_transform_eff", "mlcc_davidson_solve",
           "mlcc_server_create", "mlcc_server_destroy", "mlcc_submit", "mlcc_poll",
           "mlcc_request_footprint", "mlcc_gemm", "mlcc_gemm2", "mlcc_gemm_noalloc",
           "mlcc_debug_get", "mlcc_profile_enable", "mlcc_profile_get", "mlcc_gemm_tile", "mlcc_cnto",
           "mlcc_pair_block_occ", "mlcc_cholesky_basis", "mlcc_mo_cholesky", "mlcc_bf16_map",
           "mlcc_gemm_planes"]

NOALLOC_SCRATCH_BYTES = 16 << 20

_lib = None


def load(path: str = LIB_PATH):
    """Load the library and declare the signatures (no device call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_2006_05226_amd.build")
    lib = C.CDLL(path)
    vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    P = C.POINTER
    sig = {
        "mlcc_context_create": (i32, [C.c_int, vp, u64, P(vp)]),
        "mlcc_context_destroy": (i32, [vp]),
        "mlcc_last_error": (C.c_char_p, [vp]),
        "mlcc_context_bytes": (u64, [vp]),
        "mlcc_problem_create": (i32, [vp, P(ProblemDesc), P(vp)]),
        "mlcc_problem_destroy": (i32, [vp]),
        "mlcc_problem_dims": (i32, [vp, P(i64)]),
        "mlcc_set_amplitudes": (i32, [vp, vp, vp]),
        "mlcc_residual": (i32, [vp, vp, vp, vp, P(dbl)]),
        "mlcc_ground_state": (i32, [vp, P(SolverOpts), vp, P(dbl), P(Info)]),
        "mlcc_jacobian_transform": (i32, [vp, i32, vp, vp]),
        "mlcc_jacobian_transform_eff": (i32, [vp, dbl, i32, vp, vp]),
        "mlcc_davidson_solve": (i32, [vp, i32, P(SolverOpts), vp, vp, P(Info)]),
        "mlcc_server_create": (i32, [vp, P(ServerOpts), P(vp)]),
        "mlcc_server_destroy": (i32, [vp]),
        "mlcc_submit": (i32, [vp, P(ProblemDesc), i32, P(SolverOpts), P(SolverOpts), P(u64)]),
        "mlcc_poll": (i32, [vp, u64, P(Result)]),
        "mlcc_request_footprint": (u64, [P(ProblemDesc), i32, P(SolverOpts)]),
        "mlcc_gemm": (i32, [vp, i32, i64, i64, i64, i64, i64, dbl, vp, P(i64), vp, P(i64), dbl,
                            vp, P(i64)]),
        "mlcc_gemm2": (i32, [vp, i32, i64, i64, i64, i64, i64, dbl, vp, P(i64), vp, P(i64), dbl,
                             vp, P(i64), P(i64)]),
        "mlcc_gemm_noalloc": (i32, [vp, i32, i64, i64, i64, i64, i64, dbl, vp, P(i64), vp, P(i64),
                                    dbl, vp, P(i64), P(i64)]),
        "mlcc_debug_get": (i32, [vp, i32, vp]),
        "mlcc_profile_enable": (i32, [vp, i32]),
        "mlcc_profile_get": (i32, [vp, P(KernelStat), i32]),
        "mlcc_gemm_tile": (i32, [vp, i32, i32, P(i32)]),
        "mlcc_gemm_planes": (i32, [vp, i32]),
        "mlcc_pair_block_occ": (i32, [vp, i32]),
        "mlcc_bf16_map": (i32, [vp, C.c_char_p]),
        "mlcc_cholesky_basis": (i32, [vp, i32, vp, vp, dbl, i32, vp, P(i32), vp]),
        "mlcc_mo_cholesky": (i32, [vp, i32, i32, i32, vp, i32, vp, vp, vp, i32, vp]),
        "mlcc_cnto": (i32, [vp, i32, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class MlccError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(a):
    """Data pointer of a NumPy array or a torch tensor (device or host)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous, "arrays must be C-contiguous"
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        assert a.is_contiguous(), "tensors must be contiguous"
        if getattr(a, "is_cuda", False):
            # the library's stream does not wait for torch's: finish the work
            # that produced this tensor (an upload, a fill) first
            import torch
            torch.cuda.current_stream(a.device).synchronize()
        return a.data_ptr()
    raise TypeError(type(a))


def _f64(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.float64)
    return a


def opts(tol=1e-8, max_iter=100, diis_dim=8, max_subspace=0, n_guess=0, effective=False):
    return SolverOpts(tol, max_iter, diis_dim, max_subspace, n_guess, 1 if effective else 0)


class Context:
    def __init__(self, device=0, stream=None, hbm_budget=0):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.mlcc_context_create(device, stream, hbm_budget, C.byref(h))
        if st != OK:
            raise MlccError(st, self.lib.mlcc_last_error(None).decode())
        self.h = h

    def check(self, st, ok=(OK,)):
        if st not in ok:
            raise MlccError(st, self.lib.mlcc_last_error(self.h).decode())
        return st

    def last_error(self):
        return self.lib.mlcc_last_error(self.h).decode()

    def bytes(self):
        return self.lib.mlcc_context_bytes(self.h)

    def gemm(self, prec, M, N, K, R, Z, alpha, A, sA, B, sB, beta, Cm, sC):
        a4 = (C.c_int64 * 4)(*sA)
        b4 = (C.c_int64 * 4)(*sB)
        c3 = (C.c_int64 * 3)(*sC)
        return self.check(self.lib.mlcc_gemm(self.h, prec, M, N, K, R, Z, alpha, _ptr(A), a4,
                                             _ptr(B), b4, beta, _ptr(Cm), c3))

    def gemm_noalloc(self, prec, M, N, K, R, Z, alpha, A, sA, B, sB, beta, Cm, sC, lvl=None):
        """mlcc_gemm_noalloc: the engine with its split partial sums in the
        library's fixed device array; enqueued on the context stream, not
        waited for."""
        a4 = (C.c_int64 * 4)(*sA)
        b4 = (C.c_int64 * 4)(*sB)
        c3 = (C.c_int64 * 3)(*sC)
        l6 = None if lvl is None else (C.c_int64 * 6)(*lvl)
        return self.check(self.lib.mlcc_gemm_noalloc(self.h, prec, M, N, K, R, Z, alpha, _ptr(A),
                                                     a4, _ptr(B), b4, beta, _ptr(Cm), c3, l6))

    def gemm_tile(self, bm=0, bn=0):
        """Force the bm x bn output tile on later engine calls of this context
        whose tile menu has it (0, 0: the cost model picks); returns the tile of
        the context's previous engine call."""
        last = (C.c_int32 * 2)()
        self.check(self.lib.mlcc_gemm_tile(self.h, bm, bn, last))
        return (last[0], last[1])

    def gemm_planes(self, mode=0):
        """Packed BF16 planes for the split and plain BF16 products of this
        context: 0 where the cost rule picks them, 1 wherever allowed, -1
        never."""
        self.check(self.lib.mlcc_gemm_planes(self.h, mode))

    def bf16_map(self, tags=None):
        """Contractions that run plain BF16 products in precision "bf16" on
        problems created afterwards: a list of names, [] for none, None for
        the built-in map."""
        arg = None if tags is None else ",".join(tags).encode()
        self.check(self.lib.mlcc_bf16_map(self.h, arg))

    def pair_block_occ(self, occ=0):
        """Occupied indices per pair block of the MLCC2 doubles on this
        context's problems (0: the memory rule)."""
        self.check(self.lib.mlcc_pair_block_occ(self.h, occ))

    def cholesky_basis(self, n_ao, G, tau, nu=None, max_vectors=None):
        """Pivots and Q^-T of the Cholesky basis of the AO pair matrix G
        (mlcc_cholesky_basis); nu: MO screening weights or None.  Q^-T is
        returned only when max_vectors^2 doubles (default max_vectors: every
        pair) fit in 1 GiB; otherwise None (pivots only): pass max_vectors."""
        npair = n_ao * (n_ao + 1) // 2
        cap = npair if max_vectors is None else max_vectors
        piv = np.empty(cap, dtype=np.int32)
        nv = C.c_int32()
        QiT = np.empty(cap * cap) if cap * cap <= (1 << 27) else None
        G = _f64(G)
        nu = _f64(nu)
        self.check(self.lib.mlcc_cholesky_basis(self.h, n_ao, _ptr(G), _ptr(nu), float(tau), cap,
                                                _ptr(piv), C.byref(nv), _ptr(QiT)))
        n = nv.value
        return piv[:n].copy(), (QiT[: n * n].reshape(n, n).copy() if QiT is not None else None)

    def mo_cholesky(self, n_ao, n_mo, G, piv, QinvT, Cmo, precision="fp64", p_batch=0, out=None):
        """MO Cholesky vectors [n_vec][n_mo][n_mo] by Algorithm 1 (mlcc_mo_cholesky)."""
        piv = np.ascontiguousarray(piv, dtype=np.int32)
        nvec = len(piv)
        if out is None:
            out = np.empty((nvec, n_mo, n_mo))
        G, QinvT, Cmo = _f64(G), _f64(QinvT), _f64(Cmo)
        self.check(self.lib.mlcc_mo_cholesky(self.h, PREC[precision], n_ao, n_mo, _ptr(G), nvec,
                                             _ptr(piv), _ptr(QinvT), _ptr(Cmo), p_batch, _ptr(out)))
        return out

    def profile(self, on=True):
        self.check(self.lib.mlcc_profile_enable(self.h, 1 if on else 0))

    def profile_stats(self):
        buf = (KernelStat * 256)()
        n = self.lib.mlcc_profile_get(self.h, buf, 256)
        if n < 0:
            self.check(n)
        return {buf[i].name.decode(): dict(launches=buf[i].launches, ms=buf[i].ms,
                                           flops=buf[i].flops) for i in range(min(n, 256))}

    def close(self):
        if self.h:
            self.lib.mlcc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """One MLCC problem on a context (see mlcc_problem_create)."""

    def __init__(self, ctx: Context, L, eps, n_occ, n_vir, n_occ_act=None, n_vir_act=None,
                 model="mlcc2", precision="fp64", n_chol=None, seed=None, fock=None,
                 ccsd_space=None, flags=0):
        """L=None with n_chol and seed: Cholesky vectors drawn on the device
        (MLCC_SYNTH_L).  fock: the full [n][n] Fock matrix of a semicanonical
        basis (eps its diagonal), or None for diag(eps).  ccsd_space:
        (n_occ_ccsd, n_vir_ccsd) of model "mlccsd3" (three-level MLCCSD).
        flags: INPUT_ON_DEVICE and/or DETERMINISTIC, added to the descriptor."""
        self.ctx = ctx
        L = _f64(L)
        eps = _f64(eps)
        fock = _f64(fock)
        synth = L is None
        n_chol = n_chol if synth else L.shape[0]
        self._keep = (L, eps, fock)
        d = ProblemDesc(n_occ, n_vir, n_chol,
                        n_occ if n_occ_act is None else n_occ_act,
                        n_vir if n_vir_act is None else n_vir_act,
                        MODEL[model], PREC[precision], _ptr(L), _ptr(eps),
                        (SYNTH_L if synth else 0) | int(flags), int(seed or 0), _ptr(fock),
                        *(ccsd_space or (0, 0)))
        h = C.c_void_p()
        ctx.check(ctx.lib.mlcc_problem_create(ctx.h, C.byref(d), C.byref(h)))
        self._keep = None  # the library copied the inputs
        self.h = h
        dims = (C.c_int64 * 8)()
        ctx.check(ctx.lib.mlcc_problem_dims(h, dims))
        (self.n_occ, self.n_vir, self.n_chol, self.o, self.v, self.M, self.n1,
         self.dim) = list(dims)
        self.model = model

    def close(self):
        if self.h:
            self.ctx.lib.mlcc_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_amplitudes(self, t1, x2=None):
        t1 = _f64(t1)
        x2 = _f64(x2)
        self.ctx.check(self.ctx.lib.mlcc_set_amplitudes(self.h, _ptr(t1), _ptr(x2)))

    def residual(self, doubles=True, x2_out=None):
        """Omega_1, Omega_2, the doubles used and the energy.  doubles=False
        skips Omega_2 and the doubles (host M x M arrays); x2_out (a device
        tensor or host array [M][M]) receives the doubles in place."""
        om1 = np.empty((self.n_vir, self.n_occ))
        om2 = np.empty((self.M, self.M)) if (self.M and doubles) else None
        x2 = x2_out if x2_out is not None else \
            (np.empty((self.M, self.M)) if (self.M and doubles) else None)
        e = C.c_double()
        self.ctx.check(self.ctx.lib.mlcc_residual(self.h, _ptr(om1), _ptr(om2), _ptr(x2),
                                                  C.byref(e)))
        return om1, om2, x2, e.value

    def ground_state(self, tol=1e-10, max_iter=100, diis_dim=8):
        t1 = np.empty((self.n_vir, self.n_occ))
        e = C.c_double()
        info = Info()
        o = opts(tol=tol, max_iter=max_iter, diis_dim=diis_dim)
        st = self.ctx.lib.mlcc_ground_state(self.h, C.byref(o), _ptr(t1), C.byref(e),
                                            C.byref(info))
        self.ctx.check(st, ok=(OK, E_NOCONV))
        return dict(t1=t1, energy=e.value, iterations=info.iterations,
                    converged=bool(info.converged), residual=info.residual, status=st)

    def jacobian_transform(self, c, sigma=None):
        """c: [n_vec][dim] (numpy host or torch device); returns sigma alike."""
        n_vec = c.shape[0] if c.ndim > 1 else 1
        if sigma is None:
            if isinstance(c, np.ndarray):
                sigma = np.empty_like(c, dtype=np.float64)
            else:
                sigma = c.new_empty(c.shape)
        c = _f64(c)
        self.ctx.check(self.ctx.lib.mlcc_jacobian_transform(self.h, n_vec, _ptr(c), _ptr(sigma)))
        return sigma

    def jacobian_transform_eff(self, omega, c1, s1=None):
        n_vec = c1.shape[0] if c1.ndim > 1 else 1
        if s1 is None:
            s1 = np.empty_like(c1, dtype=np.float64) if isinstance(c1, np.ndarray) \
                else c1.new_empty(c1.shape)
        c1 = _f64(c1)
        self.ctx.check(self.ctx.lib.mlcc_jacobian_transform_eff(self.h, float(omega), n_vec,
                                                                _ptr(c1), _ptr(s1)))
        return s1

    def davidson(self, n_roots, tol=1e-8, max_iter=100, max_subspace=0, n_guess=0,
                 effective=False, want_vectors=False):
        w = np.empty(n_roots)
        r1 = np.empty((n_roots, self.n1)) if want_vectors else None
        info = Info()
        o = opts(tol=tol, max_iter=max_iter, max_subspace=max_subspace, n_guess=n_guess,
                 effective=effective)
        st = self.ctx.lib.mlcc_davidson_solve(self.h, n_roots, C.byref(o), _ptr(w), _ptr(r1),
                                              C.byref(info))
        self.ctx.check(st, ok=(OK, E_NOCONV))
        return dict(omega=w, r1=r1, iterations=info.iterations, converged=bool(info.converged),
                    residual=info.residual, transforms=info.transforms,
                    complex_roots=info.complex_roots, status=st)

    def cnto(self, R, omega, n_occ_act, n_vir_act, want_L=True, L_device=False):
        """CNTOs (mlcc_cnto) from excitation vectors R [n_states][n_vir][n_occ]
        and energies omega.  Returns dict(m_eig, n_eig, C, eps, fock, L); L is
        a host array, or a torch tensor on the GPU with L_device=True."""
        R = _f64(np.asarray(R).reshape(len(omega), self.n1))
        w = _f64(np.asarray(omega, dtype=np.float64))
        n = self.n_occ + self.n_vir
        m_eig, n_eig = np.empty(self.n_occ), np.empty(self.n_vir)
        Cm, eps, fock = np.empty((n, n)), np.empty(n), np.empty((n, n))
        L = None
        if want_L:
            if L_device:
                import torch
                L = torch.empty((self.n_chol, n, n), dtype=torch.float64, device="cuda")
            else:
                L = np.empty((self.n_chol, n, n))
        self.ctx.check(self.ctx.lib.mlcc_cnto(self.h, len(w), _ptr(R), _ptr(w), n_occ_act,
                                              n_vir_act, _ptr(m_eig), _ptr(n_eig), _ptr(Cm),
                                              _ptr(eps), _ptr(fock), _ptr(L)))
        return dict(m_eig=m_eig, n_eig=n_eig, C=Cm, eps=eps, fock=fock, L=L)

    def debug_get(self, which):
        sizes = {0: (self.n_occ + self.n_vir,) * 2,
                 1: (self.n_chol, self.n_occ + self.n_vir, self.n_occ + self.n_vir),
                 2: (self.M, self.M), 3: (self.n_vir, self.n_occ), 4: (self.M, self.M)}
        out = np.empty(sizes[which])
        self.ctx.check(self.ctx.lib.mlcc_debug_get(self.h, which, _ptr(out)))
        return out


class Server:
    """Continuous-batching server on a context (mlcc_server_create)."""

    def __init__(self, ctx: Context, max_slots=0, max_queue=0, hbm_budget=0, host_budget=0):
        self.ctx = ctx
        h = C.c_void_p()
        o = ServerOpts(max_slots, max_queue, hbm_budget, host_budget)
        ctx.check(ctx.lib.mlcc_server_create(ctx.h, C.byref(o), C.byref(h)))
        self.h = h
        self._keep = {}

    @staticmethod
    def desc(L, eps, n_occ, n_vir, n_occ_act, n_vir_act, model="mlcc2", precision="fp64",
             n_chol=None, seed=None, fock=None, ccsd_space=None):
        """Problem descriptor; L=None with seed set draws L on the device;
        fock: a full Fock matrix (semicanonical basis) or None; ccsd_space:
        (n_occ_ccsd, n_vir_ccsd) of model "mlccsd3"."""
        eps = _f64(eps)
        fock = _f64(fock)
        if L is None:
            d = ProblemDesc(n_occ, n_vir, n_chol, n_occ_act, n_vir_act, MODEL[model],
                            PREC[precision], None, _ptr(eps), SYNTH_L, seed, _ptr(fock),
                            *(ccsd_space or (0, 0)))
            return d, (eps, fock)
        L = _f64(L)
        d = ProblemDesc(n_occ, n_vir, L.shape[0], n_occ_act, n_vir_act, MODEL[model],
                        PREC[precision], _ptr(L), _ptr(eps), 0, 0, _ptr(fock),
                        *(ccsd_space or (0, 0)))
        return d, (L, eps, fock)

    def submit(self, desc, n_roots, gs_tol=1e-8, es_tol=1e-6, effective=True, max_iter=100):
        gs = opts(tol=gs_tol, max_iter=max_iter)
        es = opts(tol=es_tol, max_iter=max_iter, effective=effective)
        t = C.c_uint64()
        st = self.ctx.lib.mlcc_submit(self.h, C.byref(desc), n_roots, C.byref(gs), C.byref(es),
                                      C.byref(t))
        if st != OK:
            raise MlccError(st, "submit rejected")
        return t.value

    def poll(self, ticket):
        r = Result()
        st = self.ctx.lib.mlcc_poll(self.h, ticket, C.byref(r))
        if st == PENDING:
            return None
        if st != OK:
            raise MlccError(st, "poll failed")
        return dict(status=r.status, omega=list(r.omega[: min(r.n_roots, 16)]), e_corr=r.e_corr,
                    t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done,
                    gs_iterations=r.gs_iterations, es_iterations=r.es_iterations)

    def wait(self, ticket, poll_s=0.001, timeout_s=600.0):
        import time
        t0 = time.time()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.time() - t0 > timeout_s:
                raise TimeoutError(ticket)
            time.sleep(poll_s)

    def close(self):
        if self.h:
            self.ctx.lib.mlcc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(desc, n_roots, effective=True):
    lib = load()
    es = opts(effective=effective)
    return lib.mlcc_request_footprint(C.byref(desc), n_roots, C.byref(es))


def philox4x32_10(ctr, key):
    """Reference Philox4x32-10 (Salmon et al., SC'11) on Python ints, used by
    the tests to pin the device generator of MLCC_SYNTH_L."""
    M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for _ in range(10):
        p0, p1 = M0 * x0, M1 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF, \
            ((p0 >> 32) ^ x3 ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF
        k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
    return x0, x1, x2, x3
