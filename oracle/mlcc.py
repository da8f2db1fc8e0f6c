"""Plain FP64 oracle for MLCC2 and MLCCSD (CCS/CCSD) on Cholesky vectors.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Conventions (shared with the library's C ABI, restated here so the oracle stands
on its own):

* Orbitals: ``n = O + V``; occupied first, each block active-first.  Active
  occupied are ``0..o-1``, active virtual are ``O..O+v-1``.
* ``L[K, p, q]`` are the MO Cholesky vectors, symmetric in ``p, q``, so that
  ``g_pqrs = sum_K L[K,p,q] L[K,r,s]`` (Appendix A, first equation).
* ``eps[p]``: the MO Fock matrix is ``diag(eps)`` (canonical Hartree-Fock).
* ``t1[A, I]``: singles over all virtual ``A`` and occupied ``I``.
* Doubles are full symmetric arrays ``x[a, i, b, j] = x[b, j, a, i]`` over the
  active space, with ``X2 = 1/2 sum x_aibj E_ai E_bj`` and the biorthonormal
  projection ``<mu_aibj| E_ck E_dl |HF> = d(ai,ck) d(bj,dl) + d(ai,dl) d(bj,ck)``.
  Flattened, ``x.reshape(v*o, v*o)`` has pair index ``a*o + i``.

The paper prints the Fock matrix in the X1 basis without its one-electron part
(Appendix A, "ground state equations" subsection).  Here the one-electron part
is ``h = F - G(D_HF)`` with ``F = diag(eps)``, so ``F~ = h~ + G~`` reduces to
``diag(eps)`` at ``t1 = 0``.

Every function below uses only analytic operations (no abs/conj/real) on its
amplitude arguments, so that the Jacobian can be taken by complex step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_ES = dict(optimize=True)


def _einsum(spec, *ops):
    """numpy.einsum of the given expression, evaluated as a sequence of
    pairwise products along numpy's optimal contraction path, each product by
    torch.einsum on the CPU (batched BLAS) when torch is available.  Same
    arithmetic as the expression up to rounding order; numpy's own fallback
    for pairwise products that do not map onto BLAS is a single-threaded loop
    that makes the larger parity cases impractical."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        return np.einsum(spec, *ops, **_ES)
    lhs, out = spec.replace(" ", "").split("->")
    subs = lhs.split(",")
    path = np.einsum_path(spec, *ops, optimize="optimal")[0][1:]
    dt = np.result_type(*ops)
    terms = [(sb, torch.from_numpy(np.ascontiguousarray(op, dtype=dt))) for sb, op in zip(subs, ops)]
    for pair in path:
        pair = sorted(pair, reverse=True)
        picked = [terms.pop(i) for i in pair]
        rest = "".join(sb for sb, _ in terms) + out
        idx = "".join(dict.fromkeys("".join(sb for sb, _ in picked)))
        keep = "".join(c for c in idx if c in rest)
        res = torch.einsum(",".join(sb for sb, _ in picked) + "->" + keep, *[t for _, t in picked])
        terms.append((keep, res))
    (sb, t), = terms
    return torch.einsum(sb + "->" + out, t).numpy()


@dataclass(frozen=True)
class Dims:
    O: int  # all occupied
    V: int  # all virtual
    o: int  # active occupied (prefix of the occupied block)
    v: int  # active virtual (prefix of the virtual block)

    @property
    def n(self):
        return self.O + self.V

    @property
    def M(self):
        return self.o * self.v

    # index slices into the MO dimension
    @property
    def occ(self):
        return slice(0, self.O)

    @property
    def vir(self):
        return slice(self.O, self.O + self.V)

    @property
    def aocc(self):
        return slice(0, self.o)

    @property
    def avir(self):
        return slice(self.O, self.O + self.v)


# --------------------------------------------------------------------------
# Integrals, reference, X1 transformation (Sec. 2.1; Appendix A)
# --------------------------------------------------------------------------

def eri(L):
    """Full 4-index integrals g_pqrs = sum_K L^K_pq L^K_rs (Appendix A, eq. for
    the Cholesky decomposition).  Small systems only."""
    return np.einsum("Kpq,Krs->pqrs", L, L)


def two_electron_fock(L, d: Dims):
    """G_pq = sum_I (2 g_pqII - g_pIIq), the closed-shell Coulomb minus exchange
    of the Hartree-Fock density, written with the Cholesky vectors (the two-
    electron part of the Fock expression in Appendix A)."""
    occ = d.occ
    dK = np.einsum("Kii->K", L[:, occ, occ])
    coul = _einsum("Kpq,K->pq", L, dK)
    exch = _einsum("Kpi,Kiq->pq", L[:, :, occ], L[:, occ, :])
    return 2.0 * coul - exch


def core_hamiltonian(L, eps, d: Dims, fock=None):
    """One-electron integrals h implied by the reference: F = h + G(D_HF), so
    h = F - G with F = diag(eps) (canonical) or a given Fock matrix (e.g. the
    semicanonical basis of Sec. 2.2, whose active-inactive blocks couple)."""
    F = np.diag(eps).astype(L.dtype) if fock is None else np.asarray(fock, dtype=L.dtype)
    return F - two_electron_fock(L, d)


def hf_energy(L, eps, d: Dims):
    """E_HF = sum_I (h_II + F_II)."""
    h = core_hamiltonian(L, eps, d)
    return float(np.trace(h[d.occ, d.occ]) + np.sum(eps[: d.O]))


def t1_matrix(t1, d: Dims):
    """n x n matrix T with T[A, I] = t_AI (virtual row, occupied column)."""
    T = np.zeros((d.n, d.n), dtype=np.result_type(t1, float))
    T[d.vir, d.occ] = t1
    return T


def x1_transform(X, t1, d: Dims):
    """X1 (T1) similarity transformation of one-index-pair quantities.

    exp(-T1) a+_p exp(T1) = a+_p - sum_A t_Ap a+_A  and
    exp(-T1) a_q  exp(T1) = a_q  + sum_I t_qI a_I,  so an operator
    sum_pq X_pq a+_p a_q becomes sum_pq [(1 - T) X (1 + T)]_pq a+_p a_q.
    Works on a matrix (n, n) or a stack of Cholesky vectors (K, n, n)."""
    T = t1_matrix(t1, d)
    one = np.eye(d.n)
    return (one - T) @ X @ (one + T)


def fock_x1(Lt, ht, d: Dims):
    """F~_PQ = h~_PQ + sum_I (2 g~_PQII - g~_PIIQ) in Cholesky form."""
    return ht + two_electron_fock(Lt, d)


def orbital_denominators(eps, d: Dims):
    """eps_aibj = e_a + e_b - e_i - e_j over the active space, shape (v,o,v,o)."""
    ea = eps[d.avir]
    ei = eps[d.aocc]
    dai = ea[:, None] - ei[None, :]
    return dai[:, :, None, None] + dai[None, None, :, :]


def singles_denominators(eps, d: Dims):
    """e_A - e_I, shape (V, O)."""
    return eps[d.vir][:, None] - eps[d.occ][None, :]


def exch_occ(x):
    """x[a,i,b,j] -> x[a,j,b,i] (exchange of the two occupied indices)."""
    return x.transpose(0, 3, 2, 1)


def u_of(x):
    """u_aibj = 2 x_aibj - x_ajbi."""
    return 2.0 * x - exch_occ(x)


@dataclass
class Dressed:
    Lt: np.ndarray  # X1-transformed Cholesky vectors (K, n, n)
    Ft: np.ndarray  # Fock matrix in the X1 basis (n, n)


def dress(L, eps, d: Dims, t1, h=None):
    """X1-transformed Cholesky vectors and Fock matrix."""
    if h is None:
        h = core_hamiltonian(L, eps, d)
    Lt = x1_transform(L, t1, d)
    ht = x1_transform(h, t1, d)
    return Dressed(Lt=Lt, Ft=fock_x1(Lt, ht, d))


# --------------------------------------------------------------------------
# Residuals (Sec. 2.1 eqs. mlcc2_1/2 and mlccsd_1/2; Appendix A.1)
# --------------------------------------------------------------------------

def g_aibj(Lt, d: Dims):
    """g~_aibj = sum_K L~^K_ai L~^K_bj over the active space (v,o,v,o)."""
    Lai = Lt[:, d.avir, d.aocc]
    return _einsum("Kai,Kbj->aibj", Lai, Lai)


def omega_singles(D: Dressed, d: Dims, x2):
    """Singles residual with active doubles x2 (s for MLCC2, t for MLCCSD),
    Appendix A, codable MLCC2 Omega vector:

      Omega_AI = F~_AI + [I act] sum_bcjK u_bicj L~^K_jc L~^K_Ab
                       - [A act] sum_jkbK u_ajbk L~^K_kb L~^K_jI
                       + [A,I act] sum_jb u_aibj F~_jb
    """
    Lt, Ft = D.Lt, D.Ft
    om = Ft[d.vir, d.occ].copy()
    if d.o == 0 or d.v == 0 or x2 is None:
        return om
    u = u_of(x2)
    Ljc = Lt[:, d.aocc, d.avir]                          # L~_jc = L_jc (ov block)
    om[:, : d.o] += _einsum("bicj,Kjc,KAb->Ai", u, Ljc, Lt[:, d.vir, d.avir])
    om[: d.v, :] -= _einsum("ajbk,Kkb,KjI->aI", u, Ljc, Lt[:, d.aocc, d.occ])
    om[: d.v, : d.o] += _einsum("aibj,jb->ai", u, Ft[d.aocc, d.avir])
    return om


def mlcc2_s_analytic(D: Dressed, eps, d: Dims):
    """Analytic solution of the MLCC2 doubles equation in the semicanonical
    basis: s_aibj = -g~_aibj / eps_aibj (untransformed Fock diagonal)."""
    return -g_aibj(D.Lt, d) / orbital_denominators(eps, d)


def mlcc2_omega(L, eps, d: Dims, t1, s, h=None):
    """MLCC2 residual as a function of independent (t1, s):
      Omega_1 from omega_singles,
      Omega_2 = <mu2| H~ + [F, S2] |HF> = g~_aibj + eps_aibj s_aibj."""
    D = dress(L, eps, d, t1, h)
    om1 = omega_singles(D, d, s)
    om2 = None
    if d.M > 0:
        om2 = g_aibj(D.Lt, d) + orbital_denominators(eps, d) * s
    return om1, om2


def _blk(Lt, d, p, q):
    """Active blocks of L~: p, q in {'o','v'}."""
    sl = {"o": d.aocc, "v": d.avir}
    return Lt[:, sl[p], sl[q]]


def ccsd_doubles(D: Dressed, d: Dims, t2):
    """Closed-shell CCSD doubles residual with X1-dressed integrals, all
    explicit indices active (Appendix A, MLCCSD Omega vector; written from the
    standard spin-adapted closed-shell derivation, with every integral dressed).

      Omega = A2 + B2 + P(C2 + D2 + E2),  P X_aibj = X_aibj + X_bjai
    """
    Lt, Ft = D.Lt, D.Ft
    Lvo, Lov = _blk(Lt, d, "v", "o"), _blk(Lt, d, "o", "v")
    Loo, Lvv = _blk(Lt, d, "o", "o"), _blk(Lt, d, "v", "v")
    E = _einsum

    g_vovo = E("Kai,Kbj->aibj", Lvo, Lvo)   # g~_aibj
    g_oooo = E("Kki,Klj->kilj", Loo, Loo)   # g~_kilj
    g_ovov = E("Kkc,Kld->kcld", Lov, Lov)   # g~_kcld
    g_oovv = E("Kki,Kac->kiac", Loo, Lvv)   # g~_kiac
    g_voov = E("Kai,Kkc->aikc", Lvo, Lov)   # g~_aikc
    Fvv = Ft[d.avir, d.avir]
    Foo = Ft[d.aocc, d.aocc]

    t = t2
    u = u_of(t)
    L_ovov = 2.0 * g_ovov - g_ovov.transpose(0, 3, 2, 1)   # L~_kcld = 2g~_kcld - g~_kdlc
    L_voov = 2.0 * g_voov - E("Kac,Kki->aikc", Lvv, Loo)   # L~_aikc = 2g~_aikc - g~_acki

    # A2: g~_aibj + sum_cd t_cidj g~_acbd  (ladder)
    A2 = g_vovo + E("cidj,Kac,Kbd->aibj", t, Lvv, Lvv)
    # B2: sum_kl t_akbl (g~_kilj + sum_cd t_cidj g~_kcld)
    B2 = E("akbl,kilj->aibj", t, g_oooo + E("cidj,kcld->kilj", t, g_ovov))
    # C2: -1/2 sum_ck t_bkcj Y_aick - sum_ck t_bkci Y_ajck,
    #     Y_aick = g~_kiac - 1/2 sum_dl t_aldi g~_kdlc
    Y = g_oovv.transpose(2, 1, 3, 0) - 0.5 * E("aldi,kdlc->aick", t, g_ovov)
    C2 = -0.5 * E("bkcj,aick->aibj", t, Y) - E("bkci,ajck->aibj", t, Y)
    # D2: 1/2 sum_ck u_bjck (L~_aikc + 1/2 sum_dl u_aidl L~_ldkc)
    Z = L_voov + 0.5 * E("aidl,ldkc->aikc", u, L_ovov)
    D2 = 0.5 * E("bjck,aikc->aibj", u, Z)
    # E2: sum_c t_aicj (F~_bc - sum_dkl u_bkdl g~_ldkc)
    #     - sum_k t_aibk (F~_kj + sum_cdl u_cldj g~_kdlc)
    Wvv = Fvv - E("bkdl,ldkc->bc", u, g_ovov)
    Woo = Foo + E("cldj,kdlc->kj", u, g_ovov)
    E2 = E("aicj,bc->aibj", t, Wvv) - E("aibk,kj->aibj", t, Woo)

    R = C2 + D2 + E2
    return A2 + B2 + R + R.transpose(2, 3, 0, 1)


def mlccsd_omega(L, eps, d: Dims, t1, t2, h=None):
    """MLCCSD (CCS/CCSD) residual: singles as MLCC2 with t in place of s,
    doubles = active-space CCSD doubles with dressed integrals."""
    D = dress(L, eps, d, t1, h)
    om1 = omega_singles(D, d, t2)
    om2 = ccsd_doubles(D, d, t2) if d.M > 0 else None
    return om1, om2


def ccsd_space_mask(d: Dims, o_t, v_t):
    """True at the doubles (a, i, b, j) whose four indices all lie in the
    CCSD space: the first v_t active virtuals and the first o_t active
    occupied orbitals (nested prefixes of the CC2 space)."""
    pair = (np.arange(d.v)[:, None] < v_t) & (np.arange(d.o)[None, :] < o_t)
    return pair[:, :, None, None] & pair[None, None, :, :]


def mlccsd3_omega(L, eps, d: Dims, o_t, v_t, t1, x2, h=None):
    """Three-level MLCCSD (CCS/CC2/CCSD) residual, Sec. 2.1 (X = X1 + S2 + T2,
    S2 in the larger active space and perturbative, T2 in the smaller one and
    a correction to S2).  The paper prints no equations for this model; the
    reading used here:

    * x2 holds the doubles over the CC2 space (d.o, d.v): S2 + T2, where T2
      lives only on the CCSD space;
    * singles and the doubles projections inside the CCSD space are those of
      the full similarity transform exp(-X) H exp(X) (CCSD level, including
      every coupling to the S2 amplitudes outside it);
    * the remaining doubles projections of the CC2 space keep the CC2 form
      <mu2| H~ + [F, X2] |HF> = g~_aibj + eps_aibj x_aibj.

    Inside the CCSD space the model reaches CCSD, outside it MLCC2; with an
    empty CCSD space it is MLCC2, and with the CCSD space equal to the CC2
    space it is MLCCSD (CCS/CCSD)."""
    D = dress(L, eps, d, t1, h)
    om1 = omega_singles(D, d, x2)
    if d.M == 0:
        return om1, None
    om2 = g_aibj(D.Lt, d) + orbital_denominators(eps, d) * x2
    inner = ccsd_space_mask(d, o_t, v_t)
    if inner.any():
        om2 = np.where(inner, ccsd_doubles(D, d, x2), om2)
    return om1, om2


def ccs_omega(L, eps, d: Dims, t1, h=None):
    D = dress(L, eps, d, t1, h)
    return D.Ft[d.vir, d.occ].copy()


# --------------------------------------------------------------------------
# Energy (Appendix A, correlation energy)
# --------------------------------------------------------------------------

def correlation_energy(L, d: Dims, t1, x2):
    """E = sum t_AI t_BJ L_IAJB + sum_act x_aibj L_iajb,  L_pqrs = 2g_pqrs - g_psrq,
    with untransformed integrals."""
    Lov = L[:, d.occ, d.vir]  # L^K_IA
    e = 2.0 * _einsum("AI,BJ,KIA,KJB->", t1, t1, Lov, Lov) \
        - _einsum("AI,BJ,KIB,KJA->", t1, t1, Lov, Lov)
    if x2 is not None and d.M > 0:
        Lia = L[:, d.aocc, d.avir]
        e = e + 2.0 * _einsum("aibj,Kia,Kjb->", x2, Lia, Lia) \
            - _einsum("aibj,Kib,Kja->", x2, Lia, Lia)
    return e


def mp2_energy(L, eps, d: Dims):
    """Closed-form MP2 over the active space:
    E = -sum g_aibj (2 g_aibj - g_ajbi) / eps_aibj."""
    g = g_aibj(L, d)
    return float(-np.sum(g * (2.0 * g - exch_occ(g)) / orbital_denominators(eps, d)))


# --------------------------------------------------------------------------
# Ground state: DIIS-accelerated quasi-Newton (Sec. 2.1)
# --------------------------------------------------------------------------

MODELS = ("ccs", "mlcc2", "mlccsd", "mlccsd3")


class Problem:
    """Inputs plus the model; caches h.  fock: the full Fock matrix when the
    basis is semicanonical rather than canonical (eps is then its diagonal,
    which the denominators use).  mlccsd3: d's active space is the CC2 space
    and ccsd_space = (o_t, v_t) the CCSD space inside it."""

    def __init__(self, L, eps, d: Dims, model: str, fock=None, ccsd_space=None):
        assert model in MODELS
        self.L = np.asarray(L, dtype=np.float64)
        self.eps = np.asarray(eps, dtype=np.float64)
        self.d = d
        self.model = model
        if model == "ccs":
            self.d = Dims(d.O, d.V, 0, 0)
        if model == "mlccsd3":
            o_t, v_t = ccsd_space
            assert 0 <= o_t <= d.o and 0 <= v_t <= d.v
            self.ccsd_space = (o_t, v_t)
        self.h = core_hamiltonian(self.L, self.eps, self.d, fock=fock)

    @property
    def iterated_doubles(self):
        """Doubles solved by the quasi-Newton/DIIS iteration (MLCCSD models);
        MLCC2 solves them analytically instead."""
        return self.model in ("mlccsd", "mlccsd3")

    # residual in the independent variables (t1, x2)
    def omega(self, t1, x2):
        d = self.d
        if self.model == "ccs" or d.M == 0:
            D = dress(self.L, self.eps, d, t1, self.h)
            return D.Ft[d.vir, d.occ].copy(), None
        if self.model == "mlcc2":
            return mlcc2_omega(self.L, self.eps, d, t1, x2, self.h)
        if self.model == "mlccsd3":
            return mlccsd3_omega(self.L, self.eps, d, *self.ccsd_space, t1, x2, self.h)
        return mlccsd_omega(self.L, self.eps, d, t1, x2, self.h)

    def s_analytic(self, t1):
        D = dress(self.L, self.eps, self.d, t1, self.h)
        return mlcc2_s_analytic(D, self.eps, self.d)

    def energy(self, t1, x2):
        return correlation_energy(self.L, self.d, t1, x2)


def _diis_extrapolate(xs, es):
    m = len(xs)
    B = np.empty((m + 1, m + 1))
    B[:m, :m] = np.array([[np.dot(a, b) for b in es] for a in es])
    B[m, :m] = B[:m, m] = -1.0
    B[m, m] = 0.0
    rhs = np.zeros(m + 1)
    rhs[m] = -1.0
    c = np.linalg.solve(B, rhs)[:m]
    return sum(ci * xi for ci, xi in zip(c, xs))


def ground_state(P: Problem, tol=1e-10, max_iter=200, diis_dim=8, t1_guess=None):
    """Solve Omega = 0.  MLCC2: s is re-solved analytically each iteration and
    DIIS acts on t1; MLCCSD: DIIS on (t1, t2).  Quasi-Newton step
    dx = -Omega / (eps_A - eps_I)  (and / eps_aibj for t2).  Three-level
    MLCCSD iterates all its doubles the same way: on the CC2-level entries
    the step lands on the analytic -g~/eps at once.

    Returns dict(t1, x2, energy, iterations, converged, history)."""
    d = P.d
    dai = singles_denominators(P.eps, d)
    daibj = orbital_denominators(P.eps, d) if d.M > 0 else None
    t1 = np.zeros((d.V, d.O)) if t1_guess is None else np.array(t1_guess, float)
    t2 = np.zeros((d.v, d.o, d.v, d.o)) if (P.iterated_doubles and d.M > 0) else None
    xs, es, hist = [], [], []
    converged = False
    E = None
    for it in range(1, max_iter + 1):
        if P.model == "mlcc2" and d.M > 0:
            x2 = P.s_analytic(t1)
        else:
            x2 = t2
        om1, om2 = P.omega(t1, x2)
        E = P.energy(t1, x2)
        res = np.linalg.norm(om1) if om2 is None or P.model == "mlcc2" \
            else np.sqrt(np.linalg.norm(om1) ** 2 + np.linalg.norm(om2) ** 2)
        hist.append((E, res))
        if res < tol:
            converged = True
            break
        t1n = t1 - om1 / dai
        if P.iterated_doubles and om2 is not None:
            t2n = t2 - om2 / daibj
            vec = np.concatenate([t1n.ravel(), t2n.ravel()])
            err = np.concatenate([om1.ravel(), om2.ravel()])
        else:
            vec, err = t1n.ravel(), om1.ravel()
        xs.append(vec)
        es.append(err)
        if len(xs) > diis_dim:
            xs.pop(0)
            es.pop(0)
        vec = _diis_extrapolate(xs, es)
        t1 = vec[: d.V * d.O].reshape(d.V, d.O)
        if P.iterated_doubles and om2 is not None:
            t2 = vec[d.V * d.O:].reshape(d.v, d.o, d.v, d.o)
    x2 = P.s_analytic(t1) if (P.model == "mlcc2" and d.M > 0) else t2
    return dict(t1=t1, x2=x2, energy=E, iterations=it, converged=converged,
                history=hist)


# --------------------------------------------------------------------------
# Jacobian transformation (Sec. 2.1 Jacobians; Appendix A.2)
# --------------------------------------------------------------------------

def jacobian_transform(P: Problem, t1, x2, c1, c2, h=1e-30):
    """sigma = A c with A = dOmega/dx at (t1, x2), by complex-step
    differentiation (exact to rounding: every operation is analytic).

    For MLCC2 the variables are (t1, s) with s independent, so that the
    doubles-doubles block is eps_aibj * delta (F untransformed)."""
    t1c = t1 + 1j * h * c1
    x2c = None
    if x2 is not None:
        x2c = x2 + 1j * h * (c2 if c2 is not None else 0.0)
    om1, om2 = P.omega(t1c, x2c)
    s1 = om1.imag / h
    s2 = None if om2 is None else om2.imag / h
    return s1, s2


def jacobian_transform_fd(P: Problem, t1, x2, c1, c2, h=1e-5):
    """Central finite differences of the residual (cross-check only)."""
    xp2 = None if x2 is None else x2 + h * c2
    xm2 = None if x2 is None else x2 - h * c2
    p1, p2 = P.omega(t1 + h * c1, xp2)
    m1, m2 = P.omega(t1 - h * c1, xm2)
    s2 = None if p2 is None else (p2 - m2) / (2 * h)
    return (p1 - m1) / (2 * h), s2


# packed <-> full doubles coordinates (unique pairs ai >= bj)

def packed_index(M):
    r, c = np.tril_indices(M)
    return r, c


def full_from_packed(xp, d: Dims):
    M = d.M
    r, c = packed_index(M)
    X = np.zeros((M, M), dtype=xp.dtype)
    X[r, c] = xp
    X[c, r] = xp
    return X.reshape(d.v, d.o, d.v, d.o)


def packed_from_full(x, d: Dims):
    r, c = packed_index(d.M)
    return x.reshape(d.M, d.M)[r, c]


def has_doubles(P: Problem):
    return P.model != "ccs" and P.d.M > 0


def jacobian_dense(P: Problem, t1, x2):
    """Dense Jacobian in (singles, packed doubles) coordinates, column by
    column from jacobian_transform.  Small systems only."""
    d = P.d
    n1 = d.V * d.O
    n2 = d.M * (d.M + 1) // 2 if has_doubles(P) else 0
    A = np.zeros((n1 + n2, n1 + n2))
    for col in range(n1 + n2):
        e = np.zeros(n1 + n2)
        e[col] = 1.0
        c1 = e[:n1].reshape(d.V, d.O)
        c2 = full_from_packed(e[n1:], d) if n2 else None
        s1, s2 = jacobian_transform(P, t1, x2, c1, c2)
        A[:n1, col] = s1.ravel()
        if n2:
            A[n1:, col] = packed_from_full(s2, d)
    return A


def dense_eigenvalues(A, n_roots=None):
    w = np.linalg.eigvals(A)
    w = w[np.argsort(w.real)]
    return w if n_roots is None else w[:n_roots]


def cis_matrix(L, eps, d: Dims):
    """Closed-shell singlet CIS matrix: (e_A - e_I) d + 2 g_AIJB - g_ABJI,
    rows (A,I), columns (B,J)."""
    Lvo = L[:, d.vir, d.occ]
    Lvv = L[:, d.vir, d.vir]
    Loo = L[:, d.occ, d.occ]
    A = 2.0 * np.einsum("KAI,KBJ->AIBJ", Lvo, Lvo) - np.einsum("KAB,KJI->AIBJ", Lvv, Loo)
    n1 = d.V * d.O
    A = A.reshape(n1, n1) + np.diag(singles_denominators(eps, d).ravel())
    return A


# --------------------------------------------------------------------------
# Full-space nonsymmetric Davidson (eigenvalues of A; Sec. 2.1)
# --------------------------------------------------------------------------

def _diag_precond(P: Problem):
    d = P.d
    D1 = singles_denominators(P.eps, d).ravel()
    if not has_doubles(P):
        return D1
    return np.concatenate([D1, orbital_denominators(P.eps, d).ravel()])


def davidson(P: Problem, t1, x2, n_roots, tol=1e-8, max_iter=100, n_guess=None,
             max_space=None):
    """Lowest n_roots eigenvalues of the Jacobian.  Vectors are stored as
    (singles, full symmetric doubles) and the Euclidean metric of that storage
    is used throughout.  Guesses: unit singles at the lowest e_A - e_I.

    The doubles amplitudes live in the subspace symmetric under (ai) <-> (bj);
    transformed vectors and new directions are projected onto it, so that the
    rounding-level asymmetry of the complex-step transform cannot excite the
    (unphysical) antisymmetric part of the operator."""
    d = P.d
    n1 = d.V * d.O
    full2 = has_doubles(P)
    dim = n1 + (d.M * d.M if full2 else 0)
    Dg = _diag_precond(P)
    n_guess = n_guess or (n_roots + 2)
    max_space = max_space or max(20 * n_roots, n_guess + 2 * n_roots)

    def sym(x):
        if not full2:
            return x
        y = x.copy()
        D2 = y[n1:].reshape(d.M, d.M)
        y[n1:] = (0.5 * (D2 + D2.T)).ravel()
        return y

    def apply(x):
        c1 = x[:n1].reshape(d.V, d.O)
        c2 = x[n1:].reshape(d.v, d.o, d.v, d.o) if full2 else None
        s1, s2 = jacobian_transform(P, t1, x2, c1, c2)
        return sym(np.concatenate([s1.ravel(), s2.ravel()]) if full2 else s1.ravel())

    order = np.lexsort((np.arange(n1) % d.O, np.arange(n1) // d.O, Dg[:n1]))
    V = np.zeros((0, dim))
    AV = np.zeros((0, dim))
    new = []
    for k in range(n_guess):
        e = np.zeros(dim)
        e[order[k]] = 1.0
        new.append(e)
    omega = None
    for it in range(1, max_iter + 1):
        for w in new:
            w = sym(w)
            n0 = np.linalg.norm(w)
            for _ in range(2):
                w = w - V.T @ (V @ w)
            nw = np.linalg.norm(w)
            if nw < 1e-10 or nw < 1e-8 * n0:
                continue
            w = w / nw
            V = np.vstack([V, w])
            AV = np.vstack([AV, apply(w)])
        R = V @ AV.T  # R[i, j] = v_i . (A v_j)
        w_, Y = np.linalg.eig(R)
        idx = np.argsort(w_.real)[:n_roots]
        omega = w_[idx]
        Y = Y[:, idx].real
        res_norms = []
        new = []
        for k in range(n_roots):
            y = Y[:, k] / np.linalg.norm(V.T @ Y[:, k])
            x = V.T @ y
            r = AV.T @ y - omega[k].real * x
            rn = np.linalg.norm(r)
            res_norms.append(rn)
            if rn > tol:
                den = omega[k].real - Dg
                den = np.where(np.abs(den) < 1e-8, 1e-8, den)
                new.append(r / den)
        if not new:
            return dict(omega=omega.real, converged=True, iterations=it,
                        residuals=res_norms, complex=bool(np.any(omega.imag != 0)))
        if len(V) + len(new) > max_space:
            # collapse onto the current Ritz vectors (no re-transformation)
            X = V.T @ Y
            AX = AV.T @ Y
            Q, Rq = np.linalg.qr(X)
            Ri = np.linalg.inv(Rq)
            V = (Q).T.copy()
            AV = (AX @ Ri).T.copy()
    return dict(omega=omega.real, converged=False, iterations=max_iter,
                residuals=res_norms, complex=bool(np.any(omega.imag != 0)))
