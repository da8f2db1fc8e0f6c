"""Seeded synthetic inputs: MO Cholesky vectors and orbital energies.

This module only draws random numbers in the shapes of the method's inputs; it
holds none of the method's arithmetic.  Both the library's tests/benchmark and
the CPU oracle take their inputs from here.

Recipe (one ``numpy.random.default_rng(seed)`` stream, PCG64):

1. for K = 0..n_chol-1: draw an (n, n) standard-normal block, keep its upper
   triangle and mirror it (``L^K_pq = L^K_qp``), scale by
   ``sigma * exp(-K / 10)``, ``sigma = 0.5 / sqrt(n_occ * n_vir)``;
   the decaying scale mimics the falling pivots of a pivoted Cholesky
   decomposition, sigma keeps the integrals at a physical magnitude;
2. occupied energies ``U[-1.5, -0.3]`` (n_occ draws), sorted ascending;
3. virtual energies ``U[0.1, 3.0]`` (n_vir draws), sorted ascending.

Orbital order is the library's: occupied block first, then virtual; in each
block the active orbitals come first.  The active occupied orbitals are the
``n_occ_act`` highest occupied ones (placed first, ascending), the active
virtual ones are the ``n_vir_act`` lowest virtual ones.  Because the entries of
L are i.i.d., the relabelling does not change their distribution, so L is drawn
directly in that order.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np


@dataclass
class Inputs:
    L: np.ndarray      # (n_chol, n, n) float64 (or float32 if requested)
    eps: np.ndarray    # (n,) float64
    n_occ: int
    n_vir: int
    n_chol: int
    n_occ_act: int
    n_vir_act: int
    seed: int

    @property
    def n(self):
        return self.n_occ + self.n_vir

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.L, dtype=np.float64).tobytes())
        h.update(np.ascontiguousarray(self.eps, dtype=np.float64).tobytes())
        return h.hexdigest()[:16]


def chol_scale(n_occ: int, n_vir: int) -> float:
    return 0.5 / np.sqrt(n_occ * n_vir)


def gen_inputs(n_occ: int, n_vir: int, n_chol: int, n_occ_act: int | None = None,
               n_vir_act: int | None = None, seed: int = 0, dtype=np.float64,
               scale: float | None = None) -> Inputs:
    n_occ_act = n_occ if n_occ_act is None else n_occ_act
    n_vir_act = n_vir if n_vir_act is None else n_vir_act
    n = n_occ + n_vir
    rng = np.random.default_rng(seed)
    sigma = chol_scale(n_occ, n_vir) if scale is None else scale
    L = np.empty((n_chol, n, n), dtype=dtype)
    chunk = max(1, min(n_chol, (1 << 24) // (n * n)))
    for K0 in range(0, n_chol, chunk):
        # drawing a (k, n, n) block consumes the stream exactly like k (n, n) draws
        z = rng.standard_normal((min(chunk, n_chol - K0), n, n))
        up = np.triu(z)
        blk = up + np.triu(z, 1).transpose(0, 2, 1)
        scale = sigma * np.exp(-np.arange(K0, K0 + len(z)) / 10.0)
        L[K0:K0 + len(z)] = scale[:, None, None] * blk
    e_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    e_vir = np.sort(rng.uniform(0.1, 3.0, n_vir))
    e_occ = np.concatenate([e_occ[n_occ - n_occ_act:], e_occ[: n_occ - n_occ_act]])
    eps = np.concatenate([e_occ, e_vir]).astype(np.float64)
    return Inputs(L=L, eps=eps, n_occ=n_occ, n_vir=n_vir, n_chol=n_chol,
                  n_occ_act=n_occ_act, n_vir_act=n_vir_act, seed=seed)


def gen_eps(n_occ: int, n_vir: int, n_occ_act: int | None = None, seed: int = 0) -> np.ndarray:
    """Orbital energies alone (same distributions and ordering as gen_inputs,
    own stream), for requests whose Cholesky vectors are drawn on the device."""
    n_occ_act = n_occ if n_occ_act is None else n_occ_act
    rng = np.random.default_rng(seed)
    e_occ = np.sort(rng.uniform(-1.5, -0.3, n_occ))
    e_vir = np.sort(rng.uniform(0.1, 3.0, n_vir))
    e_occ = np.concatenate([e_occ[n_occ - n_occ_act:], e_occ[: n_occ - n_occ_act]])
    return np.concatenate([e_occ, e_vir]).astype(np.float64)


def serving_stream(n_req: int, seed_sizes: int = 0, seed_arrivals: int = 1, lo: int = 20,
                   hi: int = 80):
    """Sizes of a stream of MLCC2 excitation requests: n_occ uniform in
    [lo, hi], n_vir = 10 n_occ, n_chol = 3 n_vir, active o = round(0.375 n_occ)
    occupied and v = 10 o virtual; request r draws its inputs with seed 1000 + r.
    Also the unit-rate exponential inter-arrival gaps (scaled by 1/rate)."""
    sizes = np.random.default_rng(seed_sizes).integers(lo, hi + 1, size=n_req)
    reqs = []
    for r, no in enumerate(int(x) for x in sizes):
        nv = 10 * no
        o = int(round(0.375 * no))
        reqs.append(dict(n_occ=no, n_vir=nv, n_chol=3 * nv, n_occ_act=o, n_vir_act=10 * o,
                         seed=1000 + r))
    gaps = np.random.default_rng(seed_arrivals).exponential(1.0, size=n_req)
    return reqs, gaps


def gen_vectors(n_vec: int, n_occ: int, n_vir: int, m_doubles: int, seed: int):
    """Random trial vectors (singles (n_vec, V, O) and symmetric doubles
    (n_vec, M, M)) for Jacobian-transform parity and timing."""
    rng = np.random.default_rng(seed)
    c1 = rng.standard_normal((n_vec, n_vir, n_occ))
    c2 = None
    if m_doubles > 0:
        c2 = rng.standard_normal((n_vec, m_doubles, m_doubles)) * 0.1
        c2 = c2 + c2.transpose(0, 2, 1)
    return c1, c2


def gen_amplitudes(n_occ: int, n_vir: int, n_occ_act: int, n_vir_act: int, seed: int,
                   scale1: float = 0.01, scale2: float = 0.01):
    """Random (non-converged) amplitudes for residual/Jacobian parity at an
    arbitrary point: t1 (V, O), doubles full symmetric (v, o, v, o)."""
    rng = np.random.default_rng(seed)
    t1 = scale1 * rng.standard_normal((n_vir, n_occ))
    M = n_occ_act * n_vir_act
    x = scale2 * rng.standard_normal((M, M))
    x = 0.5 * (x + x.T)
    return t1, x.reshape(n_vir_act, n_occ_act, n_vir_act, n_occ_act)


# The workloads, with the sizes used throughout the tests and the benchmark.
CONFIGS = {
    # plain CC2 ground state (full active), FP64
    "cc2_5_20_60": dict(n_occ=5, n_vir=20, n_chol=60, n_occ_act=5, n_vir_act=20),
    # two-electron CCSD (full active) for the exact-diagonalisation pin
    "ccsd_1_8_60": dict(n_occ=1, n_vir=8, n_chol=60, n_occ_act=1, n_vir_act=8),
    # MLCC2 excitation energies, CC2 active 15/150, CCS elsewhere
    "mlcc2_40_400_1200": dict(n_occ=40, n_vir=400, n_chol=1200, n_occ_act=15, n_vir_act=150),
    # MLCCSD (CCS/CCSD) 60/600/2000 with CCSD active 12/120
    "mlccsd_60_600_2000": dict(n_occ=60, n_vir=600, n_chol=2000, n_occ_act=12, n_vir_act=120),
    # three-level MLCCSD (CCS/CC2/CCSD) on the same system: CC2 space 30/300,
    # CCSD space 12/120 inside it
    "mlccsd3_60_600_2000": dict(n_occ=60, n_vir=600, n_chol=2000, n_occ_act=30, n_vir_act=300,
                                n_occ_ccsd=12, n_vir_ccsd=120),
    # large MLCC2 reduced-space run, active 50/500
    "mlcc2_150_1200_3600": dict(n_occ=150, n_vir=1200, n_chol=3600, n_occ_act=50, n_vir_act=500),
}


# ---------------------------------------------------------------------------
# Cholesky vectors drawn on the device (the library's MLCC_SYNTH_L), regenerated
# block by block on the host, so that a workload too large for the host can
# still be checked at sampled elements.  Philox4x32-10 (Salmon, Moraes, Dror,
# Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) with counter
# (min(p,q) n + max(p,q), K, 0, 0) and key (seed lo, seed hi); Box-Muller on
# the first two output words: z = sqrt(-2 ln u1) cos(2 pi u2), u = (w + 1/2)
# 2^-32; L[K][p][q] = (sigma exp(-K/10)) z with sigma = 0.5 / sqrt(n_occ n_vir).
# ---------------------------------------------------------------------------
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_U32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32-10 on arrays of 32-bit counter words (broadcast); returns
    the four output words as uint64 arrays holding 32-bit values."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & _U32 for c in (c0, c1, c2, c3))
    m0, m1 = np.uint64(_PHILOX_M[0]), np.uint64(_PHILOX_M[1])
    ka, kb = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = m0 * x0          # 32 x 32 -> 64 bit, exact in uint64
        p1 = m1 * x2
        x0, x1, x2, x3 = (((p1 >> np.uint64(32)) ^ x1 ^ np.uint64(ka)) & _U32, p1 & _U32,
                          ((p0 >> np.uint64(32)) ^ x3 ^ np.uint64(kb)) & _U32, p0 & _U32)
        ka = (ka + _PHILOX_W[0]) & 0xFFFFFFFF
        kb = (kb + _PHILOX_W[1]) & 0xFFFFFFFF
    return x0, x1, x2, x3


def device_cholesky_block(Ks, rows, cols, n_occ: int, n_vir: int, seed: int) -> np.ndarray:
    """L[K][p][q] for K in Ks, p in rows, q in cols (index arrays), as the
    library's device generator draws them for a problem with n_occ + n_vir
    orbitals and the given seed.  Returns float64 (len(Ks), len(rows), len(cols))."""
    Ks = np.asarray(Ks, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    n = n_occ + n_vir
    sigma = chol_scale(n_occ, n_vir)
    out = np.empty((len(Ks), len(rows), len(cols)))
    lo = np.minimum(rows[:, None], cols[None, :])
    hi = np.maximum(rows[:, None], cols[None, :])
    pq = (lo * n + hi).astype(np.uint64)
    step = max(1, (1 << 22) // max(1, pq.size))
    for k0 in range(0, len(Ks), step):
        kk = Ks[k0:k0 + step]
        x, y, _, _ = philox4x32_10(pq[None, :, :], kk[:, None, None].astype(np.uint64), 0, 0,
                                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
        u1 = (x.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)
        u2 = (y.astype(np.float64) + 0.5) * (1.0 / 4294967296.0)
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
        out[k0:k0 + len(kk)] = (sigma * np.exp(-kk.astype(np.float64) / 10.0))[:, None, None] * z
    return out


# ---------------------------------------------------------------------------
# AO-basis inputs of the MO Cholesky-vector construction (two-step Cholesky
# decomposition: pivots first, then the vectors through the RI-like expression)
# ---------------------------------------------------------------------------
def pair_index(n_ao: int):
    """Packed pair index of alpha >= beta: (alpha, beta) arrays of length
    n_ao (n_ao + 1) / 2, in the order alpha * (alpha + 1) / 2 + beta."""
    a, b = np.tril_indices(n_ao)
    return a, b


def gen_ao_eri(n_ao: int, n_aux: int, seed: int, decay: float = 0.15):
    """Synthetic AO electron-repulsion integrals g_(ab)(cd) as a positive
    semidefinite matrix over packed pairs a >= b: g = sum_P B^P_ab B^P_cd with
    B^P symmetric, i.i.d. normal entries scaled by exp(-decay P) (a decaying
    spectrum, as the pivots of a Cholesky decomposition fall), plus the
    pair-diagonal weight exp(-|a - b| / 4) that makes distant pairs small, as
    for localized AOs.  Returns (G [npair][npair], Bfull [n_aux][n_ao][n_ao])."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n_aux, n_ao, n_ao))
    B = np.triu(z) + np.triu(z, 1).transpose(0, 2, 1)
    idx = np.arange(n_ao)
    loc = np.exp(-np.abs(idx[:, None] - idx[None, :]) / 4.0)
    B = B * loc[None] * np.exp(-decay * np.arange(n_aux))[:, None, None] / np.sqrt(n_ao)
    a, b = pair_index(n_ao)
    Bp = B[:, a, b]                       # [P][pair]
    return Bp.T @ Bp, B


def gen_mo_coefficients(n_ao: int, n_mo: int, seed: int):
    """Orthonormal MO coefficients C [n_ao][n_mo] (a random orthogonal matrix's
    first n_mo columns) whose orbitals are localized on a band of AOs."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n_ao, n_mo))
    idx = np.arange(n_ao)[:, None]
    centers = np.linspace(0, n_ao - 1, n_mo)[None, :]
    X = X * np.exp(-np.abs(idx - centers) / (0.25 * n_ao))
    Q, _ = np.linalg.qr(X)
    return Q
