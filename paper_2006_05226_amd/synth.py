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
    # large MLCC2 reduced-space run, active 50/500
    "mlcc2_150_1200_3600": dict(n_occ=150, n_vir=1200, n_chol=3600, n_occ_act=50, n_vir_act=500),
}
