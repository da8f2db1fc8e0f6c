"""Two-step Cholesky decomposition of the AO electron-repulsion integrals and
the MO Cholesky vectors built from it (Sec. 2.4: the RI-like expression for
the vectors, the MO-screened diagonal eq. cd_screening with the weights of
eq. mo_screening, and Algorithm 1) -- plain FP64 oracle.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Integrals are a matrix G over packed AO pairs ab (a >= b, the order of
synth.pair_index): G[ab][cd] = (ab|cd).  Pinned by tests/test_oracle_cholesky.py.
"""
from __future__ import annotations

import numpy as np


def screening_weights(Ca):
    """nu_a = max_p (C^a_ap)^2 over the active MOs (eq. mo_screening)."""
    return (np.asarray(Ca) ** 2).max(axis=1)


def pivot_basis(G, tau, nu=None, pairs=None, max_vectors=None):
    """First step: the Cholesky basis by pivoted (incomplete) Cholesky
    decomposition of G.  The updated diagonal D_ab = g_abab - sum_J (L^J_ab)^2
    is screened to D~_ab = nu_a D_ab nu_b (eq. cd_screening; nu = None: no
    screening); the pair with the largest D~ is the next pivot, and the
    decomposition stops when max D~ < tau.  pairs = (a, b) index arrays of
    the packed pair order.  Returns the pivots in selection order and the
    vectors L [npair][n_J] of the decomposition."""
    G = np.asarray(G, dtype=np.float64)
    npair = G.shape[0]
    w = np.ones(npair) if nu is None else nu[pairs[0]] * nu[pairs[1]]
    D = np.diag(G).copy()
    cap = npair if max_vectors is None else max_vectors
    piv, cols = [], []
    while len(piv) < cap:
        Dt = w * D
        K = int(np.argmax(Dt))
        if not Dt[K] >= tau:
            break
        col = G[:, K].copy()
        for J, l in enumerate(cols):
            col -= l * l[K]
        l = col / np.sqrt(D[K])
        D = D - l * l
        piv.append(K)
        cols.append(l)
    L = np.stack(cols, axis=1) if cols else np.zeros((npair, 0))
    return np.array(piv, dtype=np.int64), L


def inverse_factor_t(G, piv):
    """Q^-T with S_KL = (K|L) over the basis (in pivot order) and S = Q Q^T,
    Q lower triangular (the Cholesky factor)."""
    S = np.asarray(G)[np.ix_(piv, piv)]
    Q = np.linalg.cholesky(S)
    return np.linalg.inv(Q).T


def ri_vectors(G, piv, QinvT):
    """Second step in the AO basis: L^J_ab = sum_K (ab|K) [Q^-T]_KJ."""
    return np.asarray(G)[:, piv] @ QinvT


def unpack(pairvec, pairs, n_ao):
    """Columns over packed pairs -> symmetric (.., n_ao, n_ao) matrices."""
    a, b = pairs
    out = np.zeros(pairvec.shape[1:] + (n_ao, n_ao))
    v = np.moveaxis(pairvec, 0, -1)
    out[..., a, b] = v
    out[..., b, a] = v
    return out


def three_index(G, piv, pairs, n_ao):
    """(ab|K) for K in the basis, as [K][a][b]."""
    return unpack(np.asarray(G)[:, piv], pairs, n_ao)


def mo_vectors(G, piv, QinvT, C, pairs, p_batches=None):
    """Algorithm 1: for each batch P of MO indices p, X_pqK = sum_ab C_ap C_bq
    (ab|K) for all K in the basis, then L^J_pq = sum_K X_pqK [Q^-T]_KJ.
    Returns L [n_J][n_mo][n_mo]."""
    C = np.asarray(C)
    n_ao, n_mo = C.shape
    nJ = len(piv)
    if p_batches is None:
        p_batches = [np.arange(n_mo)]
    L = np.zeros((nJ, n_mo, n_mo))
    ao3 = three_index(G, piv, pairs, n_ao)
    for P in p_batches:
        X = np.einsum("ap,bq,Kab->pqK", C[:, P], C, ao3, optimize=True)
        L[:, P, :] = np.einsum("pqK,KJ->Jpq", X, QinvT, optimize=True)
    return L


def full_eri(G, pairs, n_ao):
    """(ab|cd) as a 4-index array from the packed pair matrix (small systems)."""
    a, b = pairs
    A1, B1, A2, B2 = a[:, None], b[:, None], a[None, :], b[None, :]
    g4 = np.zeros((n_ao,) * 4)
    for i1, j1 in ((A1, B1), (B1, A1)):
        for i2, j2 in ((A2, B2), (B2, A2)):
            g4[i1, j1, i2, j2] = G
    return g4


def mo_integrals_exact(G, C, pairs, n_ao):
    """g_pqrs = sum_abcd C_ap C_bq (ab|cd) C_cr C_ds from the full G."""
    return np.einsum("ap,bq,abcd,cr,ds->pqrs", C, C, full_eri(G, pairs, n_ao), C, C,
                     optimize=True)
