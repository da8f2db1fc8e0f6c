"""Pins of the two-step Cholesky decomposition oracle (oracle/cholesky.py:
Sec. 2.4, the RI-like expression, the MO-screened diagonal and Algorithm 1)
against what the definitions fix (CPU only):

* the full decomposition reproduces the integrals, and the MO vectors
  reproduce the exact MO transformation of the integrals
* an incomplete decomposition stops at max D < tau, and its residual G - L L^T
  is positive semidefinite with |residual_ij| <= sqrt(D_i D_j) < tau
* the RI-like vectors G[:, B] Q^-T are the pivoted-Cholesky vectors
* sum_J L^J_pq L^J_rs = sum_KL X_pqK (S^-1)_KL X_rsL
* batching over p does not change the vectors
* the MO-screened basis is smaller, and the error of every active MO integral
  (pq|pq) stays below (sum_ab |C_ap C_bq| sqrt(D_ab))^2 with the final D
* planted mistakes fail
"""
import numpy as np

from oracle import cholesky as oc
from paper_2006_05226_amd.synth import gen_ao_eri, gen_mo_coefficients, pair_index

N_AO, N_AUX, N_MO = 14, 40, 9


def inputs(seed=0):
    G, _ = gen_ao_eri(N_AO, N_AUX, seed)
    C = gen_mo_coefficients(N_AO, N_MO, seed + 1)
    return G, C, pair_index(N_AO)


def test_full_decomposition_is_exact():
    G, C, pairs = inputs()
    piv, L = oc.pivot_basis(G, 1e-14)
    assert len(piv) <= N_AUX
    assert np.abs(G - L @ L.T).max() < 1e-13 * np.abs(G).max()
    QiT = oc.inverse_factor_t(G, piv)
    Lmo = oc.mo_vectors(G, piv, QiT, C, pairs)
    g = oc.mo_integrals_exact(G, C, pairs, N_AO)
    assert np.abs(np.einsum("Jpq,Jrs->pqrs", Lmo, Lmo) - g).max() < 1e-12 * np.abs(g).max()


def test_incomplete_decomposition_bounds():
    G, C, pairs = inputs(1)
    tau = 1e-4 * np.diag(G).max()
    piv, L = oc.pivot_basis(G, tau)
    R = G - L @ L.T
    D = np.diag(R)
    assert D.max() < tau and D.min() > -1e-15
    assert np.linalg.eigvalsh(R).min() > -1e-13
    assert np.all(np.abs(R) <= np.sqrt(np.outer(np.maximum(D, 0), np.maximum(D, 0))) + 1e-14)
    # RI-like vectors are the decomposition's vectors
    QiT = oc.inverse_factor_t(G, piv)
    assert np.abs(oc.ri_vectors(G, piv, QiT) - L).max() < 1e-12 * np.abs(L).max()


def test_mo_vectors_identity_and_batching():
    G, C, pairs = inputs(2)
    piv, _ = oc.pivot_basis(G, 1e-6 * np.diag(G).max())
    QiT = oc.inverse_factor_t(G, piv)
    L = oc.mo_vectors(G, piv, QiT, C, pairs)
    ao3 = oc.three_index(G, piv, pairs, N_AO)
    X = np.einsum("ap,bq,Kab->pqK", C, C, ao3)
    Sinv = np.linalg.inv(G[np.ix_(piv, piv)])
    lhs = np.einsum("Jpq,Jrs->pqrs", L, L)
    rhs = np.einsum("pqK,KL,rsL->pqrs", X, Sinv, X)
    # both sides invert S: rounding grows with its condition number
    ev = np.linalg.eigvalsh(G[np.ix_(piv, piv)])
    tol = 50.0 * np.finfo(float).eps * ev.max() / ev.min()
    assert np.abs(lhs - rhs).max() < tol * np.abs(rhs).max()
    Lb = oc.mo_vectors(G, piv, QiT, C, pairs, p_batches=[np.arange(0, 4), np.arange(4, 7),
                                                         np.arange(7, N_MO)])
    # the same sums in another blocking order: rounding of products with the
    # entries of Q^-T, which grow as the square root of the condition number
    assert np.abs(Lb - L).max() < 50.0 * np.finfo(float).eps * np.sqrt(ev.max() / ev.min()) \
        * np.abs(L).max()


def test_mo_screening():
    G, C, pairs = inputs(3)
    tau = 1e-6 * np.diag(G).max()
    Ca = C[:, :3]                                   # active MOs
    nu = oc.screening_weights(Ca)
    piv0, _ = oc.pivot_basis(G, tau)
    piv, Lpair = oc.pivot_basis(G, tau, nu=nu, pairs=pairs)
    assert len(piv) < len(piv0)
    D = np.diag(G - Lpair @ Lpair.T)
    w = nu[pairs[0]] * nu[pairs[1]]
    assert (w * D).max() < tau
    QiT = oc.inverse_factor_t(G, piv)
    Lmo = oc.mo_vectors(G, piv, QiT, Ca, pairs)
    g = oc.mo_integrals_exact(G, Ca, pairs, N_AO)
    Dfull = oc.unpack(np.maximum(D, 0.0)[:, None], pairs, N_AO)[0]
    for p in range(3):
        for q in range(3):
            err = g[p, q, p, q] - np.sum(Lmo[:, p, q] ** 2)
            bound = np.sum(np.abs(np.outer(Ca[:, p], Ca[:, q])) * np.sqrt(Dfull)) ** 2
            assert -1e-14 <= err <= bound + 1e-14


def test_planted_mistakes_fail():
    G, C, pairs = inputs(4)
    piv, L = oc.pivot_basis(G, 1e-8 * np.diag(G).max())
    QiT = oc.inverse_factor_t(G, piv)
    # Q^-1 instead of Q^-T
    bad = oc.ri_vectors(G, piv, QiT.T)
    assert np.abs(bad - L).max() > 1e-3 * np.abs(L).max()
    # screening weights not squared
    nu_bad = np.abs(C[:, :3]).max(axis=1)
    nu = oc.screening_weights(C[:, :3])
    p1, _ = oc.pivot_basis(G, 1e-6 * np.diag(G).max(), nu=nu, pairs=pairs)
    p2, _ = oc.pivot_basis(G, 1e-6 * np.diag(G).max(), nu=nu_bad, pairs=pairs)
    assert len(p1) != len(p2) or np.any(p1 != p2)
