"""Correlated natural transition orbitals (CNTOs) from CCS excitation vectors,
and the semicanonical basis the multilevel models run in (Sec. 2.2: eqs. M,
N, approx_double_1, approx_double_2 and select_CNTOs) -- plain FP64 oracle.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Pinned by tests/test_oracle_cnto.py: gbar as the derivative of the X1
transformed g_aibj, the approximate doubles (with their 1/(1 + delta_{ai,bj})
on the diagonal pairs) as the first-order CIS(D)-type doubles of the CCS
state on explicit determinants, read as packed amplitudes of
sum_{ai >= bj} r_aibj E_ai E_bj, the delta terms of eqs. M and N and the
semicanonical basis.

Everything here is in the canonical basis of the full problem: L [K, n, n],
eps [n] (occupied first), a CCS excitation vector R [V, O] with its excitation
energy w.  The approximate doubles are full arrays (V, O, V, O) over all
orbitals.
"""
from __future__ import annotations

import numpy as np

from .mlcc import Dims, _einsum, core_hamiltonian


def gbar(L, d: Dims, R):
    """gbar_aibj = P^{ab}_{ij} (sum_{cJ} R_ci L^J_bj L^J_ac - sum_{kJ} R_bk L^J_kj L^J_ai)
    with P I_aibj = I_aibj + I_bjai (eq. approx_double_2)."""
    Lvo = L[:, d.vir, d.occ]
    Lvv = L[:, d.vir, d.vir]
    Loo = L[:, d.occ, d.occ]
    first = _einsum("ci,Kbj,Kac->aibj", R, Lvo, Lvv)
    second = _einsum("bk,Kkj,Kai->aibj", R, Loo, Lvo)
    I = first - second
    return I + I.transpose(2, 3, 0, 1)


def approx_doubles(L, eps, d: Dims, R, w):
    """R_aibj = -gbar_aibj / ((1 + delta_{ai,bj}) (eps_a + eps_b - eps_i - eps_j - w))
    (eq. approx_double_1)."""
    ev, eo = eps[d.vir], eps[d.occ]
    dai = ev[:, None] - eo[None, :]
    den = dai[:, :, None, None] + dai[None, None, :, :] - w
    n1 = d.V * d.O
    same = np.eye(n1).reshape(d.V, d.O, d.V, d.O)
    return -gbar(L, d, R) / ((1.0 + same) * den)


def cnto_matrices(L, eps, d: Dims, R, w):
    """M_ij and N_ab of eqs. M and N for one excitation (R, w):
    M_ij = sum_a R_ai R_aj + 1/2 sum_abk (1 + delta_{ai,bk} delta_ij) R_aibk R_ajbk,
    N_ab = sum_i R_ai R_bi + 1/2 sum_ijc (1 + delta_{ai,cj} delta_ab) R_aicj R_bicj."""
    R2 = approx_doubles(L, eps, d, R, w)
    # the delta terms: (ai) = (bk) with i = j picks R_aiai R_aiai
    rdiag = np.einsum("aiai->ai", R2) ** 2
    M = R.T @ R + 0.5 * np.einsum("aibk,ajbk->ij", R2, R2) + 0.5 * np.diag(rdiag.sum(axis=0))
    N = R @ R.T + 0.5 * np.einsum("aicj,bicj->ab", R2, R2) + 0.5 * np.diag(rdiag.sum(axis=1))
    return M, N


def fix_signs(C):
    """Column signs: the entry of largest magnitude (first of equals) positive."""
    C = C.copy()
    idx = np.argmax(np.abs(C), axis=0)
    s = np.sign(C[idx, np.arange(C.shape[1])])
    s[s == 0] = 1.0
    return C * s[None, :]


def _semicanonical(U, F, n_act):
    """Rotate within the first n_act columns of U and within the rest so that
    U^T F U is diagonal on both diagonal blocks (each in ascending order)."""
    Ua, Ui = U[:, :n_act], U[:, n_act:]
    ea, Wa = np.linalg.eigh(Ua.T @ F @ Ua)
    ei, Wi = np.linalg.eigh(Ui.T @ F @ Ui)
    return fix_signs(np.concatenate([Ua @ Wa, Ui @ Wi], axis=1)), np.concatenate([ea, ei])


def cnto_basis(L, eps, d: Dims, Rs, ws, n_occ_act, n_vir_act, fock=None):
    """Sec. 2.2: sum M and N over the excitations, diagonalise them, take the
    eigenvectors of the largest eigenvalues as the active orbitals (occupied
    and virtual separately), then make the active and inactive blocks
    semicanonical.  Returns a dict with
      Co [O, O], Cv [V, V]: new orbitals as columns (active first),
      m_eig [O], n_eig [V]: eigenvalues of M and N, descending,
      eps [n]: diagonal of the new Fock matrix (ABI order),
      fock [n, n]: the Fock matrix in the new basis,
      L [K, n, n]: Cholesky vectors in the new basis."""
    M = np.zeros((d.O, d.O))
    N = np.zeros((d.V, d.V))
    for R, w in zip(Rs, ws):
        m, nn = cnto_matrices(L, eps, d, np.asarray(R), float(w))
        M += m
        N += nn
    mw, mU = np.linalg.eigh(M)
    nw, nU = np.linalg.eigh(N)
    mw, mU = mw[::-1], mU[:, ::-1]
    nw, nU = nw[::-1], nU[:, ::-1]
    F = np.diag(eps) if fock is None else np.asarray(fock)
    Co, eo = _semicanonical(mU, F[d.occ, d.occ], n_occ_act)
    Cv, ev = _semicanonical(nU, F[d.vir, d.vir], n_vir_act)
    C = np.zeros((d.n, d.n))
    C[d.occ, d.occ] = Co
    C[d.vir, d.vir] = Cv
    Lnew = np.einsum("pr,Kpq,qs->Krs", C, L, C, optimize=True)
    return dict(Co=Co, Cv=Cv, m_eig=mw, n_eig=nw, eps=np.concatenate([eo, ev]),
                fock=C.T @ F @ C, L=Lnew, M=M, N=N)


def hf_energy_fock(L, fock, d: Dims):
    """E_HF = sum_I (h_II + F_II) with h = F - G(D_HF) and a full Fock matrix."""
    h = core_hamiltonian(L, np.diag(fock).copy(), d, fock=fock)
    return float(np.trace(h[d.occ, d.occ]) + np.trace(fock[d.occ, d.occ]))
