"""Determinant-space engine and two-electron FCI: the plain definitions that
pin the oracle's residuals, energies and Jacobians.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Everything here is second quantisation written out on explicit determinant
vectors (spin strings as bit masks, alpha and beta strings of fixed length):

* E_pq = a+_{p alpha} a_{q alpha} + a+_{p beta} a_{q beta}
* H = sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - delta_qr E_ps)
* exp(+-X) |.> by its Taylor series, exact because cluster operators are
  nilpotent
* a residual Omega_mu = <mu_bar| ... |HF> is read off as the coordinates of the
  excitation-level-1 and -2 part of the state in the ket basis
  {E_AI|HF>, E_AI E_BJ|HF> (AI >= BJ)}, solved by least squares; with the full
  symmetric doubles convention this gives Omega_aibj = c_aibj (ai != bj) and
  Omega_aiai = 2 c_aiai, i.e. the biorthonormal projection.

Sizes: n <= 6 spatial orbitals (a few hundred determinants).
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np


class DetSpace:
    def __init__(self, n: int, n_occ: int):
        self.n = n
        self.O = n_occ
        self.strings = [sum(1 << b for b in c) for c in itertools.combinations(range(n), n_occ)]
        self.index = {s: k for k, s in enumerate(self.strings)}
        ns = len(self.strings)
        self.ns = ns
        self.dim = ns * ns
        assert ns == comb(n, n_occ)
        # one-spin excitation matrices a+_p a_q on strings
        self._ex = np.zeros((n, n, ns, ns))
        for k, s in enumerate(self.strings):
            for q in range(n):
                if not (s >> q) & 1:
                    continue
                s1 = s & ~(1 << q)
                sg1 = (-1) ** bin(s & ((1 << q) - 1)).count("1")
                for p in range(n):
                    if (s1 >> p) & 1:
                        continue
                    s2 = s1 | (1 << p)
                    sg2 = (-1) ** bin(s1 & ((1 << p) - 1)).count("1")
                    self._ex[p, q, self.index[s2], k] = sg1 * sg2
        I = np.eye(ns)
        # singlet excitation operators on the product space (alpha major)
        self.E = np.array([[np.kron(self._ex[p, q], I) + np.kron(I, self._ex[p, q])
                            for q in range(n)] for p in range(n)])
        hf = (1 << n_occ) - 1
        self.hf = self.index[hf] * ns + self.index[hf]
        # excitation level of each determinant
        lvl_s = np.array([bin(s >> n_occ).count("1") for s in self.strings])
        self.level = (lvl_s[:, None] + lvl_s[None, :]).ravel()

    def hf_vector(self):
        v = np.zeros(self.dim)
        v[self.hf] = 1.0
        return v

    def hamiltonian(self, h, g):
        n = self.n
        E = self.E
        H = np.einsum("pq,pqxy->xy", h, E)
        W = np.einsum("pqrs,rsxy->pqxy", g, E)
        H += 0.5 * np.einsum("pqxz,pqzy->xy", E, W)
        H -= 0.5 * np.einsum("pqqs,psxy->xy", g, E)
        return H

    # cluster operators ----------------------------------------------------
    def t1_op(self, t1):
        O = self.O
        V = self.n - O
        X = np.zeros((self.dim, self.dim), dtype=np.result_type(t1, float))
        for A in range(V):
            for I in range(O):
                X = X + t1[A, I] * self.E[O + A, I]
        return X

    def t2_op(self, x2, o, v):
        """1/2 sum x_aibj E_ai E_bj over the active space (full symmetric x2)."""
        O = self.O
        X = np.zeros((self.dim, self.dim), dtype=np.result_type(x2, float))
        for a, i, b, j in itertools.product(range(v), range(o), range(v), range(o)):
            c = x2[a, i, b, j]
            if c != 0:
                X = X + 0.5 * c * (self.E[O + a, i] @ self.E[O + b, j])
        return X

    def fock_op(self, F):
        return np.einsum("pq,pqxy->xy", F, self.E)

    # projection -----------------------------------------------------------
    def _ket_basis(self):
        O = self.O
        V = self.n - O
        hf = self.hf_vector()
        singles = [(A, I) for A in range(V) for I in range(O)]
        cols = [self.E[O + A, I] @ hf for A, I in singles]
        pairs = []
        for p1 in range(len(singles)):
            for p2 in range(p1 + 1):
                (A, I), (B, J) = singles[p1], singles[p2]
                pairs.append((p1, p2))
                cols.append(self.E[O + A, I] @ (self.E[O + B, J] @ hf))
        return np.array(cols).T, singles, pairs

    def project(self, vec):
        """Coordinates of the level-1/2 part of vec: returns (Omega1 (V,O),
        Omega2 full (V,O,V,O)) in the biorthonormal convention."""
        O = self.O
        V = self.n - O
        B, singles, pairs = self._ket_basis()
        mask = (self.level == 1) | (self.level == 2)
        rhs = np.where(mask, vec, 0.0)
        Bm = B
        if np.iscomplexobj(rhs):
            cr = np.linalg.lstsq(Bm, rhs.real, rcond=None)[0]
            ci = np.linalg.lstsq(Bm, rhs.imag, rcond=None)[0]
            c = cr + 1j * ci
        else:
            c = np.linalg.lstsq(Bm, rhs, rcond=None)[0]
        resid = np.linalg.norm(Bm @ c - rhs)
        assert resid < 1e-9 * max(1.0, np.linalg.norm(rhs)), resid
        n1 = V * O
        om1 = c[:n1].reshape(V, O)
        om2 = np.zeros((n1, n1), dtype=c.dtype)
        for k, (p1, p2) in enumerate(pairs):
            val = c[n1 + k]
            if p1 == p2:
                om2[p1, p1] = 2.0 * val
            else:
                om2[p1, p2] = val
                om2[p2, p1] = val
        return om1, om2.reshape(V, O, V, O)


def expm_nilpotent_apply(X, vec, sign=1.0):
    """exp(sign * X) vec by the (finite) Taylor series."""
    out = vec.copy()
    term = vec.copy()
    for k in range(1, 64):
        term = sign * (X @ term) / k
        out = out + term
        if np.max(np.abs(term)) < 1e-300:
            break
    return out


class BruteForce:
    """Residuals, energies and Jacobians of CCS, MLCC2, MLCCSD and three-level
    MLCCSD from their definitions on explicit determinant vectors."""

    def __init__(self, h, g, eps, O, o, v):
        self.n = h.shape[0]
        self.O = O
        self.V = self.n - O
        self.o, self.v = o, v
        self.h, self.g = h, g
        self.eps = eps
        self.S = DetSpace(self.n, O)
        self.H = self.S.hamiltonian(h, g)
        self.F = self.S.fock_op(np.diag(eps))
        self.hf = self.S.hf_vector()
        self.E_hf = float(self.hf @ self.H @ self.hf)

    def _embed(self, x2):
        """active (v,o,v,o) -> full (V,O,V,O)."""
        full = np.zeros((self.V, self.O, self.V, self.O), dtype=np.result_type(x2, float))
        full[: self.v, : self.o, : self.v, : self.o] = x2
        return full

    def _act(self, om2):
        return om2[: self.v, : self.o, : self.v, : self.o]

    def sim(self, X, op_vec):
        """exp(-X) op exp(X) |HF> for an operator matrix op."""
        w = expm_nilpotent_apply(X, self.hf, +1.0)
        w = op_vec(w)
        return expm_nilpotent_apply(X, w, -1.0)

    def energy(self, t1, x2):
        X = self.S.t1_op(t1)
        if x2 is not None:
            X = X + self.S.t2_op(x2, self.o, self.v)
        return float(self.hf @ self.sim(X, lambda w: self.H @ w)) - self.E_hf

    def omega_mlccsd(self, t1, t2):
        X = self.S.t1_op(t1)
        if t2 is not None:
            X = X + self.S.t2_op(t2, self.o, self.v)
        om1, om2 = self.S.project(self.sim(X, lambda w: self.H @ w))
        return om1, self._act(om2)

    def omega_mlcc2(self, t1, s):
        T1 = self.S.t1_op(t1)
        S2 = self.S.t2_op(s, self.o, self.v)
        om1, _ = self.S.project(self.sim(T1 + S2, lambda w: self.H @ w))
        # <mu2| H~ + [F, S2] |HF>
        vec = self.sim(T1, lambda w: self.H @ w) + self.F @ (S2 @ self.hf) - S2 @ (self.F @ self.hf)
        _, om2 = self.S.project(vec)
        return om1, self._act(om2)

    def _ccsd_rows(self, o_t, v_t):
        """(v,o,v,o) selector of the projections inside the CCSD space of the
        three-level model: a < v_t, i < o_t, b < v_t and j < o_t."""
        a = np.arange(self.v)[:, None, None, None]
        i = np.arange(self.o)[None, :, None, None]
        b = np.arange(self.v)[None, None, :, None]
        j = np.arange(self.o)[None, None, None, :]
        return (a < v_t) & (i < o_t) & (b < v_t) & (j < o_t)

    def omega_mlccsd3(self, t1, x2, o_t, v_t):
        """Three-level MLCCSD (X = X1 + S2 + T2, x2 = S2 + T2 over the active
        space): singles and the doubles inside the CCSD space project
        exp(-X) H exp(X)|HF>; the other active doubles project
        H~|HF> + [F, X2]|HF>."""
        T1 = self.S.t1_op(t1)
        X2 = self.S.t2_op(x2, self.o, self.v)
        om1, full = self.S.project(self.sim(T1 + X2, lambda w: self.H @ w))
        vec = self.sim(T1, lambda w: self.H @ w) + self.F @ (X2 @ self.hf) - X2 @ (self.F @ self.hf)
        _, cc2 = self.S.project(vec)
        return om1, np.where(self._ccsd_rows(o_t, v_t), self._act(full), self._act(cc2))

    def jacobian_mlccsd3(self, t1, x2, c1, c2, o_t, v_t):
        """Derivative of omega_mlccsd3 along (c1, c2), from commutators:
        singles and CCSD-space rows <mu| exp(-X)[H, tau(c)]exp(X) |HF>, the
        other rows <mu2| exp(-T1)[H, tau(c1)]exp(T1) + [F, tau(c2)] |HF>."""
        T1 = self.S.t1_op(t1)
        X2 = self.S.t2_op(x2, self.o, self.v)
        tau = self._tau(c1, c2)
        comm = lambda w: self.H @ (tau @ w) - tau @ (self.H @ w)  # noqa: E731
        s1, full = self.S.project(self.sim(T1 + X2, comm))
        tau1 = self.S.t1_op(c1)
        comm1 = lambda w: self.H @ (tau1 @ w) - tau1 @ (self.H @ w)  # noqa: E731
        tau2 = self.S.t2_op(c2, self.o, self.v)
        vec = self.sim(T1, comm1) + self.F @ (tau2 @ self.hf) - tau2 @ (self.F @ self.hf)
        _, cc2 = self.S.project(vec)
        return s1, np.where(self._ccsd_rows(o_t, v_t), self._act(full), self._act(cc2))

    def _tau(self, c1, c2):
        op = self.S.t1_op(c1)
        if c2 is not None:
            op = op + self.S.t2_op(c2, self.o, self.v)
        return op

    def jacobian_mlccsd(self, t1, t2, c1, c2):
        """sigma = coordinates of P exp(-X) [H, tau(c)] exp(X) |HF>."""
        X = self.S.t1_op(t1)
        if t2 is not None:
            X = X + self.S.t2_op(t2, self.o, self.v)
        tau = self._tau(c1, c2)
        comm = lambda w: self.H @ (tau @ w) - tau @ (self.H @ w)  # noqa: E731
        s1, s2 = self.S.project(self.sim(X, comm))
        return s1, self._act(s2)

    def jacobian_mlcc2(self, t1, s, c1, c2):
        """Blocks of the MLCC2 Jacobian (Sec. 2.1):
        A11 c1 + A12 c2 = <mu1| exp(-X)[H, tau(c)]exp(X) |HF>   (X = T1 + S2)
        A21 c1 = <mu2| exp(-T1)[H, tau(c1)]exp(T1) |HF>,  A22 c2 = <mu2|[F, tau(c2)]|HF>"""
        T1 = self.S.t1_op(t1)
        S2 = self.S.t2_op(s, self.o, self.v)
        tau = self._tau(c1, c2)
        comm = lambda w: self.H @ (tau @ w) - tau @ (self.H @ w)  # noqa: E731
        s1, _ = self.S.project(self.sim(T1 + S2, comm))
        tau1 = self.S.t1_op(c1)
        comm1 = lambda w: self.H @ (tau1 @ w) - tau1 @ (self.H @ w)  # noqa: E731
        vec = self.sim(T1, comm1)
        if c2 is not None:
            tau2 = self.S.t2_op(c2, self.o, self.v)
            vec = vec + self.F @ (tau2 @ self.hf) - tau2 @ (self.F @ self.hf)
        _, s2 = self.S.project(vec)
        return s1, self._act(s2)

    def spectrum(self):
        """All eigenvalues of H in the fixed (N_alpha, N_beta) determinant space
        (singlets and the M_S = 0 components of higher multiplets)."""
        return np.linalg.eigvalsh(self.H)


def fci_two_electron(h, g):
    """Singlet two-electron FCI as the eigenproblem of the symmetric-C map
    C -> hC + Ch + G[C],  G[C]_pq = sum_rs g_prqs C_rs  (spatial wavefunction
    sum_pq C_pq phi_p(1) phi_q(2), C = C^T).  Returns sorted eigenvalues."""
    n = h.shape[0]
    basis = []
    for p in range(n):
        for q in range(p + 1):
            B = np.zeros((n, n))
            if p == q:
                B[p, p] = 1.0
            else:
                B[p, q] = B[q, p] = 1.0 / np.sqrt(2.0)
            basis.append(B)
    Hm = np.zeros((len(basis), len(basis)))
    for c, B in enumerate(basis):
        HB = h @ B + B @ h.T + np.einsum("prqs,rs->pq", g, B)
        for r, Bp in enumerate(basis):
            Hm[r, c] = np.sum(Bp * HB)
    return np.sort(np.linalg.eigvalsh(0.5 * (Hm + Hm.T)))
