"""Three-level MLCCSD (CCS/CC2/CCSD) residual of the dense oracle
(mlcc.mlccsd3_omega, with mlcc.ccsd_doubles inside the CCSD space) at sampled
doubles (a, i, b, j), for workloads whose ladder integrals over the CC2 space
do not fit in host memory.

TEST INFRASTRUCTURE ONLY -- never called by the product path.

Sec. 2.1 (X = X1 + S2 + T2) and Appendix A (MLCCSD Omega vector, in terms of
the X1-dressed Cholesky vectors): every factor of ccsd_doubles is formed over
the whole active (CC2) space from the dressed blocks L~_vo, L~_ov, L~_oo and
L~_vv (sampled.lt_block) and the dressed Fock blocks (sampled.fock_block),
except the virtual-virtual integrals g~_acbd of the ladder term, which are
formed for the sampled (a, b) only.  Each term is the one of ccsd_doubles
evaluated at the sample:

  Omega_aibj = A2 + B2 + R_aibj + R_bjai,  R = C2 + D2 + E2   (CCSD space)
  Omega_aibj = g~_aibj + eps_aibj x_aibj                      (elsewhere)

and the singles are sampled.omega1_samples with the given doubles x2.  The
Jacobian transformation follows by complex step on the same evaluation.

Pinned by tests/test_oracle_sampled_ccsd.py against mlcc.mlccsd3_omega.
"""
from __future__ import annotations

import numpy as np

from . import sampled as sm
from .mlcc import Dims, _einsum, u_of


def _blocks(Lsrc, t1, d: Dims, rows, cols):
    J = Lsrc.n_chol
    return np.concatenate([sm.lt_block(Lsrc, t1, d, np.arange(k0, min(J, k0 + sm.KCHUNK)), rows, cols)
                           for k0 in range(0, J, sm.KCHUNK)])


class Blocks:
    """Dressed active blocks of L~ (K first) and the intermediates that every
    sample shares: g~_kcld, L~_kcld = 2 g~_kcld - g~_kdlc and the E2
    intermediates W_bc = F~_bc - sum_dkl u_bkdl g~_ldkc and
    W_kj = F~_kj + sum_cdl u_cldj g~_kdlc, u = 2 x - x(i<->j)."""

    def __init__(self, Lsrc, eps, d: Dims, t1, x2):
        ao = np.arange(d.o)
        av = d.O + np.arange(d.v)
        self.d = d
        self.vo = _blocks(Lsrc, t1, d, av, ao)
        self.ov = _blocks(Lsrc, t1, d, ao, av)
        self.oo = _blocks(Lsrc, t1, d, ao, ao)
        self.vv = _blocks(Lsrc, t1, d, av, av)
        act = np.concatenate([ao, av])
        F = sm.fock_block(Lsrc, eps, d, t1, act, act)
        self.Foo, self.Fvv = F[:d.o, :d.o], F[d.o:, d.o:]
        self.t = x2
        self.u = u_of(x2)
        self.den = sm._den(eps, d)
        E = _einsum
        self.g_ovov = E("Kkc,Kld->kcld", self.ov, self.ov)
        self.L_ovov = 2.0 * self.g_ovov - self.g_ovov.transpose(0, 3, 2, 1)
        self.Wvv = self.Fvv - E("bkdl,ldkc->bc", self.u, self.g_ovov)
        self.Woo = self.Foo + E("cldj,kdlc->kj", self.u, self.g_ovov)

    def _Y(self, a, i):
        """Y_aick over (c, k): g~_kiac - 1/2 sum_dl t_aldi g~_kdlc."""
        g_kiac = _einsum("Kk,Kc->kc", self.oo[:, :, i], self.vv[:, a, :])
        return g_kiac.T - 0.5 * _einsum("ld,kdlc->ck", self.t[a, :, :, i], self.g_ovov)

    def _Z(self, a, i):
        """Z_aikc over (k, c): L~_aikc + 1/2 sum_dl u_aidl L~_ldkc,
        L~_aikc = 2 g~_aikc - g~_acki."""
        g_aikc = _einsum("K,Kkc->kc", self.vo[:, a, i], self.ov)
        g_acki = _einsum("Kc,Kk->kc", self.vv[:, a, :], self.oo[:, :, i])
        return 2.0 * g_aikc - g_acki + 0.5 * _einsum("dl,ldkc->kc", self.u[a, i], self.L_ovov)

    def _R(self, a, i, b, j):
        """C2 + D2 + E2 at (a, i, b, j)."""
        t, u = self.t, self.u
        C2 = (-0.5 * np.sum(t[b, :, :, j].T * self._Y(a, i))
              - np.sum(t[b, :, :, i].T * self._Y(a, j)))
        D2 = 0.5 * np.sum(u[b, j].T * self._Z(a, i))
        E2 = t[a, i, :, j] @ self.Wvv[b, :] - t[a, i, b, :] @ self.Woo[:, j]
        return C2 + D2 + E2

    def omega2(self, a, i, b, j, ccsd: bool):
        """Omega_aibj; ccsd: the four indices lie in the CCSD space."""
        t = self.t
        g_aibj = self.vo[:, a, i] @ self.vo[:, b, j]
        if not ccsd:
            return g_aibj + (self.den[a, i] + self.den[b, j]) * t[a, i, b, j]
        g_acbd = self.vv[:, a, :].T @ self.vv[:, b, :]
        A2 = g_aibj + np.sum(t[:, i, :, j] * g_acbd)
        g_kilj = _einsum("Kk,Kl->kl", self.oo[:, :, i], self.oo[:, :, j])
        Q = g_kilj + _einsum("cd,kcld->kl", t[:, i, :, j], self.g_ovov)
        B2 = np.sum(t[a, :, b, :] * Q)
        return A2 + B2 + self._R(a, i, b, j) + self._R(b, j, a, i)


def mlccsd3_omega2_samples(Lsrc, eps, d: Dims, o_t, v_t, t1, x2, quads, blocks=None):
    """Omega_aibj of the three-level model at quadruples (a, i, b, j) of
    active indices (a, b relative to the active virtual block); the CCSD
    space is the first v_t active virtuals and o_t active occupied."""
    B = blocks or Blocks(Lsrc, eps, d, t1, x2)
    out = []
    for a, i, b, j in np.asarray(quads):
        ccsd = a < v_t and b < v_t and i < o_t and j < o_t
        out.append(B.omega2(int(a), int(i), int(b), int(j), bool(ccsd)))
    return np.array(out)


def mlccsd3_omega1_samples(Lsrc, eps, d: Dims, t1, x2, pairs, act=None):
    """Omega_AI of the three-level model at (A, I): the singles of
    exp(-X) H exp(X) with the doubles x2 of the whole active space."""
    return sm.omega1_samples(Lsrc, eps, d, t1, pairs, act=act, x2=x2)


def mlccsd3_sigma_samples(Lsrc, eps, d: Dims, o_t, v_t, t1, x2, c1, c2, quads, pairs, h=1e-30):
    """Jacobian transformation sigma = A c of the three-level model (the
    derivative of the residual, Sec. 2.1) at sampled doubles and singles, by
    complex step: sigma = Im Omega(t1 + i h c1, x2 + i h c2) / h, every step
    of the residual above being analytic in the amplitudes.  c1 (V, O),
    c2 (v, o, v, o) symmetric."""
    tc = t1.astype(complex) + 1j * h * c1
    xc = x2.astype(complex) + 1j * h * c2
    B = Blocks(Lsrc, eps, d, tc, xc)
    s2 = mlccsd3_omega2_samples(Lsrc, eps, d, o_t, v_t, tc, xc, quads, blocks=B).imag / h
    s1 = mlccsd3_omega1_samples(Lsrc, eps, d, tc, xc, pairs).imag / h
    return s1, s2
