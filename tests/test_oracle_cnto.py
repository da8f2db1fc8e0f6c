"""Pins of the CNTO oracle (Sec. 2.2: eqs. M, N, approx_double_1,
approx_double_2, select_CNTOs) and of the full-Fock (semicanonical) model
input, against facts the definitions fix (CPU only).

* gbar is the derivative of the X1-transformed g_aibj in the direction of the
  excitation vector (eq. approx_double_2 against the X1 transformation)
* trace M = trace N, and the doubles part of the trace is the squared norm of
  the doubles over unique pairs (the delta terms of eqs. M and N)
* without doubles M = R^T R and N = R R^T (same nonzero spectrum)
* the new basis: orthogonal, semicanonical blocks, Hartree-Fock energy kept
* a full active space gives back the canonical orbitals: MLCC2 there is CC2
* MLCC2 with the full Fock matrix is unchanged by rotations among the inactive
  occupied or among the inactive virtual orbitals
* the approximate doubles of eq. approx_double_1 are the first-order
  (CIS(D)-type) doubles of the CCS state, -(F - <F>_HF - w)^-1 P_2 H R_1|HF>,
  built on explicit determinants and read as the amplitudes r of the operator
  sum_{ai >= bj} r_aibj E_ai E_bj: this fixes the 1/(1 + delta_{ai,bj}) factor
  on the diagonal pairs
* planted mistakes fail these pins
"""
import numpy as np
import pytest

from oracle import cnto as oc
from oracle import mlcc as om
from oracle.bruteforce import DetSpace
from paper_2006_05226_amd.synth import gen_inputs

pytestmark = pytest.mark.filterwarnings("ignore::numpy.exceptions.ComplexWarning")


def setup(O=3, V=5, J=14, seed=4):
    inp = gen_inputs(O, V, J, seed=seed)
    d = om.Dims(O, V, O, V)
    return inp, d


def cis_vectors(inp, d, n):
    """Lowest CIS (= CCS at the Hartree-Fock reference) roots and vectors."""
    A = om.cis_matrix(inp.L, inp.eps, om.Dims(d.O, d.V, 0, 0))
    w, U = np.linalg.eigh(A)
    return w[:n], [U[:, k].reshape(d.V, d.O) for k in range(n)]


def test_gbar_is_x1_derivative():
    inp, d = setup()
    rng = np.random.default_rng(1)
    R = rng.standard_normal((d.V, d.O))
    h = 1e-30
    Lt = om.x1_transform(inp.L.astype(complex), 1j * h * R, d)
    Lvo = Lt[:, d.vir, d.occ]
    dg = np.einsum("Kai,Kbj->aibj", Lvo, Lvo).imag / h
    g = oc.gbar(inp.L, d, R)
    assert np.abs(g - dg).max() < 1e-14 * np.abs(dg).max()


def packed_doubles_norm2(R2):
    V, O = R2.shape[:2]
    X = R2.reshape(V * O, V * O)
    s = 0.0
    for p in range(V * O):
        for q in range(p + 1):
            s += X[p, q] ** 2
    return s


def first_order_doubles_packed(inp, d, R, w):
    """-(F - <F>_HF - w)^-1 P_2 H R_1 |HF> on explicit determinants (R_1 =
    sum_ai R_ai E_ai, F = sum_p eps_p E_pp), as the coefficients r_aibj of
    sum_{ai >= bj} r_aibj E_ai E_bj |HF> (returned as a symmetric (V,O,V,O)
    array)."""
    S = DetSpace(d.n, d.O)
    H = S.hamiltonian(om.core_hamiltonian(inp.L, inp.eps, d), om.eri(inp.L))
    f = np.diag(S.fock_op(np.diag(inp.eps)))     # F is diagonal on determinants
    hf = S.hf_vector()
    vec = H @ (S.t1_op(R) @ hf)
    two = S.level == 2
    D = np.zeros_like(vec)
    D[two] = -vec[two] / (f[two] - f[S.hf] - w)
    # project() returns the biorthonormal coordinates: the ket coefficient on
    # ai != bj, twice it on ai = bj
    _, bio = S.project(D)
    n1 = d.V * d.O
    packed = bio.reshape(n1, n1).copy()
    packed[np.arange(n1), np.arange(n1)] *= 0.5
    return packed.reshape(d.V, d.O, d.V, d.O)


def test_approx_doubles_are_packed_first_order_doubles():
    """eq. approx_double_1 (with eq. approx_double_2) against the CIS(D)-type
    first-order doubles built from their definition on determinants; the
    diagonal pairs carry the 1/(1 + delta_{ai,bj}) of the packed amplitudes."""
    inp, d = setup(O=2, V=3, J=12, seed=5)
    w, Rs = cis_vectors(inp, d, 3)
    n1 = d.V * d.O
    for R, wk in zip(Rs, w):
        ref = first_order_doubles_packed(inp, d, R, wk)
        got = oc.approx_doubles(inp.L, inp.eps, d, R, wk)
        scale = np.abs(ref).max()
        assert scale > 1e-4
        assert np.abs(got - ref).max() < 1e-12 * scale
        diag = np.einsum("aiai->ai", ref)
        assert np.abs(diag).max() > 1e-3 * scale   # the diagonal pairs are exercised
        # planted mistake: the delta factor dropped (full-array doubles)
        full = -oc.gbar(inp.L, d, R) / (
            (inp.eps[d.vir][:, None] - inp.eps[d.occ][None, :])[:, :, None, None]
            + (inp.eps[d.vir][:, None] - inp.eps[d.occ][None, :])[None, None] - wk)
        assert np.abs(full - ref).max() > 1e-3 * scale
        assert np.abs(full.reshape(n1, n1) - ref.reshape(n1, n1))[~np.eye(n1, dtype=bool)].max() \
            < 1e-12 * scale


def test_traces_and_delta_factors():
    inp, d = setup()
    w, Rs = cis_vectors(inp, d, 2)
    for R, wk in zip(Rs, w):
        M, N = oc.cnto_matrices(inp.L, inp.eps, d, R, wk)
        assert np.allclose(M, M.T, atol=1e-15) and np.allclose(N, N.T, atol=1e-15)
        assert np.linalg.eigvalsh(M).min() > -1e-14 and np.linalg.eigvalsh(N).min() > -1e-14
        assert abs(np.trace(M) - np.trace(N)) < 1e-13
        R2 = oc.approx_doubles(inp.L, inp.eps, d, R, wk)
        assert abs(np.trace(M) - np.sum(R * R) - packed_doubles_norm2(R2)) < 1e-13


def test_no_doubles_limit():
    inp, d = setup()
    rng = np.random.default_rng(2)
    R = rng.standard_normal((d.V, d.O))
    M, N = oc.cnto_matrices(inp.L, inp.eps, d, R, 1e15)   # doubles ~ 1/w
    assert np.abs(M - R.T @ R).max() < 1e-12 and np.abs(N - R @ R.T).max() < 1e-12
    sv = np.linalg.svd(R, compute_uv=False) ** 2
    assert np.allclose(np.sort(np.linalg.eigvalsh(M))[::-1], sv, atol=1e-12)
    assert np.allclose(np.sort(np.linalg.eigvalsh(N))[::-1][: d.O], sv, atol=1e-12)


def test_new_basis_properties():
    inp, d = setup(O=4, V=8, J=20, seed=6)
    w, Rs = cis_vectors(inp, d, 3)
    o, v = 2, 3
    B = oc.cnto_basis(inp.L, inp.eps, d, Rs, w, o, v)
    Co, Cv, F = B["Co"], B["Cv"], B["fock"]
    assert np.abs(Co.T @ Co - np.eye(d.O)).max() < 1e-14
    assert np.abs(Cv.T @ Cv - np.eye(d.V)).max() < 1e-14
    blocks = [(slice(0, o), slice(0, o)), (slice(o, d.O), slice(o, d.O)),
              (slice(d.O, d.O + v), slice(d.O, d.O + v)), (slice(d.O + v, d.n), slice(d.O + v, d.n))]
    for b in blocks:
        blk = F[b]
        assert np.abs(blk - np.diag(np.diag(blk))).max() < 1e-14
    assert np.abs(F[d.occ, d.vir]).max() < 1e-15
    assert np.allclose(np.diag(F), B["eps"], atol=1e-15)
    # the active occupied space is spanned by the top eigenvectors of M
    mw, mU = np.linalg.eigh(B["M"])
    Pm = mU[:, -o:] @ mU[:, -o:].T
    assert np.abs(Co[:, :o] @ Co[:, :o].T - Pm).max() < 1e-12
    e0 = om.hf_energy(inp.L, inp.eps, d)
    assert abs(oc.hf_energy_fock(B["L"], F, d) - e0) < 1e-12 * abs(e0)


def test_full_active_space_is_canonical_cc2():
    inp, d = setup(O=2, V=4, J=12, seed=7)
    w, Rs = cis_vectors(inp, d, 2)
    B = oc.cnto_basis(inp.L, inp.eps, d, Rs, w, d.O, d.V)
    assert np.allclose(B["eps"], np.concatenate([np.sort(inp.eps[: d.O]), np.sort(inp.eps[d.O:])]),
                       atol=1e-13)
    P0 = om.Problem(inp.L, inp.eps, d, "mlcc2")
    P1 = om.Problem(B["L"], B["eps"], d, "mlcc2", fock=B["fock"])
    e0 = om.ground_state(P0, tol=1e-11)["energy"]
    e1 = om.ground_state(P1, tol=1e-11)["energy"]
    assert abs(e0 - e1) < 1e-12


def rotate_inactive(L, F, d, o, v, seed):
    rng = np.random.default_rng(seed)
    C = np.eye(d.n)
    qo, _ = np.linalg.qr(rng.standard_normal((d.O - o, d.O - o)))
    qv, _ = np.linalg.qr(rng.standard_normal((d.V - v, d.V - v)))
    C[o:d.O, o:d.O] = qo
    C[d.O + v:, d.O + v:] = qv
    return np.einsum("pr,Kpq,qs->Krs", C, L, C), C.T @ F @ C


@pytest.mark.parametrize("model", ["mlcc2", "mlccsd"])
def test_full_fock_invariance_under_inactive_rotations(model):
    inp, d0 = setup(O=4, V=7, J=16, seed=8)
    o, v = 2, 3
    d = om.Dims(d0.O, d0.V, o, v)
    F = np.diag(inp.eps)
    L1, F1 = rotate_inactive(inp.L, F, d, o, v, seed=9)
    assert np.abs(F1 - np.diag(np.diag(F1))).max() > 1e-3      # the Fock matrix is not diagonal
    P0 = om.Problem(inp.L, inp.eps, d, model)
    P1 = om.Problem(L1, np.diag(F1).copy(), d, model, fock=F1)
    g0 = om.ground_state(P0, tol=1e-11)
    g1 = om.ground_state(P1, tol=1e-11)
    assert abs(g0["energy"] - g1["energy"]) < 1e-12


# --- planted mistakes ------------------------------------------------------------

def test_planted_mistakes_fail(monkeypatch):
    inp, d = setup()
    w, Rs = cis_vectors(inp, d, 1)
    R, wk = Rs[0], w[0]

    # eq. M without its delta term
    R2 = oc.approx_doubles(inp.L, inp.eps, d, R, wk)
    M_wrong = R.T @ R + 0.5 * np.einsum("aibk,ajbk->ij", R2, R2)
    assert abs(np.trace(M_wrong) - np.sum(R * R) - packed_doubles_norm2(R2)) > 1e-9

    def unsymmetrised(L, d, R):
        Lvo, Lvv, Loo = L[:, d.vir, d.occ], L[:, d.vir, d.vir], L[:, d.occ, d.occ]
        return (np.einsum("ci,Kbj,Kac->aibj", R, Lvo, Lvv) - np.einsum("bk,Kkj,Kai->aibj", R, Loo, Lvo))

    h = 1e-30
    Lt = om.x1_transform(inp.L.astype(complex), 1j * h * R, d)
    Lvo = Lt[:, d.vir, d.occ]
    dg = np.einsum("Kai,Kbj->aibj", Lvo, Lvo).imag / h
    assert np.abs(unsymmetrised(inp.L, d, R) - dg).max() > 1e-6 * np.abs(dg).max()
