"""The two-step Cholesky decomposition on the GPU (Sec. 2.4): the basis by
pivoted Cholesky with and without the MO-screened diagonal, Q^-T, and the MO
Cholesky vectors of Algorithm 1 in batches over p, against the FP64 oracle
(oracle/cholesky.py) on the same seeded synthetic AO integrals."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import cholesky as oc  # noqa: E402
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import gen_ao_eri, gen_mo_coefficients, pair_index  # noqa: E402

from gpu_util import rel, tol_chain  # noqa: E402

pytestmark = pytest.mark.gpu

N_AO, N_AUX, N_MO, N_ACT = 40, 120, 24, 8


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


@pytest.fixture(scope="module")
def inputs():
    G, _ = gen_ao_eri(N_AO, N_AUX, 11)
    C = gen_mo_coefficients(N_AO, N_MO, 12)
    return G, C, pair_index(N_AO)


def cond(G, piv):
    ev = np.linalg.eigvalsh(G[np.ix_(piv, piv)])
    return ev.max() / ev.min()


def inverse_tol(G, piv):
    """Relative error bound of a triangular inverse of the n x n factor Q of
    S = Q Q^T in FP64: n eps cond(Q) with cond(Q) = sqrt(cond(S)), times 10."""
    return 10.0 * len(piv) * np.finfo(float).eps * np.sqrt(cond(G, piv))


@pytest.mark.parametrize("screened", [False, True])
def test_basis(ctx, inputs, screened):
    G, C, pairs = inputs
    tau = 1e-6 * np.diag(G).max()
    nu = oc.screening_weights(C[:, :N_ACT]) if screened else None
    piv_ref, _ = oc.pivot_basis(G, tau, nu=nu, pairs=pairs)
    piv, QiT = ctx.cholesky_basis(N_AO, G, tau, nu=nu)
    assert np.array_equal(piv, piv_ref)               # index work: bit-exact
    QiT_ref = oc.inverse_factor_t(G, piv_ref)
    assert rel(QiT, QiT_ref) < inverse_tol(G, piv_ref)
    if screened:
        piv0, _ = oc.pivot_basis(G, tau)
        assert len(piv) < len(piv0)


def test_basis_max_vectors_and_device_buffers(ctx, inputs):
    G, C, pairs = inputs
    tau = 1e-12 * np.diag(G).max()
    piv, _ = ctx.cholesky_basis(N_AO, torch.tensor(G, device="cuda"), tau, max_vectors=17)
    assert len(piv) == 17
    piv_ref, _ = oc.pivot_basis(G, tau, max_vectors=17)
    assert np.array_equal(piv, piv_ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("p_batch", [0, 5])
def test_mo_vectors(ctx, inputs, precision, p_batch):
    G, C, pairs = inputs
    tau = 1e-6 * np.diag(G).max()
    piv, QiT = ctx.cholesky_basis(N_AO, G, tau)
    QiT_ref = oc.inverse_factor_t(G, piv)
    ref = oc.mo_vectors(G, piv, QiT_ref, C, pairs)
    got = ctx.mo_cholesky(N_AO, N_MO, G, piv, QiT, C, precision=precision, p_batch=p_batch)
    if precision == "fp64":
        tol = inverse_tol(G, piv)
    else:
        # three contractions (reductions over n_ao, n_ao and the basis) whose
        # rounding is amplified by the entries of Q^-T
        tol = tol_chain(precision, max(N_AO, len(piv)), stages=3) * np.sqrt(cond(G, piv))
    assert rel(got, ref) < tol


def test_mo_vectors_full_rank_reproduce_mo_integrals(ctx, inputs):
    G, C, pairs = inputs
    piv, QiT = ctx.cholesky_basis(N_AO, G, 1e-13 * np.diag(G).max())
    L = ctx.mo_cholesky(N_AO, N_MO, G, piv, QiT, C, p_batch=7)
    g = oc.mo_integrals_exact(G, C, pairs, N_AO)
    assert rel(np.einsum("Jpq,Jrs->pqrs", L, L), g) < 1e-10


def test_device_output_and_errors(ctx, inputs):
    G, C, pairs = inputs
    piv, QiT = ctx.cholesky_basis(N_AO, G, 1e-6 * np.diag(G).max())
    out = torch.empty((len(piv), N_MO, N_MO), dtype=torch.float64, device="cuda")
    ctx.mo_cholesky(N_AO, N_MO, G, piv, QiT, C, out=out)
    host = ctx.mo_cholesky(N_AO, N_MO, G, piv, QiT, C)
    assert np.array_equal(out.cpu().numpy(), host)
    with pytest.raises(mlcc.MlccError) as e:
        ctx.cholesky_basis(N_AO, G, -1.0)
    assert e.value.status == mlcc.E_ARG
    bad = piv.copy()
    bad[0] = N_AO * (N_AO + 1) // 2
    with pytest.raises(mlcc.MlccError) as e:
        ctx.mo_cholesky(N_AO, N_MO, G, bad, QiT, C)
    assert e.value.status == mlcc.E_ARG
