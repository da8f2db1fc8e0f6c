"""Edge cases on the GPU against the FP64 oracle: an empty active space
(MLCC2 reduces to CCS: t1 = 0, roots = CIS), dimensions that are all prime
(ragged tiles everywhere, no 16-byte alignment), more trial vectors than
one Jacobian batch holds, every root of a small problem, and the size limits
of the ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import mlcc as om  # noqa: E402
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import gen_amplitudes, gen_eps, gen_inputs, gen_vectors  # noqa: E402

from gpu_util import bar, full_vec, make, rel  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


@pytest.mark.parametrize("o,v", [(0, 13), (4, 0)])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_empty_active_space_is_ccs(ctx, o, v, precision):
    """With no active pairs MLCC2 is CCS: the canonical reference already
    satisfies it (t1 = 0, E = 0) and the roots are the CIS eigenvalues."""
    O, V, J = 5, 23, 40
    inp = gen_inputs(O, V, J, o, v, seed=3)
    P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model="mlcc2", precision=precision)
    gs = P.ground_state(tol=1e-10 if precision == "fp64" else 1e-6)
    assert gs["converged"]
    assert abs(gs["energy"]) < 1e-12 and np.abs(gs["t1"]).max() < 1e-12
    dav = P.davidson(4, tol=1e-8)
    d = om.Dims(O, V, 0, 0)
    cis = np.sort(np.linalg.eigvalsh(om.cis_matrix(inp.L, inp.eps, d).reshape(V * O, V * O)))
    tol = 1e-10 if precision == "fp64" else 1e-6
    assert np.abs(np.array(dav["omega"]) - cis[:4]).max() < tol


@pytest.mark.parametrize("model", ["mlcc2", "mlccsd"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_prime_dimensions(ctx, model, precision):
    """O=7, V=37, n_chol=53, active 3/13: every extent is prime, so every
    tile is ragged and no row is 16-byte aligned."""
    tol = bar(precision, 53, 8 if model == "mlccsd" else 6)
    inp, _, P, OP, d = make(7, 37, 53, 3, 13, seed=5, model=model, precision=precision, ctx=ctx)
    t1, x2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=6, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, x2.reshape(d.M, d.M))
    om1, om2, _, e = P.residual()
    r1, r2 = OP.omega(t1, x2)
    assert rel(om1, r1) < tol and rel(om2, r2.reshape(d.M, d.M)) < tol
    assert abs(e - OP.energy(t1, x2)) < tol * abs(OP.energy(t1, x2))
    c1, c2 = gen_vectors(2, d.O, d.V, d.M, seed=7)
    sig = P.jacobian_transform(np.stack([full_vec(c1[i], c2[i]) for i in range(2)]))
    for i in range(2):
        s1, s2 = om.jacobian_transform(OP, t1, x2, c1[i], c2[i].reshape(d.v, d.o, d.v, d.o))
        assert rel(sig[i], full_vec(s1, s2)) < tol


def test_more_vectors_than_one_batch(ctx):
    """11 trial vectors in one call (batches of at most 8): every result equals
    the vector transformed alone, and the last one matches the oracle."""
    inp, _, P, OP, d = make(6, 30, 50, 3, 12, seed=8, ctx=ctx)
    t1, x2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=9, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, x2.reshape(d.M, d.M))
    c1, c2 = gen_vectors(11, d.O, d.V, d.M, seed=10)
    c = np.stack([full_vec(c1[i], c2[i]) for i in range(11)])
    sig = P.jacobian_transform(c)
    for i in (0, 7, 8, 10):
        alone = P.jacobian_transform(c[i:i + 1])[0]
        assert rel(sig[i], alone) < 1e-13
    s1, s2 = om.jacobian_transform(OP, t1, x2, c1[10], c2[10].reshape(d.v, d.o, d.v, d.o))
    assert rel(sig[10], full_vec(s1, s2)) < 1e-11


def test_every_root_of_a_small_problem(ctx):
    """CCS with V*O = 12: all 12 roots (the Davidson space spans the whole
    problem) equal the CIS spectrum."""
    O, V = 3, 4
    inp = gen_inputs(O, V, 20, seed=11)
    P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, 0, 0, model="ccs")
    P.ground_state(tol=1e-12)
    dav = P.davidson(O * V, tol=1e-9)
    cis = np.sort(np.linalg.eigvalsh(
        om.cis_matrix(inp.L, inp.eps, om.Dims(O, V, 0, 0)).reshape(V * O, V * O)))
    assert dav["converged"]
    assert np.abs(np.array(dav["omega"]) - cis).max() < 1e-10


def test_size_limits(ctx):
    """Requests beyond the supported extents are refused before any device
    memory is touched."""
    eps = gen_eps(300, 200, 300, seed=0)
    with pytest.raises(mlcc.MlccError) as e:  # 300 * 200 = 60000 active pairs > 46340
        mlcc.Problem(ctx, None, eps, 300, 200, 300, 200, n_chol=1, seed=1)
    assert e.value.status == mlcc.E_ARG
    eps = gen_eps(40000, 30000, 10, seed=0)
    with pytest.raises(mlcc.MlccError) as e:  # 70000 orbitals > 65535
        mlcc.Problem(ctx, None, eps, 40000, 30000, 10, 10, n_chol=1, seed=1)
    assert e.value.status == mlcc.E_ARG
    with pytest.raises(mlcc.MlccError) as e:
        mlcc.Problem(ctx, None, gen_eps(5, 20, 5, seed=0), 5, 20, 6, 10, n_chol=4, seed=1)
    assert e.value.status == mlcc.E_ARG


@pytest.mark.parametrize("model", ["mlcc2", "mlccsd"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_literal_scale_stress_input(ctx, model, precision):
    """Cholesky vectors at the literal scale N(0,1) exp(-J/10) (integrals of
    order 1 Eh and above, an unstable reference): a kernel-parity stress input
    for the residual and the Jacobian transformation at random amplitudes,
    with the same bars as the realistic scale."""
    O, V, J, o, v = 6, 23, 41, 4, 9
    inp = gen_inputs(O, V, J, o, v, seed=11, scale=1.0)
    P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model=model, precision=precision)
    d = om.Dims(O, V, o, v)
    OP = om.Problem(inp.L, inp.eps, d, model)
    tol = bar(precision, max(J, d.M), 8 if model == "mlccsd" else 6)
    t1, x2 = gen_amplitudes(O, V, o, v, seed=12, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, x2.reshape(d.M, d.M))
    om1, om2, _, _ = P.residual()
    r1, r2 = OP.omega(t1, x2)
    assert rel(om1, r1) < tol and rel(om2, r2.reshape(d.M, d.M)) < tol
    c1, c2 = gen_vectors(2, O, V, d.M, seed=13)
    sig = P.jacobian_transform(np.stack([full_vec(c1[i], c2[i]) for i in range(2)]))
    for i in range(2):
        s1, s2 = om.jacobian_transform(OP, t1, x2, c1[i], c2[i].reshape(v, o, v, o))
        assert rel(sig[i], full_vec(s1, s2)) < tol
    P.close()
