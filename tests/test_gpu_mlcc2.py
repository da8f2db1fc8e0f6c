"""MLCC2 / CCS on the GPU (through the C ABI) against the FP64 oracle on the
same seeded inputs: X1 basis, Fock matrix, Omega vector, energy, ground state,
Jacobian transformation, Davidson roots; error paths of the ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import mlcc as om  # noqa: E402
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import CONFIGS, gen_amplitudes, gen_inputs, gen_vectors  # noqa: E402

from gpu_util import bar, full_vec, make, rel  # noqa: E402

pytestmark = pytest.mark.gpu

# several MFMA tiles with ragged tails: M = 125 pairs, n = 48, J = 100
SMALL = dict(O=8, V=40, J=100, o=5, v=25)
K_SMALL = 125  # longest reduction (the pair count)


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


def small(ctx, model="mlcc2", precision="fp64", seed=0, **kw):
    s = dict(SMALL)
    s.update(kw)
    return make(s["O"], s["V"], s["J"], s["o"], s["v"], seed=seed, model=model,
                precision=precision, ctx=ctx)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_x1_basis_and_fock(ctx, precision):
    tol = bar(precision, K_SMALL, 2, fp64=1e-12)
    inp, _, P, OP, d = small(ctx, precision=precision)
    t1, s = gen_amplitudes(d.O, d.V, d.o, d.v, seed=1, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, s.reshape(d.M, d.M))
    P.residual()
    D = om.dress(inp.L, inp.eps, d, t1)
    Lt = P.debug_get(1)
    assert rel(Lt, D.Lt) < tol
    Ft = P.debug_get(0)
    # the residual evaluates the F~ blocks it needs: AI and active jb
    assert rel(Ft[d.vir, d.occ], D.Ft[d.vir, d.occ]) < tol
    assert rel(Ft[d.aocc, d.avir], D.Ft[d.aocc, d.avir]) < tol
    g = P.debug_get(2)
    assert rel(g, om.g_aibj(D.Lt, d).reshape(d.M, d.M)) < tol


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_residual_independent_s(ctx, precision):
    tol = bar(precision, K_SMALL, 4, fp64=1e-12)
    inp, _, P, OP, d = small(ctx, precision=precision)
    t1, s = gen_amplitudes(d.O, d.V, d.o, d.v, seed=2, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, s.reshape(d.M, d.M))
    om1, om2, x2, e = P.residual()
    r1, r2 = OP.omega(t1, s)
    assert rel(om1, r1) < tol
    assert rel(om2, r2.reshape(d.M, d.M)) < tol
    assert np.array_equal(x2, s.reshape(d.M, d.M))
    assert abs(e - OP.energy(t1, s)) < tol * abs(OP.energy(t1, s)) + 1e-15


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_residual_analytic_s(ctx, precision):
    tol = bar(precision, K_SMALL, 4, fp64=1e-12)
    inp, _, P, OP, d = small(ctx, precision=precision)
    t1, _ = gen_amplitudes(d.O, d.V, d.o, d.v, seed=3, scale1=0.05)
    P.set_amplitudes(t1)
    om1, om2, x2, e = P.residual()
    s = OP.s_analytic(t1)
    assert rel(x2, s.reshape(d.M, d.M)) < tol
    r1, _ = OP.omega(t1, s)
    assert rel(om1, r1) < tol
    assert np.abs(om2).max() < 1e-12 * np.abs(s).max() * 10  # analytic s solves Omega_2
    assert abs(e - OP.energy(t1, s)) < tol * abs(OP.energy(t1, s))


def test_first_iteration_energy_is_mp2(ctx):
    inp, _, P, OP, d = small(ctx)
    r = P.ground_state(tol=1e-10, max_iter=1)
    assert r["status"] == mlcc.E_NOCONV
    assert abs(r["energy"] - om.mp2_energy(inp.L, inp.eps, d)) < 1e-12


@pytest.mark.parametrize("cfg", ["cc2_5_20_60"])
def test_ground_state_c1(ctx, cfg):
    c = CONFIGS[cfg]
    inp = gen_inputs(seed=0, **c)
    d = om.Dims(c["n_occ"], c["n_vir"], c["n_occ_act"], c["n_vir_act"])
    ref = om.ground_state(om.Problem(inp.L, inp.eps, d, "mlcc2"), tol=1e-11)
    P = mlcc.Problem(ctx, inp.L, inp.eps, d.O, d.V, d.o, d.v, model="mlcc2")
    r = P.ground_state(tol=1e-11)
    assert r["converged"]
    assert abs(r["energy"] - ref["energy"]) < 1e-10
    assert np.abs(r["t1"] - ref["t1"]).max() < 1e-9


def test_ground_state_mlcc2_partial_active(ctx):
    inp, _, P, OP, d = small(ctx)
    ref = om.ground_state(OP, tol=1e-11)
    r = P.ground_state(tol=1e-11)
    assert r["converged"]
    assert abs(r["energy"] - ref["energy"]) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_jacobian_transform_parity(ctx, precision):
    tol = bar(precision, K_SMALL, 6)
    inp, _, P, OP, d = small(ctx, precision=precision)
    t1, s = gen_amplitudes(d.O, d.V, d.o, d.v, seed=4, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, s.reshape(d.M, d.M))
    c1, c2 = gen_vectors(3, d.O, d.V, d.M, seed=5)
    c = np.stack([full_vec(c1[i], c2[i]) for i in range(3)])
    sig = P.jacobian_transform(c)
    for i in range(3):
        r1, r2 = om.jacobian_transform(OP, t1, s, c1[i], c2[i].reshape(d.v, d.o, d.v, d.o))
        ref = full_vec(r1, r2)
        assert rel(sig[i][: d.V * d.O], r1.ravel()) < tol
        assert rel(sig[i], ref) < tol


def test_jacobian_transform_device_pointers(ctx):
    inp, _, P, OP, d = small(ctx)
    t1, s = gen_amplitudes(d.O, d.V, d.o, d.v, seed=4, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, s.reshape(d.M, d.M))
    c1, c2 = gen_vectors(2, d.O, d.V, d.M, seed=6)
    c = np.stack([full_vec(c1[i], c2[i]) for i in range(2)])
    host = P.jacobian_transform(c)
    dev = P.jacobian_transform(torch.tensor(c, device="cuda")).cpu().numpy()
    assert np.array_equal(host, dev)


def test_effective_transform_parity(ctx):
    """A11 c1 + A12 (w - eps)^-1 A21 c1 from the full-space oracle transform."""
    inp, _, P, OP, d = small(ctx)
    t1, s = gen_amplitudes(d.O, d.V, d.o, d.v, seed=7, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, s.reshape(d.M, d.M))
    c1, _ = gen_vectors(2, d.O, d.V, 0, seed=8)
    w = 0.37
    got = P.jacobian_transform_eff(w, c1.reshape(2, -1))
    D2 = om.orbital_denominators(inp.eps, d)
    for i in range(2):
        _, a21 = om.jacobian_transform(OP, t1, s, c1[i], np.zeros((d.v, d.o, d.v, d.o)))
        c2 = a21 / (w - D2)
        r1, _ = om.jacobian_transform(OP, t1, s, c1[i], c2)
        assert rel(got[i], r1.ravel()) < 1e-11


def test_davidson_matches_dense(ctx):
    inp, _, P, OP, d = make(4, 12, 30, 3, 8, seed=1, ctx=ctx)
    gs = om.ground_state(OP, tol=1e-12)
    r = P.ground_state(tol=1e-12)
    assert abs(r["energy"] - gs["energy"]) < 1e-11
    dav = P.davidson(4, tol=1e-9)
    assert dav["converged"]
    ev = om.dense_eigenvalues(om.jacobian_dense(OP, gs["t1"], gs["x2"]))
    assert np.abs(dav["omega"] - ev.real[:4]).max() < 1e-10


def test_davidson_effective_singles_matches_full(ctx):
    inp, _, P, OP, d = make(4, 12, 30, 3, 8, seed=2, ctx=ctx)
    P.ground_state(tol=1e-12)
    full = P.davidson(3, tol=1e-9)
    eff = P.davidson(3, tol=1e-9, effective=True)
    assert full["converged"] and eff["converged"]
    assert np.abs(full["omega"] - eff["omega"]).max() < 1e-8


def test_ccs_is_cis(ctx):
    inp, _, P, OP, d = make(5, 15, 40, 0, 0, seed=3, model="ccs", ctx=ctx)
    r = P.ground_state(tol=1e-12)
    assert r["converged"] and r["iterations"] == 1 and np.abs(r["t1"]).max() == 0.0
    dav = P.davidson(5, tol=1e-9)
    ref = np.linalg.eigvalsh(om.cis_matrix(inp.L, inp.eps, d))[:5]
    assert np.abs(dav["omega"] - ref).max() < 1e-10


# ---- error paths ----------------------------------------------------------------

def test_errors(ctx):
    inp = gen_inputs(3, 6, 10, 2, 3, seed=0)
    with pytest.raises(mlcc.MlccError) as e:
        mlcc.Problem(ctx, inp.L, inp.eps, 3, 6, 4, 3)
    assert e.value.status == mlcc.E_ARG
    bad = inp.eps.copy()
    bad[2] = np.nan
    with pytest.raises(mlcc.MlccError) as e:
        mlcc.Problem(ctx, inp.L, bad, 3, 6, 2, 3)
    assert e.value.status == mlcc.E_NUMERIC
    P = mlcc.Problem(ctx, inp.L, inp.eps, 3, 6, 2, 3)
    with pytest.raises(mlcc.MlccError) as e:
        P.residual()
    assert e.value.status == mlcc.E_STATE
    with pytest.raises(mlcc.MlccError) as e:
        P.davidson(2)
    assert e.value.status == mlcc.E_STATE
    small_budget = mlcc.Context(0, hbm_budget=1 << 10)
    with pytest.raises(mlcc.MlccError) as e:
        mlcc.Problem(small_budget, inp.L, inp.eps, 3, 6, 2, 3)
    assert e.value.status == mlcc.E_OOM
