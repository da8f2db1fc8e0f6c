"""MLCCSD (CCS/CCSD) on the GPU through the C ABI against the FP64 oracle:
doubles residual, Jacobian transformation (both blocks), ground state,
Davidson roots, and the two-electron case against exact diagonalisation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import mlcc as om  # noqa: E402
from oracle.bruteforce import fci_two_electron  # noqa: E402
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import CONFIGS, gen_amplitudes, gen_inputs, gen_vectors  # noqa: E402

from gpu_util import bar, full_vec, make, rel  # noqa: E402

pytestmark = pytest.mark.gpu

# ragged multi-tile sizes: M = 7*11 = 77 pairs
SIZES = [dict(O=9, V=30, J=70, o=7, v=11), dict(O=4, V=13, J=40, o=3, v=5)]


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


@pytest.mark.parametrize("sz", SIZES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_residual_parity(ctx, sz, precision):
    # longest reduction: J, the pair count or the ladder's v^2
    tol = bar(precision, max(sz["J"], sz["o"] * sz["v"], sz["v"] ** 2), 8)
    inp, _, P, OP, d = make(sz["O"], sz["V"], sz["J"], sz["o"], sz["v"], seed=2, model="mlccsd",
                            precision=precision, ctx=ctx)
    t1, t2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=3, scale1=0.05, scale2=0.05)
    P.set_amplitudes(t1, t2.reshape(d.M, d.M))
    om1, om2, _, e = P.residual()
    r1, r2 = OP.omega(t1, t2)
    assert rel(om1, r1) < tol
    assert rel(om2, r2.reshape(d.M, d.M)) < tol
    assert abs(e - OP.energy(t1, t2)) < tol * abs(OP.energy(t1, t2))


@pytest.mark.parametrize("sz", SIZES)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_jacobian_parity(ctx, sz, precision):
    tol = bar(precision, max(sz["J"], sz["o"] * sz["v"], sz["v"] ** 2), 10, fp64=1e-10)
    inp, _, P, OP, d = make(sz["O"], sz["V"], sz["J"], sz["o"], sz["v"], seed=4, model="mlccsd",
                            precision=precision, ctx=ctx)
    t1, t2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=5, scale1=0.05, scale2=0.05)
    P.set_amplitudes(t1, t2.reshape(d.M, d.M))
    c1, c2 = gen_vectors(3, d.O, d.V, d.M, seed=6)
    c = np.stack([full_vec(c1[i], c2[i]) for i in range(3)])
    sig = P.jacobian_transform(c)
    for i in range(3):
        r1, r2 = om.jacobian_transform(OP, t1, t2, c1[i], c2[i].reshape(d.v, d.o, d.v, d.o))
        assert rel(sig[i][: P.n1], r1.ravel()) < tol
        assert rel(sig[i][P.n1:], r2.ravel()) < tol
    # pure singles and pure doubles directions separately
    e1 = np.concatenate([c1[0].ravel(), np.zeros(d.M * d.M)])[None]
    s = P.jacobian_transform(e1)[0]
    r1, r2 = om.jacobian_transform(OP, t1, t2, c1[0], np.zeros((d.v, d.o, d.v, d.o)))
    assert rel(s, full_vec(r1, r2)) < tol


def test_ground_state_and_roots(ctx):
    inp, _, P, OP, d = make(5, 14, 36, 3, 6, seed=7, model="mlccsd", ctx=ctx)
    ref = om.ground_state(OP, tol=1e-11)
    r = P.ground_state(tol=1e-11)
    assert r["converged"]
    assert abs(r["energy"] - ref["energy"]) < 1e-10
    dav = P.davidson(3, tol=1e-8)
    assert dav["converged"]
    ev = om.davidson(OP, ref["t1"], ref["x2"], 3, tol=1e-9)
    assert np.abs(dav["omega"] - ev["omega"]).max() < 1e-8


def test_two_electron_equals_fci(ctx):
    """Two electrons: CCSD energy = E_FCI - E_HF and the Davidson roots are FCI
    singlet excitation energies (the GPU path end to end)."""
    c = CONFIGS["ccsd_1_8_60"]
    inp = gen_inputs(seed=0, **c)
    d = om.Dims(1, 8, 1, 8)
    P = mlcc.Problem(ctx, inp.L, inp.eps, 1, 8, 1, 8, model="mlccsd")
    r = P.ground_state(tol=1e-12)
    h = om.core_hamiltonian(inp.L, inp.eps, d)
    w = fci_two_electron(h, om.eri(inp.L))
    assert abs(r["energy"] - (w[0] - om.hf_energy(inp.L, inp.eps, d))) < 1e-11
    dav = P.davidson(4, tol=1e-9)
    assert dav["converged"]
    assert np.abs(dav["omega"] - (w[1:5] - w[0])).max() < 1e-9
