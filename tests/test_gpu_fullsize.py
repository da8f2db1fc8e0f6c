"""Parity at the full benchmark sizes (CC2 5/20/60, MLCC2 40/400/1200 with
15/150 active, MLCCSD 60/600/2000 with 12/120 CCSD): ground-state energies and
excitation energies against oracle reference values written by
tests/golden/make_reference.py (FP64 oracle, same seeded inputs, seeds 0-2), and a batch
of four Jacobian transformations at 40/400/1200 against the oracle computed
here, element by element.

Bars: FP64 1e-10 Eh; FP32 and split-BF16 (mixed) 1e-6 Eh for energies and
1e-5 eV (3.67e-7 Eh) for excitation energies."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import mlcc as om  # noqa: E402
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import CONFIGS, gen_amplitudes, gen_inputs, gen_vectors  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EV = 27.211386245988  # Hartree in eV (CODATA 2018)
TOL = {"fp64": dict(e=1e-10, w=1e-10, gs=1e-10, es=1e-8),
       "fp32": dict(e=1e-6, w=1e-5 / EV, gs=1e-6, es=1e-6),
       "bf16x3": dict(e=1e-6, w=1e-5 / EV, gs=1e-6, es=1e-6),
       "bf16": dict(e=1e-6, w=1e-5 / EV, gs=1e-6, es=1e-6)}


SEEDS = [0, 1, 2]


def reference(name, seed=0):
    suffix = "" if seed == 0 else f"_seed{seed}"
    with open(os.path.join(GOLDEN, f"reference_{name}{suffix}.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


_inputs = {}


def inputs(name, seed=0):
    if (name, seed) not in _inputs:
        _inputs.clear()  # one workload's inputs at a time
        inp = gen_inputs(seed=seed, **CONFIGS[name])
        # the stored values belong to exactly these inputs
        assert inp.digest() == reference(name, seed)["inputs_sha256_16"]
        _inputs[(name, seed)] = inp
    return _inputs[(name, seed)]


def solve(ctx, name, precision, effective=False, seed=0):
    ref = reference(name, seed)
    c = CONFIGS[name]
    inp = inputs(name, seed)
    P = mlcc.Problem(ctx, inp.L, inp.eps, c["n_occ"], c["n_vir"], c["n_occ_act"], c["n_vir_act"],
                     model=ref["model"], precision=precision)
    t = TOL[precision]
    gs = P.ground_state(tol=t["gs"])
    dav = P.davidson(len(ref["omega"]), tol=t["es"], effective=effective)
    P.close()
    return ref, gs, dav


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("name", ["cc2_5_20_60", "mlcc2_40_400_1200", "mlccsd_60_600_2000"])
def test_energies_and_roots(ctx, name, precision, seed):
    ref, gs, dav = solve(ctx, name, precision, seed=seed)
    t = TOL[precision]
    assert gs["converged"] and dav["converged"]
    print(f"{name} seed {seed} {precision}: dE={gs['energy'] - ref['e_corr']:.2e} "
          f"dw={np.abs(np.array(dav['omega']) - ref['omega']).max():.2e}")
    assert abs(gs["energy"] - ref["e_corr"]) < t["e"]
    assert np.abs(np.array(dav["omega"]) - ref["omega"]).max() < t["w"]


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("name", ["mlcc2_40_400_1200", "mlccsd_60_600_2000"])
def test_bf16_map_energies_and_roots(ctx, name, seed):
    """MLCC_BF16 with the built-in plain-BF16 map on the two workloads the map
    was chosen on: energies and roots within the mixed-precision bars.  (The
    strongly correlated fully active 5/20/60 system is not covered: with its
    Cholesky vectors in BF16 it misses the bar.)"""
    ref, gs, dav = solve(ctx, name, "bf16", seed=seed)
    t = TOL["bf16"]
    assert gs["converged"] and dav["converged"]
    print(f"{name} seed {seed} bf16: dE={gs['energy'] - ref['e_corr']:.2e} "
          f"dw={np.abs(np.array(dav['omega']) - ref['omega']).max():.2e}")
    assert abs(gs["energy"] - ref["e_corr"]) < t["e"]
    assert np.abs(np.array(dav["omega"]) - ref["omega"]).max() < t["w"]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_effective_singles_roots(ctx, precision):
    """The effective-singles solver (used by the serving loop) reaches the
    full-space oracle roots."""
    ref, gs, dav = solve(ctx, "mlcc2_40_400_1200", precision, effective=True)
    t = TOL[precision]
    assert dav["converged"]
    assert np.abs(np.array(dav["omega"]) - ref["omega"]).max() < max(t["w"], 1e-9)


_jac_ref = {}


def _fullsize_jacobian_case():
    """Inputs, amplitudes, trial vectors and the oracle's complex-step
    transformation of each of the four vectors (computed once)."""
    if not _jac_ref:
        name = "mlcc2_40_400_1200"
        c = CONFIGS[name]
        inp = inputs(name)
        d = om.Dims(c["n_occ"], c["n_vir"], c["n_occ_act"], c["n_vir_act"])
        t1, x2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=1, scale1=0.01, scale2=0.001)
        c1, c2 = gen_vectors(4, d.O, d.V, d.M, seed=2)
        OP = om.Problem(inp.L, inp.eps, d, "mlcc2")
        refs = [om.jacobian_transform(OP, t1, x2, c1[i], c2[i].reshape(d.v, d.o, d.v, d.o))
                for i in range(4)]
        _jac_ref.update(inp=inp, d=d, t1=t1, x2=x2, c1=c1, c2=c2, refs=refs)
    return _jac_ref


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_jacobian_transform_fullsize(ctx, precision):
    """The four trial vectors at 40/400/1200 (active 15/150) through the
    launch configuration the benchmark times (one batch of 4), element by
    element against the oracle's complex-step transformation of each vector:
    max |error| over the singles and over the doubles block, each relative to
    that block's largest reference element.  Bar: FP64 1e-11; mixed
    precisions tol_chain over the longest reduction (the 2250 pairs) and six
    chained contractions."""
    from gpu_util import bar
    case = _fullsize_jacobian_case()
    inp, d = case["inp"], case["d"]
    P = mlcc.Problem(ctx, inp.L, inp.eps, d.O, d.V, d.o, d.v, precision=precision)
    P.set_amplitudes(case["t1"], case["x2"].reshape(d.M, d.M))
    cvec = np.concatenate([case["c1"].reshape(4, -1), case["c2"].reshape(4, -1)], axis=1)
    sig = P.jacobian_transform(cvec)
    P.close()
    tol = bar(precision, max(inp.n_chol, d.M), 6)
    n1 = d.V * d.O
    for i, (r1, r2) in enumerate(case["refs"]):
        e1 = np.abs(sig[i][:n1] - r1.ravel()).max() / np.abs(r1).max()
        e2 = np.abs(sig[i][n1:] - r2.ravel()).max() / np.abs(r2).max()
        print(f"{precision} vector {i}: singles {e1:.2e} doubles {e2:.2e} (bar {tol:.1e})")
        assert e1 < tol and e2 < tol
