"""Parity at the full 150/1200/3600 MLCC2 workload (active 50/500, Cholesky
vectors drawn on the device, the launch configuration bench.py times) against
oracle values at sampled elements (tests/golden/make_c4_samples.py, which
regenerates the needed blocks of the Cholesky vectors from the generator's
definition and evaluates oracle/sampled.py):

* g~_aibj at 1200 quadruples, from the analytic s2 (s = -g~ / eps) that the
  pair-blocked ground-state path writes,
* Omega_AI at 208 (A, I) over active and inactive orbitals,
* the effective transformation sigma_AI at the same (A, I) for two vectors.

FP64 element by element within 1e-11 of the largest sample; FP32 and
split-BF16 within the bound of gpu_util.tol_chain for reductions of M terms."""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import CONFIGS, device_cholesky_block, gen_eps  # noqa: E402

from gpu_util import tol_chain  # noqa: E402

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "c4_samples_mlcc2_150_1200_3600.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def dense(entry, V, O):
    a = np.zeros((V, O))
    a[np.ix_(entry["rows"], entry["cols"])] = np.asarray(entry["values"]).reshape(
        len(entry["rows"]), len(entry["cols"]))
    return a


def test_golden_inputs_match_generator(gold):
    """The stored values belong to these inputs: orbital energies and a probe
    block of the generated Cholesky vectors (CPU recomputation)."""
    c = CONFIGS[gold["config"]]
    O, V = c["n_occ"], c["n_vir"]
    eps = gen_eps(O, V, c["n_occ_act"], seed=gold["seed"])
    assert hashlib.sha256(eps.tobytes()).hexdigest()[:16] == gold["eps_sha256"]
    blk = device_cholesky_block([0, 1, 37, 3599], [0, 149, 150, 1349], [1, 77, 640, 1300], O, V,
                                gold["seed"])
    assert hashlib.sha256(np.ascontiguousarray(blk).tobytes()).hexdigest()[:16] == gold["probe_sha256"]


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_c4_sampled_parity(gold, precision):
    c = CONFIGS[gold["config"]]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    M = o * v
    eps = gen_eps(O, V, o, seed=gold["seed"])
    print(f"c4 parity {precision}: problem", flush=True)
    ctx = mlcc.Context(0)
    P = mlcc.Problem(ctx, None, eps, O, V, o, v, model="mlcc2", precision=precision, n_chol=J,
                     seed=gold["seed"])
    t1 = dense(gold["t1"], V, O)
    P.set_amplitudes(t1)
    x2 = torch.empty((M, M), dtype=torch.float64, device="cuda")
    print(f"c4 parity {precision}: residual", flush=True)
    om1, _, _, _ = P.residual(doubles=False, x2_out=x2)
    q = np.asarray(gold["quads"])
    ai = q[:, 0] * o + q[:, 1]
    bj = q[:, 2] * o + q[:, 3]
    s = x2.view(-1)[torch.tensor(ai * M + bj, device="cuda")].cpu().numpy()
    dai = eps[O:O + v][:, None] - eps[:o][None, :]
    g = -s * (dai[q[:, 0], q[:, 1]] + dai[q[:, 2], q[:, 3]])
    del x2
    torch.cuda.empty_cache()
    pairs = np.asarray(gold["pairs"])
    got_om = om1[pairs[:, 0], pairs[:, 1]]
    print(f"c4 parity {precision}: effective transform", flush=True)
    cv = np.stack([dense(e, V, O).ravel() for e in gold["c"]])
    sig = P.jacobian_transform_eff(gold["w"], cv)
    P.close()
    ctx.close()
    tol = 1e-11 if precision == "fp64" else tol_chain(precision, M)
    # errors relative to the scale of each quantity; the two trial vectors have
    # unit norm, so the transformation's scale is the larger of their samples
    sig_scale = max(np.abs(np.asarray(s)).max() for s in gold["sigma"])
    checks = [("g", g, np.asarray(gold["g"]), None),
              ("omega1", got_om, np.asarray(gold["omega1"]), None)]
    for k in range(len(gold["sigma"])):
        got = sig[k].reshape(V, O)[pairs[:, 0], pairs[:, 1]]
        checks.append((f"sigma{k}", got, np.asarray(gold["sigma"][k]), sig_scale))
    for name, got, ref, scale in checks:
        err = np.abs(got - ref).max() / (scale or np.abs(ref).max())
        print(f"c4 parity {precision} {name}: max |err| / max |ref| = {err:.2e} (tol {tol:.1e})",
              flush=True)
        assert err < tol, (name, err)
