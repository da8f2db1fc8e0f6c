"""The descriptor flags MLCC_INPUT_ON_DEVICE and MLCC_DETERMINISTIC: inputs
stated to be device memory give the same bits as the same inputs from the
host and are checked; repeated runs give bitwise equal residuals,
transformations, ground states and roots, with and without the flag, also
on packed BF16 planes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2006_05226_amd import mlcc  # noqa: E402
from paper_2006_05226_amd.synth import gen_amplitudes, gen_inputs, gen_vectors  # noqa: E402

from gpu_util import full_vec  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


def _run(P, d_o, d_v, O, V, seed):
    """Residual and a two-vector transformation at fixed amplitudes."""
    M = d_o * d_v
    t1, x2 = gen_amplitudes(O, V, d_o, d_v, seed=seed, scale1=0.05, scale2=0.02)
    P.set_amplitudes(t1, x2.reshape(M, M))
    om1, om2, _, e = P.residual()
    c1, c2 = gen_vectors(2, O, V, M, seed=seed + 1)
    sig = P.jacobian_transform(np.stack([full_vec(c1[i], c2[i]) for i in range(2)]))
    return om1, om2, e, sig


@pytest.mark.parametrize("model,precision", [("mlcc2", "fp64"), ("mlccsd", "bf16x3")])
def test_device_inputs_equal_host_inputs(ctx, model, precision):
    O, V, J, o, v = 9, 61, 130, 4, 22
    inp = gen_inputs(O, V, J, o, v, seed=21)
    fock = np.diag(inp.eps)
    P_host = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model=model, precision=precision,
                          fock=fock)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (inp.L, inp.eps, fock)]
    P_dev = mlcc.Problem(ctx, dev[0], dev[1], O, V, o, v, model=model, precision=precision,
                         fock=dev[2], flags=mlcc.INPUT_ON_DEVICE)
    a = _run(P_host, o, v, O, V, seed=22)
    b = _run(P_dev, o, v, O, V, seed=22)
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_device_flag_rejects_host_memory(ctx):
    O, V, J, o, v = 5, 23, 40, 2, 8
    inp = gen_inputs(O, V, J, o, v, seed=3)
    L_d = torch.from_numpy(inp.L).cuda()
    eps_d = torch.from_numpy(inp.eps).cuda()
    cases = [(inp.L, eps_d, None), (L_d, inp.eps, None), (L_d, eps_d, np.diag(inp.eps))]
    for L, eps, fock in cases:
        with pytest.raises(mlcc.MlccError) as e:
            mlcc.Problem(ctx, L, eps, O, V, o, v, fock=fock, flags=mlcc.INPUT_ON_DEVICE)
        assert e.value.status == mlcc.E_ARG
        assert "MLCC_INPUT_ON_DEVICE" in str(e.value)
    # synthetic L is not read: only eps has to be device memory
    P = mlcc.Problem(ctx, None, eps_d, O, V, o, v, n_chol=J, seed=5,
                     flags=mlcc.INPUT_ON_DEVICE)
    assert P.ground_state(tol=1e-8)["converged"]
    with pytest.raises(mlcc.MlccError):
        mlcc.Problem(ctx, None, inp.eps, O, V, o, v, n_chol=J, seed=5, flags=mlcc.INPUT_ON_DEVICE)
    with pytest.raises(mlcc.MlccError):
        mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, flags=8)  # no such flag


def test_served_device_inputs_equal_problem(ctx):
    """A request whose inputs are device memory (flag set) is copied at
    submission and solves to the bits of the same problem run directly."""
    O, V, J, o, v = 8, 80, 240, 3, 30
    inp = gen_inputs(O, V, J, o, v, seed=31)
    P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, precision="fp32")
    g = P.ground_state(tol=1e-8)
    w = P.davidson(3, tol=1e-7, effective=True)["omega"]
    L_d = torch.from_numpy(inp.L).cuda()
    eps_d = torch.from_numpy(inp.eps).cuda()
    srv = mlcc.Server(ctx, max_slots=2)
    d, keep = mlcc.Server.desc(L_d, eps_d, O, V, o, v, precision="fp32")
    d.flags |= mlcc.INPUT_ON_DEVICE
    r = srv.wait(srv.submit(d, 3, gs_tol=1e-8, es_tol=1e-7))
    eps_h = np.ascontiguousarray(inp.eps)
    d.eps = eps_h.ctypes.data  # a host pointer under the flag: rejected
    with pytest.raises(mlcc.MlccError) as e:
        srv.submit(d, 3)
    assert e.value.status == mlcc.E_ARG
    srv.close()
    assert r["status"] == mlcc.OK
    assert r["e_corr"] == g["energy"]
    assert np.array_equal(np.array(r["omega"][:3]), w)


@pytest.mark.parametrize("precision,planes", [("fp64", 0), ("bf16x3", 1), ("bf16", 1)])
def test_repeat_runs_are_bitwise_equal(ctx, precision, planes):
    """Two problems built from the same inputs, one with MLCC_DETERMINISTIC,
    and a repeated call on one of them give the same bits; planes=1 forces
    the packed-plane BF16 products (split-K sums included where chosen)."""
    O, V, J, o, v = 12, 150, 400, 6, 60
    inp = gen_inputs(O, V, J, o, v, seed=41)
    ctx.gemm_planes(planes)
    try:
        runs = []
        for flags in (0, mlcc.DETERMINISTIC):
            P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, precision=precision, flags=flags)
            a = _run(P, o, v, O, V, seed=42)
            b = _run(P, o, v, O, V, seed=42)
            for x, y in zip(a, b):
                assert np.array_equal(np.asarray(x), np.asarray(y))
            g = P.ground_state(tol=1e-6 if precision == "bf16" else 1e-8)
            w = P.davidson(3, tol=1e-6, effective=True)["omega"]
            runs.append((a, g["energy"], g["t1"], np.array(w)))
        (a0, e0, t0, w0), (a1, e1, t1, w1) = runs
        for x, y in zip(a0, a1):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert e0 == e1 and np.array_equal(t0, t1) and np.array_equal(w0, w1)
    finally:
        ctx.gemm_planes(0)
