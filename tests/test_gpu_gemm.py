"""GEMM engine (every Cholesky-index contraction runs on it) against a plain
NumPy reference: FP64 and FP32 MFMA, strided / batched / batch-reduced
operands, ragged edges, split reductions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2006_05226_amd import mlcc  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return mlcc.Context(0)


def ref_gemm(A, sA, B, sB, M, N, K, R, Z):
    out = np.zeros((Z, M, N))
    for z in range(Z):
        for r in range(R):
            ia = z * sA[3] + r * sA[2] + np.arange(M)[:, None] * sA[0] + np.arange(K)[None, :] * sA[1]
            ib = z * sB[3] + r * sB[2] + np.arange(K)[:, None] * sB[0] + np.arange(N)[None, :] * sB[1]
            out[z] += A[ia] @ B[ib]
    return out


CASES = [
    # M, N, K, R, Z, A-layout ('k' = k contiguous, 'm'), B-layout ('k', 'n')
    (1, 1, 1, 1, 1, "k", "n"),
    (37, 45, 19, 1, 1, "k", "n"),
    (130, 129, 70, 1, 1, "m", "n"),
    (300, 260, 200, 1, 1, "k", "k"),
    (64, 64, 64, 1, 1, "m", "k"),
    (17, 3, 5, 40, 1, "k", "n"),        # batch-reduce with tiny tiles -> split
    (40, 15, 150, 12, 1, "k", "n"),
    (33, 31, 9, 1, 7, "k", "n"),        # independent batches
    (5, 300, 2000, 1, 1, "k", "n"),     # long reduction -> split
    (1, 257, 333, 1, 3, "k", "n"),
    (256, 256, 256, 1, 1, "m", "n"),
    (513, 511, 97, 1, 1, "m", "n"),
]


def strides(layout, rows, cols):
    # element (r, c) of a rows x cols operand
    return (cols, 1) if layout in ("k",) else (1, rows)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES)
def test_gemm(ctx, prec, case):
    M, N, K, R, Z, al, bl = case
    rng = np.random.default_rng(hash(case) % 2**32)
    # A element (m, k): 'k' -> row-major [M][K], 'm' -> [K][M]
    sAm, sAk = (K, 1) if al == "k" else (1, M)
    sBk, sBn = (N, 1) if bl == "n" else (1, K)
    sA = [sAm, sAk, M * K, M * K * R]
    sB = [sBk, sBn, K * N, K * N * R]
    A = rng.standard_normal(M * K * R * Z)
    B = rng.standard_normal(K * N * R * Z)
    C0 = rng.standard_normal(Z * M * N)
    ref = 0.7 * ref_gemm(A, sA, B, sB, M, N, K, R, Z) - 0.3 * C0.reshape(Z, M, N)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = torch.tensor(A, dtype=dt, device="cuda")
    Bd = torch.tensor(B, dtype=dt, device="cuda")
    Cd = torch.tensor(C0, dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda")
    ctx.gemm(mlcc.PREC[prec], M, N, K, R, Z, 0.7, Ad, sA, Bd, sB, -0.3, Cd, [N, 1, M * N])
    got = Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)
    scale = np.sqrt(K * R) * 1.0 + 1.0
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.abs(got - ref).max() <= tol * scale, np.abs(got - ref).max()


def test_gemm_rejects_host_pointers(ctx):
    A = np.zeros(4)
    with pytest.raises(mlcc.MlccError):
        ctx.gemm(mlcc.FP64, 2, 2, 1, 1, 1, 1.0, A, [1, 1, 0, 0], A, [1, 1, 0, 0], 0.0, A,
                 [2, 1, 0])
