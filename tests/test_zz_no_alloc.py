"""mlcc_gemm_noalloc (the engine for callers that cannot allocate) against
mlcc_gemm2 on the same operands, through the C ABI: two calls in a row, the
second smaller; a product whose split partial sums would not fit the fixed
array; no device bytes charged to the context by the no-allocation calls."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2006_05226_amd import mlcc  # noqa: E402

pytestmark = pytest.mark.gpu

# unit roundoff of the accumulator
U = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}


def split_order_bound(prec, KR):
    """Largest element difference expected between two evaluations of one
    product that differ only in how the reduction is split, for unit-variance
    operands: an unsplit chain of KR accumulations into partial sums of size
    ~sqrt(k) has a rounding error of rms ~ u KR / sqrt(2); the difference of
    two such errors has rms <= u KR, and the largest of ~1e6 outputs stays
    within 6 of those."""
    return 6.0 * U[prec] * KR


def operands(M, N, K, R, dt, seed):
    rng = np.random.default_rng(seed)
    A = torch.tensor(rng.standard_normal(R * M * K), dtype=dt, device="cuda")
    B = torch.tensor(rng.standard_normal(R * K * N), dtype=dt, device="cuda")
    C0 = torch.tensor(rng.standard_normal(M * N), dtype=dt, device="cuda")
    # A [r][m][k] (k contiguous), B [r][n][k] (k contiguous): split-BF16 eligible
    return A, [K, 1, M * K, 0], B, [1, K, K * N, 0], C0, [N, 1, 0]


def run_both(ctx, prec, M, N, K, R, seed):
    dt = torch.float64 if prec == "fp64" else torch.float32
    A, sA, B, sB, C0, sC = operands(M, N, K, R, dt, seed)
    c_ref = C0.clone()
    ctx.gemm(mlcc.PREC[prec], M, N, K, R, 1, 0.9, A, sA, B, sB, -0.4, c_ref, sC)
    torch.cuda.synchronize()
    before = ctx.bytes()
    c_na = C0.clone()
    ctx.gemm_noalloc(mlcc.PREC[prec], M, N, K, R, 1, 0.9, A, sA, B, sB, -0.4, c_na, sC)
    torch.cuda.synchronize()
    assert ctx.bytes() == before, "the no-allocation call charged device memory"
    return c_ref.cpu().numpy().astype(np.float64), c_na.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_noalloc_equals_engine_twice(prec):
    ctx = mlcc.Context(0)
    # long reductions (split over workgroups, partial sums in the fixed
    # array), then a smaller product that reuses the array's stale contents
    for (M, N, K, R), seed in (((96, 80, 4096, 2), 1), ((40, 24, 1000, 3), 2)):
        print(f"noalloc {prec} M={M} N={N} K={K} R={R}", flush=True)
        ref, got = run_both(ctx, prec, M, N, K, R, seed)
        # partial sums fit the array: same split count and tile, same bits
        assert np.array_equal(ref, got), np.abs(ref - got).max()
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_caps_splits_to_the_array(prec):
    """A wide output with a long reduction: two splits of its partial sums
    (2 x 1100^2 x 8 bytes in FP64) or four (FP32) need more than the array
    holds, so the no-allocation call runs with fewer splits than the engine
    may choose; the two results agree to the products' rounding."""
    ctx = mlcc.Context(0)
    M, N, K, R = 1100, 1100, 16384, 1
    print(f"noalloc cap {prec} M={M} N={N} K={K}", flush=True)
    ref, got = run_both(ctx, prec, M, N, K, R, 3)
    assert np.abs(ref - got).max() < split_order_bound(prec, K * R)
    # and a smaller call after it
    print(f"noalloc cap {prec} second call", flush=True)
    ref, got = run_both(ctx, prec, 64, 64, 4096, 1, 4)
    assert np.array_equal(ref, got)
    ctx.close()


def test_noalloc_argument_errors():
    ctx = mlcc.Context(0)
    x = np.zeros(4)
    with pytest.raises(mlcc.MlccError):   # host pointers are refused
        ctx.gemm_noalloc(mlcc.FP64, 2, 2, 1, 1, 1, 1.0, x, [1, 1, 0, 0], x, [1, 1, 0, 0], 0.0, x,
                         [2, 1, 0])
    ctx.close()
