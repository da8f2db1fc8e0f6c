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
    (200, 130, 64, 3, 2, "k", "k"),       # batched and batch-reduced, both k-contiguous
    (64, 64, 4096, 1, 1, "k", "k"),       # long reduction -> split, both k-contiguous
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


# per-element error bound, in units of sqrt(K*R) + 1 (unit-variance inputs):
# FP32 rounding, and for split BF16 products the ~2^-16 error of hi*hi +
# hi*lo + lo*hi
TOL = {"fp64": 1e-13, "fp32": 3e-6, "bf16x3": 4e-5}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
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

    def run(p):
        Cd = torch.tensor(C0, dtype=dt, device="cuda")
        ctx.gemm(mlcc.PREC[p], M, N, K, R, Z, 0.7, Ad, sA, Bd, sB, -0.3, Cd, [N, 1, M * N])
        return Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)

    got = run(prec)
    scale = np.sqrt(K * R) * 1.0 + 1.0
    assert np.abs(got - ref).max() <= TOL[prec] * scale, np.abs(got - ref).max()
    if prec == "bf16x3" and al == "k" and bl == "k" and K % 4 == 0 and K * R >= 64:
        # both operands k-contiguous: the split BF16 kernel ran, not FP32 MFMA
        assert np.abs(got - run("fp32")).max() > 0


def test_gemm_rejects_host_pointers(ctx):
    A = np.zeros(4)
    with pytest.raises(mlcc.MlccError):
        ctx.gemm(mlcc.FP64, 2, 2, 1, 1, 1, 1.0, A, [1, 1, 0, 0], A, [1, 1, 0, 0], 0.0, A,
                 [2, 1, 0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gemm_two_level_indices(ctx, prec):
    """Rows (A, C) and columns (B, C) split as (hi, lo) with independent
    strides, as used to push a batch of trial vectors through one launch."""
    rng = np.random.default_rng(7)
    Mh, Ml, K, Nh, Nl, R = 3, 37, 29, 4, 21, 5
    M, N = Mh * Ml, Nh * Nl
    # A element (m=(mh,ml), k) at r*sAr + mh*1000 + ml*K + k
    sAr, sA_hi = 4000, 1000
    A = rng.standard_normal(R * sAr)
    # B element (k, n=(nh,nl)) at r*sBr + k*Nl + nh*700 + nl
    sBr, sB_hi = 3000, 700
    B = rng.standard_normal(R * sBr)
    # C element (m, n) at mh*15000 + ml*400 + nh*100 + nl  (no overlaps)
    sC_hi_m, sC_hi_n, ldc = 15000, 100, 400
    C0 = rng.standard_normal(Mh * sC_hi_m)
    ref = C0.copy()
    for mh in range(Mh):
        for ml in range(Ml):
            for nh in range(Nh):
                for nl in range(Nl):
                    s = 0.0
                    for r in range(R):
                        a = A[r * sAr + mh * sA_hi + ml * K + np.arange(K)]
                        b = B[r * sBr + np.arange(K) * Nl + nh * sB_hi + nl]
                        s += a @ b
                    off = mh * sC_hi_m + ml * ldc + nh * sC_hi_n + nl
                    ref[off] = 1.5 * s + 0.5 * C0[off]
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = torch.tensor(A, dtype=dt, device="cuda")
    Bd = torch.tensor(B, dtype=dt, device="cuda")
    Cd = torch.tensor(C0, dtype=dt, device="cuda")
    import ctypes as C
    lib = ctx.lib
    # the binding's gemm has no two-level arguments: exercise them through the
    # debug entry point
    torch.cuda.synchronize()  # the uploads above run on torch's stream
    st = lib.mlcc_gemm2(ctx.h, mlcc.PREC[prec], M, N, K, R, 1, 1.5, C.c_void_p(Ad.data_ptr()),
                        (C.c_int64 * 4)(K, 1, sAr, 0), C.c_void_p(Bd.data_ptr()),
                        (C.c_int64 * 4)(Nl, 1, sBr, 0), 0.5, C.c_void_p(Cd.data_ptr()),
                        (C.c_int64 * 3)(ldc, 1, 0),
                        (C.c_int64 * 6)(Ml, sA_hi, sC_hi_m, Nl, sB_hi, sC_hi_n))
    assert st == 0, ctx.last_error()
    got = Cd.cpu().numpy().astype(np.float64)
    tol = 1e-12 if prec == "fp64" else 3e-5
    assert np.abs(got - ref).max() < tol * 10


MISALIGNED = [
    # M, N, K, R, A-layout, B-layout, element offset of A and B
    (70, 45, 37, 3, "k", "n", 1),
    (70, 45, 37, 3, "m", "k", 1),
    (37, 61, 43, 2, "m", "n", 0),   # ragged m-contiguous and n-contiguous tiles
    (129, 97, 30, 2, "k", "k", 0),  # K not a multiple of the vector width
    (161, 161, 64, 1, "m", "k", 3),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("case", MISALIGNED)
def test_gemm_vector_fallbacks(ctx, prec, case):
    """Operands whose base, stride or extent rule out 16-byte loads take the
    element-wise path; results must not depend on which path ran."""
    M, N, K, R, al, bl, shift = case
    rng = np.random.default_rng(abs(hash(case)) % 2**32)
    sAm, sAk = (K, 1) if al == "k" else (1, M)
    sBk, sBn = (N, 1) if bl == "n" else (1, K)
    sA = [sAm, sAk, M * K, 0]
    sB = [sBk, sBn, K * N, 0]
    A = rng.standard_normal(M * K * R + shift)
    B = rng.standard_normal(K * N * R + shift)
    ref = ref_gemm(A[shift:], sA, B[shift:], sB, M, N, K, R, 1)[0]
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = torch.tensor(A, dtype=dt, device="cuda")[shift:]
    Bd = torch.tensor(B, dtype=dt, device="cuda")[shift:]
    Cd = torch.zeros(M * N, dtype=dt, device="cuda")
    ctx.gemm(mlcc.PREC[prec], M, N, K, R, 1, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, 0])
    got = Cd.cpu().numpy().astype(np.float64).reshape(M, N)
    assert np.abs(got - ref).max() <= TOL[prec] * (np.sqrt(K * R) + 1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ml", [37, 16])
def test_gemm_two_level_contiguous_rows(ctx, prec, ml):
    """m-contiguous A with a two-level row index whose low extent is (37) or
    is not (16) cut by the 16-byte load units."""
    import ctypes as C
    rng = np.random.default_rng(11 + ml)
    Mh, K, N, R = 5, 23, 40, 3
    M = Mh * ml
    sA_hi, sAk, sAr = 64, 400, 400 * K   # A (m=(mh,ml), k) at r*sAr + k*sAk + mh*64 + ml
    A = rng.standard_normal(R * sAr)
    B = rng.standard_normal(R * K * N)
    ref = np.zeros((M, N))
    for r in range(R):
        idx = (r * sAr + np.arange(K)[None, :] * sAk
               + (np.arange(M) // ml)[:, None] * sA_hi + (np.arange(M) % ml)[:, None])
        ref += A[idx] @ B[r * K * N:(r + 1) * K * N].reshape(K, N)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Ad = torch.tensor(A, dtype=dt, device="cuda")
    Bd = torch.tensor(B, dtype=dt, device="cuda")
    Cd = torch.zeros(M * N, dtype=dt, device="cuda")
    torch.cuda.synchronize()  # the uploads above run on torch's stream
    st = ctx.lib.mlcc_gemm2(ctx.h, mlcc.PREC[prec], M, N, K, R, 1, 1.0, C.c_void_p(Ad.data_ptr()),
                            (C.c_int64 * 4)(1, sAk, sAr, 0), C.c_void_p(Bd.data_ptr()),
                            (C.c_int64 * 4)(N, 1, K * N, 0), 0.0, C.c_void_p(Cd.data_ptr()),
                            (C.c_int64 * 3)(N, 1, 0), (C.c_int64 * 6)(ml, sA_hi, ml * N, 0, 0, 0))
    assert st == 0, ctx.last_error()
    got = Cd.cpu().numpy().astype(np.float64).reshape(M, N)
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.abs(got - ref).max() <= tol * (np.sqrt(K * R) + 1.0)


# the engine's tile menus: vector-only kernel, general (element-wise) kernel,
# split BF16 kernel
VONLY_TILES = [(128, 128), (128, 96), (96, 128), (128, 64), (64, 128), (96, 96), (96, 64),
               (64, 96), (64, 64), (128, 32), (32, 128), (96, 32), (32, 96), (64, 32), (32, 64),
               (32, 32), (96, 160), (160, 96), (64, 160), (160, 64), (32, 160), (160, 32)]
GENERAL_TILES = [(128, 128), (128, 64), (64, 128), (64, 64), (128, 32), (32, 128), (64, 32),
                 (32, 64), (32, 32), (96, 160)]
SPLIT_TILES = [(128, 128), (128, 96), (96, 128), (128, 64), (64, 128), (96, 96), (64, 64),
               (128, 32), (32, 128), (64, 32), (32, 64), (32, 32), (96, 160), (160, 96)]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("vector", [True, False])
def test_every_tile(ctx, prec, vector):
    """Each tile of the menus, forced, on every operand layout: ragged edges
    in m, n (and k for the general kernel), a batch-reduced reduction split
    over blocks.  In FP64 this covers both rotation sides of the 4x4x4
    products (A rotated when a wave has fewer A than B fragments)."""
    M, N, K, R = (204, 188, 76, 2) if vector else (203, 187, 77, 2)
    rng = np.random.default_rng(5 if vector else 6)
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = rng.standard_normal(M * K * R)
    B = rng.standard_normal(K * N * R)
    layouts = [("k", "k"), ("k", "n"), ("m", "k"), ("m", "n")]
    if prec == "bf16x3":
        layouts = [("k", "k")]
        menu = SPLIT_TILES if vector else GENERAL_TILES
    else:
        menu = VONLY_TILES if vector else GENERAL_TILES
    applied = set()
    try:
        for al, bl in layouts:
            sAm, sAk = (K, 1) if al == "k" else (1, M)
            sBk, sBn = (N, 1) if bl == "n" else (1, K)
            sA = [sAm, sAk, M * K, 0]
            sB = [sBk, sBn, K * N, 0]
            ref = ref_gemm(A, sA, B, sB, M, N, K, R, 1)[0]
            Ad = torch.tensor(A, dtype=dt, device="cuda")
            Bd = torch.tensor(B, dtype=dt, device="cuda")
            for bm, bn in menu:
                ctx.gemm_tile(bm, bn)
                Cd = torch.zeros(M * N, dtype=dt, device="cuda")
                ctx.gemm(mlcc.PREC[prec], M, N, K, R, 1, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, 0])
                used = ctx.gemm_tile(bm, bn)
                if used == (bm, bn):
                    applied.add(used)
                got = Cd.cpu().numpy().astype(np.float64).reshape(M, N)
                err = np.abs(got - ref).max()
                assert err <= TOL[prec] * (np.sqrt(K * R) + 1.0), (al, bl, bm, bn, used, err)
    finally:
        ctx.gemm_tile(0, 0)
    assert applied == set(menu), sorted(set(menu) - applied)


def bf16_round(x):
    """float32 values rounded to BF16 (nearest, ties to even), as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("case", [c for c in CASES if c[5] == "k" and c[6] == "k"])
def test_plain_bf16_product(case):
    """MLCC_BF16 with the engine's own calls ("gemm") on the plain-BF16 map:
    the product of the operands rounded to BF16 (exact in FP32) accumulated
    in FP32; with an empty map the same call is bit-identical to split BF16."""
    M, N, K, R, Z, _, _ = case
    ctx = mlcc.Context(0)  # the map belongs to the context
    rng = np.random.default_rng(hash(case) % 2**32)
    sA = [K, 1, M * K, M * K * R]
    sB = [1, K, K * N, K * N * R]
    A = rng.standard_normal(M * K * R * Z).astype(np.float32)
    B = rng.standard_normal(K * N * R * Z).astype(np.float32)
    ref = ref_gemm(bf16_round(A), sA, bf16_round(B), sB, M, N, K, R, Z)
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")

    def run(p):
        Cd = torch.zeros(Z * M * N, dtype=torch.float32, device="cuda")
        ctx.gemm(mlcc.PREC[p], M, N, K, R, Z, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, M * N])
        return Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)

    ctx.bf16_map(["gemm"])
    got = run("bf16")
    assert np.abs(got - ref).max() <= TOL["fp32"] * (np.sqrt(K * R) + 1.0)
    split = run("bf16x3")
    assert np.abs(got - split).max() > 0  # one product, not three
    ctx.bf16_map([])
    assert np.array_equal(run("bf16"), split)
    ctx.close()
