"""Split and plain BF16 products on packed planes (the engine's path for large
BF16 products: both operands converted once into BF16 hi / lo planes, then a
kernel that streams them into LDS with direct loads), forced on small shapes
that span several tiles, ragged edges, batches, batch reductions and split
reductions.

References: the exact (FP64) sum of the BF16 products the method defines —
hi*hi + hi*lo + lo*hi for split products, hi*hi for plain ones, with
hi = bf16(x), lo = bf16(x - hi) rounded to nearest even — which the kernel
must reproduce up to FP32 accumulation; and the plain FP64 product, which
split products must reproduce to their ~2^-16 product error."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2006_05226_amd import mlcc  # noqa: E402

pytestmark = pytest.mark.gpu

# error bounds per unit of sqrt(K R) + 1 on unit-variance inputs (as the
# engine's other parity tests): FP32 accumulation, and split BF16 against
# the exact product
TOL_ACC = 3e-6
TOL_SPLIT = 4e-5


def bf16_round(x):
    """float32 values rounded to BF16 (nearest, ties to even), as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def split_planes(x):
    hi = bf16_round(x)
    lo = bf16_round(np.asarray(x, dtype=np.float32) - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


def batched(A, sA, B, sB, M, N, K, R, Z):
    out = np.zeros((Z, M, N))
    for z in range(Z):
        for r in range(R):
            ia = z * sA[3] + r * sA[2] + np.arange(M)[:, None] * sA[0] + np.arange(K)[None, :] * sA[1]
            ib = z * sB[3] + r * sB[2] + np.arange(K)[:, None] * sB[0] + np.arange(N)[None, :] * sB[1]
            out[z] += A[ia] @ B[ib]
    return out


def plane_bytes(M, N, K, R, Z, a_shared, planes):
    rup = lambda x, m: (x + m - 1) // m * m  # noqa: E731
    kp = rup(K * R, 64)
    za = 1 if a_shared else Z
    return planes * 2 * kp * (za * rup(M, 256) + Z * rup(N, 256))


# M, N, K, R, Z, A shared by the batches (K a multiple of 4: the split
# products' condition on operands outside library allocations)
CASES = [
    (1, 1, 4, 1, 1, False),
    (37, 45, 20, 1, 1, False),       # one ragged tile, K below one k-step
    (300, 260, 200, 1, 1, False),    # several tiles, ragged in m, n and k
    (200, 130, 64, 3, 2, False),     # batched and batch-reduced
    (517, 263, 100, 2, 3, True),     # A shared by the batches
    (64, 64, 4096, 1, 1, False),     # long reduction: split over blocks
    (5, 300, 2000, 1, 1, False),
]


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_planes_products(case, plain):
    M, N, K, R, Z, a_shared = case
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(abs(hash(case)) % 2**32)
    # A (m, k) at z*sAz + r*M*K + m*K + k; B (k, n) at z*K*N*R + r*K*N + n*K + k
    sA = [K, 1, M * K, 0 if a_shared else M * K * R]
    sB = [1, K, K * N, K * N * R]
    A = rng.standard_normal(M * K * R * (1 if a_shared else Z)).astype(np.float32)
    B = rng.standard_normal(K * N * R * Z).astype(np.float32)
    ah, al = split_planes(A)
    bh, bl = split_planes(B)
    if plain:
        ref = batched(ah, sA, bh, sB, M, N, K, R, Z)
    else:
        ref = (batched(ah, sA, bh, sB, M, N, K, R, Z) + batched(ah, sA, bl, sB, M, N, K, R, Z)
               + batched(al, sA, bh, sB, M, N, K, R, Z))
    exact = batched(A.astype(np.float64), sA, B.astype(np.float64), sB, M, N, K, R, Z)
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")
    C0 = rng.standard_normal(Z * M * N).astype(np.float32)
    prec = "bf16" if plain else "bf16x3"
    if plain:
        ctx.bf16_map(["gemm"])

    def run(mode):
        ctx.gemm_planes(mode)
        Cd = torch.tensor(C0, device="cuda")
        ctx.gemm(mlcc.PREC[prec], M, N, K, R, Z, 0.5, Ad, sA, Bd, sB, -1.5, Cd, [N, 1, M * N])
        return Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)

    got = run(1)
    # the planes were allocated (the product ran on them)
    assert ctx.bytes() >= plane_bytes(M, N, K, R, Z, a_shared, 1 if plain else 2)
    c0 = C0.astype(np.float64).reshape(Z, M, N)
    scale = np.sqrt(K * R) + 1.0
    err = np.abs(got - (0.5 * ref - 1.5 * c0)).max()
    assert err <= TOL_ACC * scale, err
    if not plain:
        assert np.abs(got - (0.5 * exact - 1.5 * c0)).max() <= TOL_SPLIT * scale
    # the unpacked kernel multiplies the same BF16 values
    unpacked = run(-1)
    assert np.abs(got - unpacked).max() <= 2 * TOL_ACC * scale
    ctx.close()


PLANE_TILES = [(256, 256), (128, 128)]


@pytest.mark.parametrize("plain", [False, True])
def test_every_plane_tile(plain):
    """Each tile of the planes menu, forced, on a shape ragged in m, n and k
    with a batch reduction; the tile is reported as used."""
    M, N, K, R = 300, 270, 76, 2
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(21 + plain)
    sA = [K, 1, M * K, 0]
    sB = [1, K, K * N, 0]
    A = rng.standard_normal(M * K * R).astype(np.float32)
    B = rng.standard_normal(K * N * R).astype(np.float32)
    ah, al = split_planes(A)
    bh, bl = split_planes(B)
    ref = batched(ah, sA, bh, sB, M, N, K, R, 1)[0]
    if not plain:
        ref += batched(ah, sA, bl, sB, M, N, K, R, 1)[0] + batched(al, sA, bh, sB, M, N, K, R, 1)[0]
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")
    prec = "bf16" if plain else "bf16x3"
    if plain:
        ctx.bf16_map(["gemm"])
    ctx.gemm_planes(1)
    for bm, bn in PLANE_TILES:
        ctx.gemm_tile(bm, bn)
        Cd = torch.zeros(M * N, device="cuda")
        ctx.gemm(mlcc.PREC[prec], M, N, K, R, 1, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, 0])
        assert ctx.gemm_tile(0, 0) == (bm, bn)
        got = Cd.cpu().numpy().astype(np.float64).reshape(M, N)
        assert np.abs(got - ref).max() <= TOL_ACC * (np.sqrt(K * R) + 1.0), (bm, bn)
    ctx.close()


def test_planes_two_level_indices():
    """Two-level row and column indices (a batch of trial vectors in one
    launch) read by the packing pass, and C written through them."""
    import ctypes as C
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(31)
    Mh, Ml, K, Nh, Nl, R = 3, 70, 44, 4, 33, 3
    M, N = Mh * Ml, Nh * Nl
    sAr, sA_hi = 12000, 3400   # A (m=(mh,ml), k) at r*sAr + mh*sA_hi + ml*K + k
    sBr, sB_hi = 9000, 1600    # B (k, n=(nh,nl)) at r*sBr + nh*sB_hi + nl*K + k
    A = rng.standard_normal(R * sAr).astype(np.float32)
    B = rng.standard_normal(R * sBr).astype(np.float32)
    ah, al = split_planes(A)
    bh, bl = split_planes(B)
    ldc, sC_hi_m, sC_hi_n = 200, 20000, 50  # C (m, n) at mh*20000 + ml*200 + nh*50 + nl
    ref = np.zeros(Mh * sC_hi_m)
    ia = (np.arange(R)[:, None, None] * sAr + (np.arange(M) // Ml)[None, :, None] * sA_hi
          + (np.arange(M) % Ml)[None, :, None] * K + np.arange(K)[None, None, :])
    ib = (np.arange(R)[:, None, None] * sBr + (np.arange(N) // Nl)[None, :, None] * sB_hi
          + (np.arange(N) % Nl)[None, :, None] * K + np.arange(K)[None, None, :])
    prod = sum(ah[ia[r]] @ bh[ib[r]].T + ah[ia[r]] @ bl[ib[r]].T + al[ia[r]] @ bh[ib[r]].T
               for r in range(R))
    off = ((np.arange(M) // Ml) * sC_hi_m + (np.arange(M) % Ml) * ldc)[:, None] + \
        ((np.arange(N) // Nl) * sC_hi_n + (np.arange(N) % Nl))[None, :]
    ref[off] = prod
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")
    Cd = torch.zeros(Mh * sC_hi_m, device="cuda")
    torch.cuda.synchronize()
    ctx.gemm_planes(1)
    st = ctx.lib.mlcc_gemm2(ctx.h, mlcc.BF16X3, M, N, K, R, 1, 1.0, C.c_void_p(Ad.data_ptr()),
                            (C.c_int64 * 4)(K, 1, sAr, 0), C.c_void_p(Bd.data_ptr()),
                            (C.c_int64 * 4)(1, K, sBr, 0), 0.0, C.c_void_p(Cd.data_ptr()),
                            (C.c_int64 * 3)(ldc, 1, 0),
                            (C.c_int64 * 6)(Ml, sA_hi, sC_hi_m, Nl, sB_hi, sC_hi_n))
    assert st == 0, ctx.last_error()
    assert ctx.bytes() >= plane_bytes(M, N, K, R, 1, True, 2)
    got = Cd.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= TOL_ACC * (np.sqrt(K * R) + 1.0)
    ctx.close()


def test_planes_large_product_default_rule():
    """The doubles-to-singles product of MLCC2 150/1200/3600 (active 50/500):
    5 batches of 3601 x 5000 x 5000 with a shared A, 0.9 TFLOP, which the
    default rule packs; sampled outputs against the exact BF16 products."""
    ctx = mlcc.Context(0)
    M, N, K, Z = 3601, 5000, 5000, 5
    g = torch.Generator(device="cuda").manual_seed(5)
    Ad = torch.randn(M * K, device="cuda", generator=g)
    Bd = torch.randn(Z * N * K, device="cuda", generator=g)
    Cd = torch.zeros(Z * M * N, device="cuda")
    ctx.gemm(mlcc.BF16X3, M, N, K, 1, Z, 1.0, Ad, [K, 1, 0, 0], Bd, [1, K, 0, N * K], 0.0, Cd,
             [N, 1, M * N])
    assert ctx.bytes() >= plane_bytes(M, N, K, 1, Z, True, 2)
    A = Ad.cpu().numpy().reshape(M, K)
    B = Bd.cpu().numpy().reshape(Z, N, K)
    got = Cd.cpu().numpy().reshape(Z, M, N).astype(np.float64)
    rng = np.random.default_rng(3)
    for _ in range(64):
        z, m, n = rng.integers(Z), rng.integers(M), rng.integers(N)
        ah, al = split_planes(A[m])
        bh, bl = split_planes(B[z, n])
        ref = ah @ bh + ah @ bl + al @ bh
        assert abs(got[z, m, n] - ref) <= TOL_ACC * (np.sqrt(K) + 1.0), (z, m, n)
    ctx.close()


@pytest.mark.parametrize("plain", [False, True])
def test_planes_unaligned_operands(plain):
    """Operands that start off a 16-byte boundary (A shifted by 1 element, B
    by 3): the packing pass gathers them element by element."""
    M, N, K, R, Z = 290, 270, 84, 2, 2
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(41 + plain)
    sA = [K, 1, M * K, M * K * R]
    sB = [1, K, K * N, K * N * R]
    A = rng.standard_normal(1 + M * K * R * Z).astype(np.float32)
    B = rng.standard_normal(3 + K * N * R * Z).astype(np.float32)
    ah, al = split_planes(A[1:])
    bh, bl = split_planes(B[3:])
    ref = batched(ah, sA, bh, sB, M, N, K, R, Z)
    if not plain:
        ref += batched(ah, sA, bl, sB, M, N, K, R, Z) + batched(al, sA, bh, sB, M, N, K, R, Z)
    Ad = torch.tensor(A, device="cuda")[1:]
    Bd = torch.tensor(B, device="cuda")[3:]
    prec = "bf16" if plain else "bf16x3"
    if plain:
        ctx.bf16_map(["gemm"])
    ctx.gemm_planes(1)
    Cd = torch.zeros(Z * M * N, device="cuda")
    ctx.gemm(mlcc.PREC[prec], M, N, K, R, Z, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, M * N])
    assert ctx.bytes() >= plane_bytes(M, N, K, R, Z, False, 1 if plain else 2)
    got = Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)
    assert np.abs(got - ref).max() <= TOL_ACC * (np.sqrt(K * R) + 1.0)
    ctx.close()


# operand layouts the unpacked split kernel cannot read: A contiguous along m,
# B contiguous along n, k groups cut by a K that is not a multiple of 4
LAYOUTS = [("m", "n", 84), ("m", "k", 84), ("k", "n", 84), ("k", "k", 83), ("m", "n", 83)]


@pytest.mark.parametrize("layout", LAYOUTS)
def test_planes_any_operand_layout(layout):
    """Split products of any operand layout run on packed planes (the packing
    pass transposes operands contiguous along m or n through LDS tiles)."""
    al_, bl_, K = layout
    M, N, R, Z = 290, 270, 2, 2
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(abs(hash(layout)) % 2**32)
    sAm, sAk = (K, 1) if al_ == "k" else (1, M)
    sBk, sBn = (N, 1) if bl_ == "n" else (1, K)
    sA = [sAm, sAk, M * K, M * K * R]
    sB = [sBk, sBn, K * N, K * N * R]
    A = rng.standard_normal(M * K * R * Z).astype(np.float32)
    B = rng.standard_normal(K * N * R * Z).astype(np.float32)
    ah, al = split_planes(A)
    bh, bl = split_planes(B)
    ref = (batched(ah, sA, bh, sB, M, N, K, R, Z) + batched(ah, sA, bl, sB, M, N, K, R, Z)
           + batched(al, sA, bh, sB, M, N, K, R, Z))
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")
    ctx.gemm_planes(1)
    Cd = torch.zeros(Z * M * N, device="cuda")
    ctx.gemm(mlcc.BF16X3, M, N, K, R, Z, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, M * N])
    assert ctx.bytes() >= plane_bytes(M, N, K, R, Z, False, 2)
    got = Cd.cpu().numpy().astype(np.float64).reshape(Z, M, N)
    assert np.abs(got - ref).max() <= TOL_ACC * (np.sqrt(K * R) + 1.0)
    ctx.close()


def test_plain_map_keeps_fp32_for_other_layouts():
    """A contraction on the plain-BF16 map whose operands the split kernel
    cannot read keeps FP32 MFMA (as the map's accuracy study measured it),
    also when packing is forced: bitwise the FP32 result."""
    M, N, K, R = 200, 180, 96, 2
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(51)
    sA = [1, M, M * K, 0]   # A contiguous along m
    sB = [N, 1, K * N, 0]   # B contiguous along n
    Ad = torch.tensor(rng.standard_normal(M * K * R).astype(np.float32), device="cuda")
    Bd = torch.tensor(rng.standard_normal(K * N * R).astype(np.float32), device="cuda")

    def run(prec):
        Cd = torch.zeros(M * N, device="cuda")
        ctx.gemm(mlcc.PREC[prec], M, N, K, R, 1, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, 0])
        return Cd.cpu().numpy()

    ctx.bf16_map(["gemm"])
    ctx.gemm_planes(1)
    assert np.array_equal(run("bf16"), run("fp32"))
    ctx.close()


# FP32 cases: K and the batch-reduced k' of any length (the FP32 packing
# reads element by element when a row is not 16-byte aligned)
CASES_F32 = CASES + [(70, 90, 33, 2, 2, False), (257, 129, 7, 3, 1, True)]


@pytest.mark.parametrize("case", CASES_F32)
def test_f32_planes_products(case):
    """FP32 products on FP32 planes (the planes kernel's FP32 mode, forced)
    against the FP64 product: FP32 accumulation error only, and the same
    result bounds as the FP32 kernel they replace."""
    M, N, K, R, Z, a_shared = case
    ctx = mlcc.Context(0)
    rng = np.random.default_rng(abs(hash(("f32",) + case)) % 2**32)
    sA = [K, 1, M * K, 0 if a_shared else M * K * R]
    sB = [1, K, K * N, K * N * R]
    A = rng.standard_normal(M * K * R * (1 if a_shared else Z)).astype(np.float32)
    B = rng.standard_normal(K * N * R * Z).astype(np.float32)
    ref = batched(A.astype(np.float64), sA, B.astype(np.float64), sB, M, N, K, R, Z)
    Ad, Bd = torch.tensor(A, device="cuda"), torch.tensor(B, device="cuda")
    outs = []
    for mode in (1, -1):
        Cd = torch.zeros(Z * M * N, device="cuda", dtype=torch.float32)
        ctx.gemm_planes(mode)
        ctx.gemm(mlcc.FP32, M, N, K, R, Z, 1.0, Ad, sA, Bd, sB, 0.0, Cd, [N, 1, M * N])
        outs.append(Cd.cpu().numpy().reshape(Z, M, N).astype(np.float64))
    ctx.gemm_planes(0)
    # FP32 products and accumulation (the other parity tests' derived bar,
    # one contraction over K R terms), relative to the largest output
    from gpu_util import tol_chain
    scale = np.abs(ref).max()
    err_planes, err_fp32 = (np.abs(got - ref).max() for got in outs)
    assert err_planes <= tol_chain("fp32", K * R, 1) * scale
    assert err_fp32 <= tol_chain("fp32", K * R, 1) * scale
    assert err_planes <= 2.0 * err_fp32 + 1e-7 * scale
