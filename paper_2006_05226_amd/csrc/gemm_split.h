// Split-BF16 products of the contraction engine: FP32 operands on the BF16
// matrix cores.  Included by the FP32 instantiation units after
// gemm_kernel.h (the FP64 units never instantiate it).
#pragma once

#include "gemm_kernel.h"

namespace mlcc {
namespace gk {

// FP32 operands on the BF16 matrix cores: each element x is split into
// hi = bf16(x) and lo = bf16(x - hi) when it is staged, and a fragment
// product is hi*hi + hi*lo + lo*hi (three v_mfma_f32_16x16x32_bf16, FP32
// accumulation; the dropped lo*lo term is below 2^-16 of the product).
// Both operands k-contiguous, vector-only loads.  Lane l of the bf16 MFMA
// holds A[l%16][8*(l/16) + e] and B[8*(l/16) + e][l%16], e < 8 (measured), so
// a lane's fragment is one 16-byte read of a [m][k] LDS row.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf4v __attribute__((ext_vector_type(4)));

template <typename TC, int BM, int BN, bool PLAIN>
__global__ __launch_bounds__((WaveGrid<BM, BN>::NT)) void k_gemm_split(KParams kp) {
  typedef WaveGrid<BM, BN> WG;
  constexpr int BK = Tr<float>::BK, VEC = Tr<float>::VEC, LEN = BK + 8;  // 80-byte rows
  constexpr int WTM = BM / WG::WM, WTN = BN / WG::WN, FM = WTM / 16, FN = WTN / 16;
  static_assert(BK == 32 && VEC == 4, "tile");
  typedef Stage<float, BM, false, true, WG::NT> SA;
  typedef Stage<float, BN, false, true, WG::NT> SB;
  __shared__ __attribute__((aligned(16))) __bf16 Ah[2][BM][LEN];
  __shared__ __attribute__((aligned(16))) __bf16 Al[2][PLAIN ? 1 : BM][LEN];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[2][BN][LEN];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[2][PLAIN ? 1 : BN][LEN];

  const GemmArgs &p = kp.a;
  // plain BF16: hi products only, no lo planes
  constexpr bool plain = PLAIN;
  const int64_t L = blockIdx.x;
  const int64_t w = (L % kXcd) * kp.per_xcd + L / kXcd;
  if (w >= kp.nwork) return;
  int64_t tm, tn, zs;
  tile_of(kp, w, tm, tn, zs);
  const int64_t z = zs / kp.splits;
  const int split = (int)(zs % kp.splits);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WG::WN, wn = wave % WG::WN, g = lane >> 4, l16 = lane & 15;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t total = p.R * kp.ktiles;
  const int64_t s_begin = split * kp.steps_per_split;
  const int64_t s_end = min(total, s_begin + kp.steps_per_split);
  const float *Az = static_cast<const float *>(p.A) + z * p.sAz;
  const float *Bz = static_cast<const float *>(p.B) + z * p.sBz;

  SA sa;
  SB sb;
  sa.init_v(tid, m0, p.Mlo, p.sAm, p.M, p.sAm_hi);
  sb.init_v(tid, n0, p.Nlo, p.sBn, p.N, p.sBn_hi);

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0, 0, 0, 0};

  float ra[SA::U][VEC], rb[SB::U][VEC];
  int64_t lr = s_begin / kp.ktiles;
  int64_t lk0 = (s_begin - lr * kp.ktiles) * BK;
  auto load_next = [&]() {
    sa.load_v(ra, Az + lr * p.sAr, lk0, p.K, p.sAk);
    sb.load_v(rb, Bz + lr * p.sBr, lk0, p.K, p.sBk);
    lk0 += BK;
    if (lk0 >= kp.ktiles * BK) {
      lk0 = 0;
      ++lr;
    }
  };
  auto split_store = [](const float (&x)[VEC], __bf16 *hi, __bf16 *lo) {
    bf4v h, l;
#pragma unroll
    for (int q = 0; q < VEC; ++q) {
      h[q] = (__bf16)x[q];
      l[q] = (__bf16)(x[q] - (float)h[q]);
    }
    *reinterpret_cast<bf4v *>(hi) = h;
    if constexpr (!plain) *reinterpret_cast<bf4v *>(lo) = l;
  };
  auto store = [&](int buf) {
    sa.mask(ra);
    sb.mask(rb);
#pragma unroll
    for (int e = 0; e < SA::U; ++e)
      split_store(ra[e], &Ah[buf][sa.row[e]][sa.col[e]], plain ? nullptr : &Al[buf][sa.row[e]][sa.col[e]]);
#pragma unroll
    for (int e = 0; e < SB::U; ++e)
      split_store(rb[e], &Bh[buf][sb.row[e]][sb.col[e]], plain ? nullptr : &Bl[buf][sb.row[e]][sb.col[e]]);
  };

  int cur = 0;
  if (s_begin < s_end) {
    load_next();
    store(0);
  }
  __syncthreads();
  for (int64_t step = s_begin; step < s_end; ++step) {
    const bool more = step + 1 < s_end;
    if (more) load_next();
    bf8v ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int r = wm * WTM + i * 16 + l16;
      ah[i] = *reinterpret_cast<const bf8v *>(&Ah[cur][r][g * 8]);
      if constexpr (!plain) al[i] = *reinterpret_cast<const bf8v *>(&Al[cur][r][g * 8]);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int r = wn * WTN + j * 16 + l16;
      bh[j] = *reinterpret_cast<const bf8v *>(&Bh[cur][r][g * 8]);
      if constexpr (!plain) bl[j] = *reinterpret_cast<const bf8v *>(&Bl[cur][r][g * 8]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    if constexpr (!plain) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  epilogue<float, TC, FM, FN, WTM, WTN, false>(kp, acc, m0, n0, z, split, lane, wm, wn);
}

}  // namespace gk
}  // namespace mlcc

// Tile menus of the split products and of the plain BF16 products.
#define MLCC_GEMM_TILES_PLAIN(X) \
  X(128, 128) X(128, 64) X(64, 128) X(96, 160) X(160, 96) X(64, 64) X(128, 32) X(32, 128) X(32, 32)
#define MLCC_GEMM_TILES_SPLIT(X) \
  X(128, 128) X(128, 96) X(96, 128) X(128, 64) X(64, 128) X(96, 96) X(64, 64) X(128, 32) X(32, 128) \
  X(64, 32) X(32, 64) X(32, 32) X(96, 160) X(160, 96)
