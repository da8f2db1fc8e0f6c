// Split and plain BF16 products on packed operand planes.  Included by the
// FP32 instantiation units after gemm_kernel.h and gemm_split.h.
//
// For large contractions the FP32 operands are first converted once into
// BF16 planes, hi = bf16(x) and lo = bf16(x - hi) (hi only for plain
// products), laid out [batch][row][k'] with k' = r * K + k the flattened
// reduction index: rows padded to a multiple of kPlaneRowPad, k' padded to a
// multiple of kPlaneKPad, padding zero.  The product kernel then streams
// the planes into LDS with direct global-to-LDS loads (global_load_lds_dwordx4):
// no VGPR staging, no per-step conversion, no bounds checks inside the
// k-loop.  The conversion is the same as the split kernel's (round to
// nearest even, twice), so both kernels multiply the same BF16 values.
//
// LDS layout: per operand, plane and stage, rows of KS BF16 (KS = 32 or 64
// per k-step: CH = KS / 8 chunks of 16 bytes).  One load instruction of a
// wave fills 1 KB of LDS (512 / KS rows), lane c writing bytes 16c..16c+15;
// the lane therefore loads logical chunk (c % CH) ^ swz(row) of row c / CH,
// so that chunk g of row r sits at physical chunk g ^ swz(r), swz(r) =
// (r / 2) % CH.  With it the 16-byte fragment reads (16 rows, one chunk) run
// free of bank conflicts: measured with SQ_LDS_BANK_CONFLICT on the 256 x 256
// split tile, 0 against 0.16 of the busy cycles without a swizzle, with
// (r / 4) % 4, or with a variant that also flips on bit 3 of r, and 0.71
// against 0.65 matrix-core busy.
#pragma once

#include "gemm_kernel.h"
#include "gemm_split.h"

namespace mlcc {
namespace gk {

constexpr int kPlaneBK = 32;       // k of one v_mfma_f32_16x16x32_bf16
constexpr int kPlaneRowPad = 256;  // the largest tile dimension of the menu
constexpr int kPlaneKPad = 64;

// One operand seen as Z batches of `rows` rows, each row R slices of K
// elements, with an optional two-level row index: contiguous along k
// (s_k = 1, k_pack_planes) or along the rows (k_pack_planes_t).
struct PackArgs {
  const float *X;
  int64_t rows, K, R, Z;
  int64_t s_row, s_r, s_z, s_k;
  int64_t lo, s_hi;        // two-level row index (lo <= 0: one level)
  int64_t rows_p, kp;      // padded plane extents
  __bf16 *hi, *lo_plane;   // [Z][rows_p][kp]; lo_plane unused for plain products
  int vec4;                // every group of 4 elements (k % 4 == 0) is one aligned 16-byte load
};

// One thread per 8 consecutive k' of one row (one 16-byte group of each
// plane); consecutive threads walk along k', so the FP32 reads of a wave are
// contiguous within a slice.  Padding rows and k' >= R K are written as zero.
template <bool PLAIN> __global__ __launch_bounds__(256) void k_pack_planes(PackArgs a) {
  const int64_t chunks = a.kp / 8;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.Z * a.rows_p * chunks) return;
  const int64_t rz = t / chunks, ch = t - rz * chunks;
  const int64_t z = rz / a.rows_p, m = rz - z * a.rows_p;
  const int64_t k0 = ch * 8, KK = a.R * a.K;
  bf8v h, l;
  if (m < a.rows && a.vec4) {
    // K and KK are multiples of 4: each half of the chunk is one 16-byte
    // group inside one slice, wholly inside or wholly past the reduction
    const float *X = a.X + z * a.s_z + two_level(m, a.lo, a.s_row, a.s_hi);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int64_t kk = k0 + 4 * g, r = kk / a.K, k = kk - r * a.K;
      f4 v = f4{0.0f, 0.0f, 0.0f, 0.0f};
      if (kk < KK) v = *reinterpret_cast<const f4 *>(X + r * a.s_r + k);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        h[4 * g + q] = (__bf16)v[q];
        l[4 * g + q] = (__bf16)(v[q] - (float)h[4 * g + q]);
      }
    }
  } else if (m < a.rows) {
    const float *X = a.X + z * a.s_z + two_level(m, a.lo, a.s_row, a.s_hi);
    int64_t r = k0 / a.K, k = k0 - r * a.K;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float x = k0 + q < KK ? X[r * a.s_r + k] : 0.0f;
      h[q] = (__bf16)x;
      l[q] = (__bf16)(x - (float)h[q]);
      if (++k == a.K) {
        k = 0;
        ++r;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) h[q] = l[q] = (__bf16)0.0f;
  }
  const int64_t o = rz * a.kp + k0;
  *reinterpret_cast<bf8v *>(a.hi + o) = h;
  if constexpr (!PLAIN) *reinterpret_cast<bf8v *>(a.lo_plane + o) = l;
}

// Operands contiguous along the rows: 64 rows x 64 k' per block, read along
// the rows into an LDS tile, written as 16-byte groups of each plane.
template <bool PLAIN> __global__ __launch_bounds__(256) void k_pack_planes_t(PackArgs a) {
  __shared__ float t[64][65];
  const int64_t tk_n = a.kp / 64, tm_n = a.rows_p / 64;
  int64_t q = blockIdx.x;
  const int64_t tk = q % tk_n;
  q /= tk_n;
  const int64_t tm = q % tm_n, z = q / tm_n;
  const int64_t m0 = tm * 64, k0 = tk * 64, KK = a.R * a.K;
  const float *X = a.X + z * a.s_z;
  const int tid = threadIdx.x;
  for (int e = 0; e < 16; ++e) {
    const int u = tid + e * 256, dm = u & 63, dk = u >> 6;
    const int64_t m = m0 + dm, kk = k0 + dk;
    float x = 0.0f;
    if (m < a.rows && kk < KK) {
      const int64_t r = kk / a.K, k = kk - r * a.K;
      x = X[two_level(m, a.lo, a.s_row, a.s_hi) + r * a.s_r + k * a.s_k];
    }
    t[dm][dk] = x;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int c = tid + e * 256, dm = c >> 3, ch = c & 7;
    bf8v h, l;
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const float x = t[dm][ch * 8 + qq];
      h[qq] = (__bf16)x;
      l[qq] = (__bf16)(x - (float)h[qq]);
    }
    const int64_t o = (z * a.rows_p + m0 + dm) * a.kp + k0 + ch * 8;
    *reinterpret_cast<bf8v *>(a.hi + o) = h;
    if constexpr (!PLAIN) *reinterpret_cast<bf8v *>(a.lo_plane + o) = l;
  }
}

struct PlaneOps {
  const __bf16 *ah, *al, *bh, *bl;  // al, bl null for plain products
  int64_t a_zs, b_zs;               // plane batch strides (0: one plane for every batch)
};

// Chunk swizzle of a row of CH 16-byte chunks: chunk g of row r sits at
// g ^ plane_swz<CH>(r).
template <int CH> __device__ __forceinline__ int plane_swz(int r) { return (r >> 1) & (CH - 1); }

// Fragments of one k-step (KS = 32 or 64 BF16, one or two MFMA k-slices) of a
// wave, read from a stage of LDS (A planes at As, B planes at Bs, each plane
// rows x KS BF16 with swizzled chunks); sw: this lane's swizzle.
// F32: the plane holds FP32 values (a plain plane of 4-byte elements, each
// 16-byte chunk four consecutive k); a chunk then feeds four
// v_mfma_f32_16x16x4f32, lane group g taking k = 4 g + s in the s-th (the
// same order in A and B, so the sum over a k-step is only reordered).
template <int FM, int FN, int WTM, int WTN, bool PLAIN, int KS, bool F32 = false> struct PlaneFrags {
  static constexpr int NS = KS / kPlaneBK;
  bf8v ah[NS][FM], al[NS][PLAIN ? 1 : FM], bh[NS][FN], bl[NS][PLAIN ? 1 : FN];
  __device__ __forceinline__ void read(const __bf16 *As, int plane_a, const __bf16 *Bs, int plane_b,
                                       int wm, int wn, int l16, int g, int sw) {
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      const int ch = (4 * u + g) ^ sw;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int o = (wn * WTN + j * 16 + l16) * KS + ch * 8;
        bh[u][j] = *reinterpret_cast<const bf8v *>(Bs + o);
        if constexpr (!PLAIN) bl[u][j] = *reinterpret_cast<const bf8v *>(Bs + plane_b + o);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        const int o = (wm * WTM + i * 16 + l16) * KS + ch * 8;
        ah[u][i] = *reinterpret_cast<const bf8v *>(As + o);
        if constexpr (!PLAIN) al[u][i] = *reinterpret_cast<const bf8v *>(As + plane_a + o);
      }
    }
  }
  // the products: all hi*hi first, then hi*lo, then lo*hi, so that
  // consecutive MFMAs never accumulate into the same registers
  __device__ __forceinline__ void mma(f4 (&acc)[FM][FN]) const {
    if constexpr (F32) {
#pragma unroll
      for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(__builtin_bit_cast(f4, ah[u][i])[s],
                                                              __builtin_bit_cast(f4, bh[u][j])[s],
                                                              acc[i][j], 0, 0, 0);
      return;
    }
#pragma unroll
    for (int u = 0; u < NS; ++u)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][i], bh[u][j], acc[i][j], 0, 0, 0);
    if constexpr (!PLAIN) {
#pragma unroll
      for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[u][i], bl[u][j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[u][i], bh[u][j], acc[i][j], 0, 0, 0);
    }
  }
};

typedef __attribute__((address_space(3))) void lds_void;

// 16 bytes per lane from global memory straight into LDS: lane l reads at
// base + off (base uniform over the wave) and its bytes land at dst + 16 l
// (dst uniform over the wave).
__device__ __forceinline__ void load_lds16(const char *base, uint32_t off, __bf16 *dst) {
  __builtin_amdgcn_global_load_lds(base + off, (lds_void *)dst, 16, 0, 0);
}

// Product kernel on packed planes: BM x BN output tile, WM x WN waves, a ring
// of NSTG LDS stages.
template <int WM, int WN> struct PlaneWaves {
  static constexpr int NT = 64 * WM * WN;
};

template <typename TC, int BM, int BN, int WM, int WN, bool PLAIN, int KS, int NSTG, bool F32 = false>
__global__ __launch_bounds__((PlaneWaves<WM, WN>::NT)) void k_gemm_planes(KParams kp, PlaneOps po) {
  static_assert(!F32 || PLAIN, "FP32 planes are one plane");
  constexpr int NW = WM * WN, WTM = BM / WM, WTN = BN / WN, FM = WTM / 16, FN = WTN / 16;
  constexpr int PL = PLAIN ? 1 : 2;
  constexpr int CH = KS / 8, RPL = 512 / KS;  // 16-byte chunks per row, rows per 1 KB load
  constexpr int RA = BM * KS, RB = BN * KS;   // elements of one plane of a stage
  constexpr int QA = PL * BM / RPL, QB = PL * BN / RPL;  // 1 KB loads per stage
  // Eight-wave tiles run the two waves of each SIMD half a k-step apart (see
  // the loop below); the loads of a stage are then issued by the first half.
  constexpr bool PP = NW == 8 && WM == 2;
  constexpr int NWI = PP ? NW / 2 : NW;                  // waves issuing the loads
  constexpr int EA = QA / NWI, EB = QB / NWI;
  static_assert(QA % NWI == 0 && QB % NWI == 0 && WTM % 16 == 0 && WTN % 16 == 0, "tile");
  static_assert(BM <= kPlaneRowPad && BN <= kPlaneRowPad && kPlaneRowPad % BM == 0 &&
                kPlaneRowPad % BN == 0, "plane padding");
  constexpr int STAGE = PL * (RA + RB);  // elements of one stage
  static_assert(NSTG >= 2 && NSTG * STAGE * 2 <= 160 * 1024, "LDS stages");
  constexpr int LPS = EA + EB;  // loads per stage of an issuing wave
  static_assert((NSTG - 2) * LPS <= 63, "vmcnt");
  __shared__ __attribute__((aligned(1024))) __bf16 lds[NSTG * STAGE];

  const int64_t L = blockIdx.x;
  const int64_t w = (L % kXcd) * kp.per_xcd + L / kXcd;
  if (w >= kp.nwork) return;
  int64_t tm, tn, zs;
  tile_of(kp, w, tm, tn, zs);
  const int64_t z = zs / kp.splits;
  const int split = (int)(zs % kp.splits);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform over the wave
  const int wm = wave / WN, wn = wave % WN, l16 = lane & 15;
  const int sw = plane_swz<CH>(l16), g = lane >> 4;  // this lane's fragment chunk: (4u + g) ^ sw
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t kpad = kp.ktiles * KS;
  const int s_begin = (int)(split * kp.steps_per_split);
  const int s_end = (int)min(kp.ktiles, (int64_t)s_begin + kp.steps_per_split);

  // Load q of a stage covers plane q / (rows / RPL), tile rows RPL (q % (rows
  // / RPL)) .. +RPL-1; its source is a wave-uniform offset plus this lane's
  // offset (row lane / CH of the RPL, logical chunk (lane % CH) ^ swz of the
  // row, which for RPL = 8 depends on the parity of the load's row block).
  // Every load addresses the plane buffer (A hi, B hi, A lo, B lo, within
  // 4 GB: the host checks) by its base and a 32-bit byte offset: the lane's
  // part, a wave-uniform part fixed for the tile (plane, batch, rows) and
  // the k-step's part.
  const int dr = lane / CH, dc = lane % CH;
  const uint32_t lane_b0 = 2u * (uint32_t)(dr * kpad + 8 * (dc ^ plane_swz<CH>(dr)));
  const uint32_t lane_b1 = 2u * (uint32_t)(dr * kpad + 8 * (dc ^ plane_swz<CH>(dr + RPL)));
  const char *pbase = reinterpret_cast<const char *>(po.ah);
  const int64_t a_lo = PLAIN ? 0 : po.al - po.ah, b_hi = po.bh - po.ah;
  const int64_t b_lo = PLAIN ? 0 : po.bl - po.ah;
  const int wi = PP ? wn : wave;  // this wave's index among the issuing waves
  uint32_t ua[EA], ub[EB];
#pragma unroll
  for (int e = 0; e < EA; ++e) {
    const int q = wi + NWI * e, pl = q / (BM / RPL), rq = q % (BM / RPL);
    ua[e] = 2u * (uint32_t)((pl ? a_lo : 0) + z * po.a_zs + (m0 + rq * RPL) * kpad) +
            ((RPL == 16 || (rq & 1) == 0) ? lane_b0 : lane_b1);
  }
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int q = wi + NWI * e, pl = q / (BN / RPL), rq = q % (BN / RPL);
    ub[e] = 2u * (uint32_t)((pl ? b_lo : b_hi) + z * po.b_zs + (n0 + rq * RPL) * kpad) +
            ((RPL == 16 || (rq & 1) == 0) ? lane_b0 : lane_b1);
  }
  auto issue = [&](int stage, int step) {
    __bf16 *As = lds + stage * STAGE, *Bs = As + PL * RA;
    const uint32_t k2 = 2u * (uint32_t)(step * KS);
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int q = wi + NWI * e, pl = q / (BM / RPL), rq = q % (BM / RPL);
      load_lds16(pbase, ua[e] + k2, As + pl * RA + rq * 512);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int q = wi + NWI * e, pl = q / (BN / RPL), rq = q % (BN / RPL);
      load_lds16(pbase, ub[e] + k2, Bs + pl * RB + rq * 512);
    }
  };

  f4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4{0, 0, 0, 0};

  // A ring of NSTG stages: the loads of step k + NSTG - 1 go into the stage
  // of step k - 1 once every wave has read it, so NSTG - 1 steps of loads are
  // in flight.  Before reading step k an issuing wave waits until at most the
  // loads of the NSTG - 2 later steps are outstanding (all of them near the
  // end, where fewer were issued).
  auto wait_stage = [&](int step) {
    if (NSTG > 2 && step + NSTG - 2 < s_end)
      asm volatile("s_waitcnt vmcnt(%0)" ::"n"((NSTG - 2) * LPS) : "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  };
  if constexpr (PP) {
    // Two halves of four waves, one wave of each on every SIMD (wm = 0, 1),
    // alternate between reading fragments from LDS and the products, so that
    // one half's reads run under the other half's MFMAs.  Half 0 passes the
    // barriers X_k (stage k has landed; nobody reads the stage of k - 1 any
    // more) and Y_k; half 1 is one barrier behind:
    //   half 0:  X_k  loads of k+NSTG-1, reads of k  Y_k  products of k
    //   half 1:  X_k  products of k-1                Y_k  reads of k
    // Each half waits for its own LDS reads before a barrier (lgkmcnt) and
    // half 0, which issues every load, for the loads of k before X_k
    // (vmcnt); the barriers themselves wait for nothing else, so later
    // loads stay in flight.  Both halves pass 2 n + 1 barriers for n steps.
    const int half = wm;
    auto barrier = [] {
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_barrier" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
    };
    if (half == 0)
      for (int t = 0; t < NSTG - 1; ++t)
        if (s_begin + t < s_end) issue(t, s_begin + t);
    if (half == 1) barrier();
    int cur = 0;
    for (int step = s_begin; step < s_end; ++step) {
      if (half == 0) wait_stage(step);
      barrier();
      if (half == 0 && step + NSTG - 1 < s_end) issue(cur == 0 ? NSTG - 1 : cur - 1, step + NSTG - 1);
      PlaneFrags<FM, FN, WTM, WTN, PLAIN, KS, F32> fr;
      const __bf16 *As = lds + cur * STAGE;
      fr.read(As, RA, As + PL * RA, RB, wm, wn, l16, g, sw);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      barrier();
      fr.mma(acc);
      cur = cur == NSTG - 1 ? 0 : cur + 1;
    }
    if (half == 0) barrier();
  } else {
    // Per k-step: wait for this wave's loads of the stage, a barrier (every
    // wave's loads have landed, and every wave has finished reading the
    // stage of the previous step), all fragment reads of the step, then the
    // loads of step k + NSTG - 1 into the stage of the previous step, then
    // the products.
    for (int t = 0; t < NSTG - 1; ++t)
      if (s_begin + t < s_end) issue(t, s_begin + t);
    int cur = 0;
    for (int step = s_begin; step < s_end; ++step) {
      wait_stage(step);
      __builtin_amdgcn_sched_barrier(0);
      asm volatile("s_barrier" ::: "memory");
      __builtin_amdgcn_sched_barrier(0);
      PlaneFrags<FM, FN, WTM, WTN, PLAIN, KS, F32> fr;
      const __bf16 *As = lds + cur * STAGE;
      fr.read(As, RA, As + PL * RA, RB, wm, wn, l16, g, sw);
      if (step + NSTG - 1 < s_end) issue(cur == 0 ? NSTG - 1 : cur - 1, step + NSTG - 1);
      fr.mma(acc);
      cur = cur == NSTG - 1 ? 0 : cur + 1;
    }
  }
  epilogue<float, TC, FM, FN, WTM, WTN, false>(kp, acc, m0, n0, z, split, lane, wm, wn);
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Plane geometry of a product: extents, batch counts and bytes.
struct PlaneGeom {
  int64_t mp, np, kp, za, zb;
  int pl;
  size_t bytes_a, bytes_b;  // per plane
  size_t total() const { return (size_t)pl * (bytes_a + bytes_b); }
};
inline PlaneGeom plane_geom(const GemmArgs &a, bool plain) {
  PlaneGeom g;
  g.mp = round_up(a.M, kPlaneRowPad);
  g.np = round_up(a.N, kPlaneRowPad);
  g.kp = round_up(a.R * a.K, kPlaneKPad);
  g.za = a.sAz ? a.Z : 1;
  g.zb = a.sBz ? a.Z : 1;
  g.pl = plain ? 1 : 2;
  g.bytes_a = sizeof(__bf16) * (size_t)g.za * g.mp * g.kp;
  g.bytes_b = sizeof(__bf16) * (size_t)g.zb * g.np * g.kp;
  return g;
}

inline void pack_planes(Exec &ex, PackArgs pa) {
  if (pa.s_k != 1) {  // contiguous along the rows: through LDS tiles
    const int64_t blocks = pa.Z * (pa.rows_p / 64) * (pa.kp / 64);
    MLCC_REQUIRE(blocks < ((int64_t)1 << 31), MLCC_E_ARG, "gemm: operand planes too large");
    if (pa.lo_plane)
      hipLaunchKernelGGL(k_pack_planes_t<false>, dim3((unsigned)blocks), dim3(256), 0, ex.stream, pa);
    else
      hipLaunchKernelGGL(k_pack_planes_t<true>, dim3((unsigned)blocks), dim3(256), 0, ex.stream, pa);
    MLCC_HIP(hipGetLastError());
    return;
  }
  // 16-byte groups: K a multiple of 4 and every group start 16-byte aligned
  const bool lo_ok = pa.lo <= 0 || pa.s_hi % 4 == 0;
  pa.vec4 = pa.K % 4 == 0 && pa.s_row % 4 == 0 && pa.s_r % 4 == 0 && pa.s_z % 4 == 0 && lo_ok &&
            reinterpret_cast<uintptr_t>(pa.X) % 16 == 0;
  const int64_t blocks = cdiv(pa.Z * pa.rows_p * (pa.kp / 8), 256);
  MLCC_REQUIRE(blocks < ((int64_t)1 << 31), MLCC_E_ARG, "gemm: operand planes too large");
  if (pa.lo_plane) hipLaunchKernelGGL(k_pack_planes<false>, dim3((unsigned)blocks), dim3(256), 0, ex.stream, pa);
  else hipLaunchKernelGGL(k_pack_planes<true>, dim3((unsigned)blocks), dim3(256), 0, ex.stream, pa);
  MLCC_HIP(hipGetLastError());
}

template <typename TC, int BM, int BN, int WM, int WN, bool PLAIN, int KS, int NSTG, bool F32 = false>
void launch_planes(Exec &ex, const GemmArgs &a, const PlaneOps &po, int64_t kpad, int splits) {
  KParams kp;
  kp.a = a;
  kp.splits = splits;
  kp.ktiles = kpad / KS;
  kp.steps_per_split = cdiv(kp.ktiles, splits);
  kp.tiles_m = (int)cdiv(a.M, BM);
  kp.tiles_n = (int)cdiv(a.N, BN);
  kp.nwork = (int64_t)kp.tiles_m * kp.tiles_n * a.Z * splits;
  kp.per_xcd = cdiv(kp.nwork, kXcd);
  kp.vec_a = kp.vec_b = 1;
  MLCC_REQUIRE(kp.per_xcd * kXcd < (int64_t)1 << 31, MLCC_E_ARG, "gemm: grid too large");
  kp.work = nullptr;
  if (splits > 1) kp.work = ex.scratch(sizeof(float) * (size_t)splits * a.Z * a.M * a.N);
  hipLaunchKernelGGL((k_gemm_planes<TC, BM, BN, WM, WN, PLAIN, KS, NSTG, F32>), dim3((unsigned)(kp.per_xcd * kXcd)),
                     dim3(64 * WM * WN), 0, ex.stream, kp, po);
  MLCC_HIP(hipGetLastError());
  if (splits > 1) {
    const int64_t n = a.Z * a.M * a.N;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_split_reduce<float, TC>), dim3(blocks), dim3(256), 0, ex.stream, kp);
    MLCC_HIP(hipGetLastError());
  }
}

template <typename TC, int BM, int BN, int WM, int WN, bool PLAIN, int KS, int NSTG, bool F32 = false>
int planes_occupancy(const GemmArgs &) {
  static std::atomic<int> cache{0};
  int nb = cache.load(std::memory_order_relaxed);
  if (nb > 0) return nb;
  const void *f = reinterpret_cast<const void *>(&k_gemm_planes<TC, BM, BN, WM, WN, PLAIN, KS, NSTG, F32>);
  MLCC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * WM * WN, 0));
  nb = std::max(nb, 1);
  cache.store(nb, std::memory_order_relaxed);
  return nb;
}

typedef void (*PlaneLaunchFn)(Exec &, const GemmArgs &, const PlaneOps &, int64_t, int);
struct PlaneTile {
  int bm, bn, waves, ks;
  PlaneLaunchFn fn;
  OccFn occ;
};

// Whether a split-eligible product runs on packed planes: never with a
// caller workspace (the planes are allocated) or planes beyond the lane's
// cap; otherwise as the lane's mode says, by default where the packing pass
// (read 4 bytes, write 2 per plane per operand element, ~6 TB/s measured)
// costs less than the planes kernel saves: on the 3601 x 5000 x 5000 (x 5)
// product the split kernel runs ~240 TFLOP/s unpacked and ~390 on planes,
// plain BF16 ~370 and ~700, so packing pays above ~130 (split) and ~130
// (plain) flops per packed byte; 150 is the rule, with at least 4 GFLOP so
// that the two extra launches stay negligible.
// ratio: the flops per packed byte above which packing pays (150 against the
// unpacked split kernel; 40 for split products whose operand layout leaves
// only FP32 MFMA, ~100 TFLOP/s, as the alternative).
inline bool use_planes(const Exec &ex, const GemmArgs &a, bool plain, double ratio = 150.0) {
  if (a.work || ex.planes_mode < 0) return false;
  const PlaneGeom g = plane_geom(a, plain);
  if (g.total() > ex.planes_cap) return false;
  if (ex.planes_mode > 0) return true;
  const double flops = 2.0 * (double)a.M * a.N * a.K * a.R * a.Z;
  const double pack_bytes = (4.0 / (2.0 * g.pl) + 1.0) * (double)g.total();
  return flops >= 4e9 && flops >= ratio * pack_bytes;
}

// Split products on packed planes for operands the split kernel cannot read
// (contiguous along m or n, or unaligned groups): any FP32 layout once
// packed; not for contractions on the plain-BF16 map, which keep FP32 MFMA
// there as their accuracy study measured.
inline bool planes_any_layout(const Exec &ex, const GemmArgs &a) {
  return a.bf16x3 && !a.bf16_plain && a.K > 0 && a.R > 0 && use_planes(ex, a, false, 40.0);
}

// Run the product on packed planes (kpad: the plane row length in 2-byte
// units) with the tile of the lowest modelled cost.
inline void run_planes(Exec &ex, const GemmArgs &a, const PlaneOps &po, int64_t kpad,
                       const PlaneTile *tiles, int ntiles) {
  const int64_t ncu = cu_count();
  int forced = -1;
  for (int t = 0; t < ntiles; ++t)
    if (tiles[t].bm == ex.force_bm && tiles[t].bn == ex.force_bn) forced = t;
  int best = -1, best_s = 1;
  double best_cost = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    if (forced >= 0 && t != forced) continue;
    const int bm = tiles[t].bm, bn = tiles[t].bn;
    const int64_t occ = tiles[t].occ(a), steps = kpad / tiles[t].ks;
    const int64_t blocks = cdiv(a.M, bm) * cdiv(a.N, bn) * a.Z;
    int64_t s = 1;
    if (blocks < occ * ncu && steps >= 8)
      s = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(occ * ncu / blocks, steps / 4), 128));
    const int64_t rounds = cdiv(blocks * s, occ * ncu);
    const double rate = tiles[t].waves == 8 ? 1.13 : 1.0;
    double cost = (double)rounds * (double)cdiv(steps, s) * tiles[t].ks * bm * bn * occ / rate;
    if (s > 1) cost += 2.0 * (double)s * a.Z * a.M * a.N;
    if (best < 0 || cost < best_cost) {
      best = t;
      best_s = (int)s;
      best_cost = cost;
    }
  }
  ex.last_bm = tiles[best].bm;
  ex.last_bn = tiles[best].bn;
  tiles[best].fn(ex, a, po, kpad, best_s);
}

// Pack both operands and run the product with the tile of the lowest
// modelled cost: rounds of resident blocks (the kernel's occupancy per CU)
// times each block's k-steps and outputs over its per-CU rate (rate: the
// 8-wave 256 x 256 tile, one block per CU, measured 1.13 times the rate of
// two 128 x 128 blocks per CU on the 3601 x 5000 x 5000 (x 5) product and
// on 4096^3), plus the split reduction's traffic.
template <typename TC>
void gemm_planes(Exec &ex, const GemmArgs &a, bool plain, const PlaneTile *tiles, int ntiles) {
  const PlaneGeom g = plane_geom(a, plain);
  // the product kernel addresses the planes with 32-bit byte offsets
  MLCC_REQUIRE(g.total() < ((size_t)1 << 32), MLCC_E_ARG, "gemm: operand planes too large");
  ex.planes.ensure(ex.al, g.total());
  __bf16 *base = static_cast<__bf16 *>(ex.planes.p);
  const size_t ea = g.bytes_a / sizeof(__bf16), eb = g.bytes_b / sizeof(__bf16);
  PlaneOps po;
  po.ah = base;
  po.bh = base + ea;
  po.al = plain ? nullptr : base + ea + eb;
  po.bl = plain ? nullptr : base + 2 * ea + eb;
  po.a_zs = a.sAz ? g.mp * g.kp : 0;
  po.b_zs = a.sBz ? g.np * g.kp : 0;

  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (ex.prof && ex.prof->on) {
    ev = ex.prof->next();
    MLCC_HIP(hipEventRecord(ev.first, ex.stream));
  }
  PackArgs pa;
  pa.X = static_cast<const float *>(a.A);
  pa.rows = a.M; pa.K = a.K; pa.R = a.R; pa.Z = g.za;
  pa.s_row = a.sAm; pa.s_r = a.sAr; pa.s_z = a.sAz; pa.s_k = a.sAk;
  pa.lo = a.Mlo; pa.s_hi = a.sAm_hi;
  pa.rows_p = g.mp; pa.kp = g.kp;
  pa.hi = const_cast<__bf16 *>(po.ah); pa.lo_plane = const_cast<__bf16 *>(po.al);
  pack_planes(ex, pa);
  pa.X = static_cast<const float *>(a.B);
  pa.rows = a.N; pa.Z = g.zb;
  pa.s_row = a.sBn; pa.s_r = a.sBr; pa.s_z = a.sBz; pa.s_k = a.sBk;
  pa.lo = a.Nlo; pa.s_hi = a.sBn_hi;
  pa.rows_p = g.np;
  pa.hi = const_cast<__bf16 *>(po.bh); pa.lo_plane = const_cast<__bf16 *>(po.bl);
  pack_planes(ex, pa);

  run_planes(ex, a, po, g.kp, tiles, ntiles);
  if (ev.first) {
    MLCC_HIP(hipEventRecord(ev.second, ex.stream));
    ex.prof->recs.push_back({a.tag, ev.first, ev.second, 2.0 * (double)a.M * a.N * a.K * a.R * a.Z});
  }
}

// FP32 products on the planes kernel: each operand copied once as
// [batch][row][k'] FP32 (rows padded to kPlaneRowPad, k' to kPlaneKPad / 2,
// padding zero), streamed into LDS by the same direct loads and multiplied
// by v_mfma_f32_16x16x4f32 (the kernel's F32 mode).  Operands contiguous
// along k only.  One thread per 8 consecutive k' of one row.
template <typename T> __global__ __launch_bounds__(256) void k_pack_f32(PackArgs a, T *out) {
  const int64_t chunks = a.kp / 8;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.Z * a.rows_p * chunks) return;
  const int64_t rz = t / chunks, ch = t - rz * chunks;
  const int64_t z = rz / a.rows_p, m = rz - z * a.rows_p;
  const int64_t k0 = ch * 8, KK = a.R * a.K;
  f4 v0 = f4{0.0f, 0.0f, 0.0f, 0.0f}, v1 = v0;
  if (m < a.rows) {
    const float *X = a.X + z * a.s_z + two_level(m, a.lo, a.s_row, a.s_hi);
    if (a.vec4) {
      const int64_t r0 = k0 / a.K, r1 = (k0 + 4) / a.K;
      if (k0 < KK) v0 = *reinterpret_cast<const f4 *>(X + r0 * a.s_r + (k0 - r0 * a.K));
      if (k0 + 4 < KK) v1 = *reinterpret_cast<const f4 *>(X + r1 * a.s_r + (k0 + 4 - r1 * a.K));
    } else {
      int64_t r = k0 / a.K, k = k0 - r * a.K;
      float x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        x[q] = k0 + q < KK ? X[r * a.s_r + k] : 0.0f;
        if (++k == a.K) {
          k = 0;
          ++r;
        }
      }
      v0 = f4{x[0], x[1], x[2], x[3]};
      v1 = f4{x[4], x[5], x[6], x[7]};
    }
  }
  const int64_t o = rz * a.kp + k0;
  *reinterpret_cast<f4 *>(out + o) = v0;
  *reinterpret_cast<f4 *>(out + o + 4) = v1;
}

inline void pack_f32(Exec &ex, PackArgs pa, float *out) {
  MLCC_REQUIRE(pa.s_k == 1, MLCC_E_STATE, "gemm: FP32 planes need operands contiguous along k");
  const bool lo_ok = pa.lo <= 0 || pa.s_hi % 4 == 0;
  pa.vec4 = pa.K % 4 == 0 && pa.s_row % 4 == 0 && pa.s_r % 4 == 0 && pa.s_z % 4 == 0 && lo_ok &&
            reinterpret_cast<uintptr_t>(pa.X) % 16 == 0;
  const int64_t blocks = cdiv(pa.Z * pa.rows_p * (pa.kp / 8), 256);
  MLCC_REQUIRE(blocks < ((int64_t)1 << 31), MLCC_E_ARG, "gemm: operand planes too large");
  hipLaunchKernelGGL(k_pack_f32<float>, dim3((unsigned)blocks), dim3(256), 0, ex.stream, pa, out);
  MLCC_HIP(hipGetLastError());
}

struct F32Geom {
  int64_t mp, np, kpf, za, zb;
  size_t bytes_a, bytes_b;
  size_t total() const { return bytes_a + bytes_b; }
};
inline F32Geom f32_geom(const GemmArgs &a) {
  F32Geom g;
  g.mp = round_up(a.M, kPlaneRowPad);
  g.np = round_up(a.N, kPlaneRowPad);
  g.kpf = round_up(a.R * a.K, kPlaneKPad / 2);
  g.za = a.sAz ? a.Z : 1;
  g.zb = a.sBz ? a.Z : 1;
  g.bytes_a = sizeof(float) * (size_t)g.za * g.mp * g.kpf;
  g.bytes_b = sizeof(float) * (size_t)g.zb * g.np * g.kpf;
  return g;
}

// Whether an FP32 product runs on FP32 planes: operands contiguous along k,
// no caller workspace, planes within the lane's cap; by default from 4 GFLOP
// and 300 flops per byte the packing moves (it reads and writes 4 bytes per
// operand element).  Measured: the 3601 x 5000 x 5000 (x 5) product (~750
// flops per byte) 108.6 -> 118.0 TFLOP/s with packing; the 40/400/1200 MLCC2
// transformation (~135) 3.6% slower on planes, so below the rule.  The
// outputs must also fill at least 85% of the padded plane rows x columns:
// the CCS product with 150 rows (padded to 256) ran 19.0 ms on planes
// against 13.6 on the FP32 kernel.
inline bool use_planes_f32(const Exec &ex, const GemmArgs &a) {
  if (a.work || ex.planes_mode < 0 || a.K <= 0 || a.R <= 0 || a.sAk != 1 || a.sBk != 1) return false;
  const F32Geom g = f32_geom(a);
  if (g.total() > ex.planes_cap) return false;
  if (ex.planes_mode > 0) return true;
  const double flops = 2.0 * (double)a.M * a.N * a.K * a.R * a.Z;
  const double fill = (double)a.M * a.N / ((double)g.mp * g.np);
  return flops >= 4e9 && flops >= 300.0 * 2.0 * (double)g.total() && fill >= 0.85;
}

template <typename TC>
void gemm_planes_f32(Exec &ex, const GemmArgs &a, const PlaneTile *tiles, int ntiles) {
  const F32Geom g = f32_geom(a);
  MLCC_REQUIRE(g.total() < ((size_t)1 << 32), MLCC_E_ARG, "gemm: operand planes too large");
  ex.planes.ensure(ex.al, g.total());
  float *fa = static_cast<float *>(ex.planes.p), *fb = fa + g.bytes_a / sizeof(float);
  const int64_t kpad = 2 * g.kpf;  // the kernel counts the plane rows in 2-byte units
  PlaneOps po;
  po.ah = reinterpret_cast<const __bf16 *>(fa);
  po.bh = reinterpret_cast<const __bf16 *>(fb);
  po.al = po.bl = nullptr;
  po.a_zs = a.sAz ? g.mp * kpad : 0;
  po.b_zs = a.sBz ? g.np * kpad : 0;
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (ex.prof && ex.prof->on) {
    ev = ex.prof->next();
    MLCC_HIP(hipEventRecord(ev.first, ex.stream));
  }
  PackArgs pa;
  pa.X = static_cast<const float *>(a.A);
  pa.rows = a.M; pa.K = a.K; pa.R = a.R; pa.Z = g.za;
  pa.s_row = a.sAm; pa.s_r = a.sAr; pa.s_z = a.sAz; pa.s_k = a.sAk;
  pa.lo = a.Mlo; pa.s_hi = a.sAm_hi;
  pa.rows_p = g.mp; pa.kp = g.kpf;
  pa.hi = nullptr; pa.lo_plane = nullptr;
  pack_f32(ex, pa, fa);
  pa.X = static_cast<const float *>(a.B);
  pa.rows = a.N; pa.Z = g.zb;
  pa.s_row = a.sBn; pa.s_r = a.sBr; pa.s_z = a.sBz; pa.s_k = a.sBk;
  pa.lo = a.Nlo; pa.s_hi = a.sBn_hi;
  pa.rows_p = g.np;
  pack_f32(ex, pa, fb);
  run_planes(ex, a, po, kpad, tiles, ntiles);
  if (ev.first) {
    MLCC_HIP(hipEventRecord(ev.second, ex.stream));
    ex.prof->recs.push_back({a.tag, ev.first, ev.second, 2.0 * (double)a.M * a.N * a.K * a.R * a.Z});
  }
}

}  // namespace gk
}  // namespace mlcc

// Tile menus of the planes kernel: (BM, BN, WM, WN, k per step, LDS stages).
// Measured on the 3601 x 5000 x 5000 (x 5) product, TFLOP/s with packing,
// split / plain: 256 x 256 with 8 waves (one block per CU, two waves per
// SIMD, the two halves half a step apart) 369 / 835, 354 / 797 with both
// halves in step; 128 x 128 with 4 waves (two blocks per CU) 305 split;
// 256 x 256 with 4 waves (one per SIMD, 128 x 128 per wave) 311 / 673;
// 4-wave 256 x 128 and 128 x 256 269 and 256 split.  More stages of shorter
// steps do not pay: plain 256 x 256 with 32-deep steps in 3 or 4 stages
// (96 KB of loads in flight instead of 64) 769 / 751.  Taller or lower
// bands of tiles per XCD (4 or 16 tile rows instead of 8) change the split
// rate by under 2%.
#ifndef MLCC_GEMM_TILES_PLANES
#define MLCC_GEMM_TILES_PLANES(X) X(256, 256, 2, 4, 32, 2) X(128, 128, 2, 2, 32, 2)
#endif
// Plain products (one plane): k-steps of 64, two MFMA k-slices per barrier.
#ifndef MLCC_GEMM_TILES_PLANES_PLAIN
#define MLCC_GEMM_TILES_PLANES_PLAIN(X) X(256, 256, 2, 4, 64, 2) X(128, 128, 2, 2, 64, 2)
#endif
// FP32 products on FP32 planes: the F32 mode of the plain kernel, 32 FP32
// values (128 bytes) per row and k-step.
#ifndef MLCC_GEMM_TILES_PLANES_F32
#define MLCC_GEMM_TILES_PLANES_F32(X) X(256, 256, 2, 4, 64, 2) X(128, 128, 2, 2, 64, 2)
#endif
