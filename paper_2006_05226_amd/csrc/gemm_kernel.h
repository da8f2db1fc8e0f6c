// Batched, batch-reduced, strided GEMM on CDNA4 matrix cores (MFMA): the
// kernel template, included by one translation unit per operand type.
//
//   C_z[m][n] = alpha * sum_{r<R} sum_{k<K} A_zr[m][k] * B_zr[k][n] + beta * Cin_z[m][n]
//
// Design
// * A block owns a BM x BN tile of C.  Its waves form a WM x WN grid, two
//   waves along a tile dimension that is a multiple of 32 and one along any
//   other multiple of 16 (the menus below hold only the former); each wave
//   owns a (BM/WM) x (BN/WN) sub-tile of 16 x 16 fragments.
// * FP32: v_mfma_f32_16x16x4f32, one instruction per 16x16x4 fragment product.
//   Lane l holds A[i = l%16][k], B[k][j = l%16] with k-group l/16; output
//   element e of lane l is D[4*(l/16) + e][l%16].
// * FP64: v_mfma_f64_4x4x4f64 (four independent 4x4x4 blocks per wave, twice
//   the FP64 rate of the 16x16x4 form on gfx950).  Lane 16*k + 4*b + i holds
//   A_b[i][k] and B_b[k][i]; lane 16*i + 4*b + j receives D_b[i][j] (measured
//   with a one-wave probe).  A 16x16x4 fragment product is four instructions:
//   in instruction r the B fragment is read with its 16 columns rotated by 4r,
//   so block b multiplies rows 4b..4b+3 with columns 4((b+r)%4)..+3.  When a
//   wave has fewer A fragments than B fragments the roles swap (A is read
//   rotated), so the rotated reads are the fewer ones.
// * Within one k-step of BK, k-group g of a fragment covers k = g*S .. g*S+S-1
//   (S = BK/4), the same assignment for A and B, so a lane's k-values are
//   contiguous.
// * Each operand is staged through double-buffered LDS in the layout of its
//   contiguous global dimension: [m][k] rows when k is contiguous (fragment
//   reads are 16-byte vectors along k), [k][m] rows when m is contiguous.
//   Global loads move 16 bytes per thread along the contiguous dimension when
//   stride and bounds allow it (element alignment suffices: compute queues
//   run in the unaligned access mode), element by element otherwise.
//   Row padding keeps fragment reads free of bank conflicts.
// * The next k-step's global loads are issued before the MFMAs of the current
//   one; one barrier per k-step.
// * The reduction range (R x ceil(K/BK) k-steps) can be split over blocks;
//   split partials go to a workspace and are summed in a fixed order, so the
//   result is deterministic.
// * One-dimensional grid, remapped so that each XCD (consecutive workgroup
//   ids go round-robin over the 8 XCDs) receives a contiguous range of output
//   tiles, ordered in bands of 8 tile rows (tile_of), so that the blocks
//   resident on an XCD together share operand panels in its L2.
#pragma once

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "mlcc_internal.h"

namespace mlcc {
namespace gk {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
// 16-byte global loads at element alignment: compute queues run in the
// unaligned access mode, so a 16-byte load needs only in-range bytes, not a
// 16-byte aligned address.
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int kXcd = 8;

// wave grid and thread count of a BM x BN tile
template <int BM, int BN> struct WaveGrid {
  static constexpr int WM = BM % 32 == 0 ? 2 : 1, WN = BN % 32 == 0 ? 2 : 1;
  static constexpr int NT = 64 * WM * WN;
  static_assert(BM % (16 * WM) == 0 && BN % (16 * WN) == 0, "tile");
};

struct KParams {
  GemmArgs a;
  int splits;
  int tiles_m, tiles_n;
  int64_t ktiles, steps_per_split, nwork, per_xcd;
  void *work;  // [splits][Z][M][N] accumulators when splits > 1
  int vec_a, vec_b;  // 16-byte global loads allowed (unit stride)
};

__device__ __forceinline__ int64_t two_level(int64_t i, int64_t lo_n, int64_t s_lo, int64_t s_hi) {
  if (lo_n <= 0) return i * s_lo;
  const int64_t hi = i / lo_n;
  return hi * s_hi + (i - hi * lo_n) * s_lo;
}

template <typename T> struct Tr;
#ifndef MLCC_F64_BK
#define MLCC_F64_BK 16
#endif
template <> struct Tr<double> {
  static constexpr int BK = MLCC_F64_BK, VEC = 2, S = BK / 4;
  typedef d2 v16;   // LDS (16-byte aligned)
  typedef d2u g16;  // global memory (element aligned)
};
template <> struct Tr<float> {
  static constexpr int BK = 32, VEC = 4, S = 8;
  typedef f4 v16;
  typedef f4u g16;
};

// Operand tile of a block: ROWS x COLS in LDS (COLS contiguous), loaded from
// global memory as units of VEC contiguous elements.  KMAJ: the operand's
// contiguous global dimension is its output dimension (m or n), so LDS holds
// [k][m]; otherwise LDS holds [m][k].
template <typename T, int BMN, bool KMAJ, bool VONLY, int NT> struct Stage {
  static constexpr int BK = Tr<T>::BK, VEC = Tr<T>::VEC;
  static constexpr int PK = 16 / (int)sizeof(T);      // [m][k] rows: +16 bytes
  static constexpr int PM = sizeof(T) == 8 ? 4 : 2;   // [k][m] rows: see the bank note
  static constexpr int ROWS = KMAJ ? BK : BMN;
  static constexpr int LEN = KMAJ ? BMN + PM : BK + PK;
  static constexpr int U = BMN * BK / VEC / NT;  // units per thread
  static_assert(U * VEC * NT == BMN * BK, "tile");
  // Bank note: with k = g*S + s, the four k-groups of a [k][m] fragment read
  // sit S rows apart; S * LEN * sizeof(T) is 64 mod 256 (FP32) or 128 mod 256
  // (FP64) for every BMN that is a multiple of 8, so one pass of a ds_read
  // touches disjoint banks.

  int64_t off[U];   // element offset of the unit's first element (valid rows)
  int row[U], col[U];
  bool ok[U];       // output index of the unit's first element in range
  bool vec[U];      // the unit may use one 16-byte load
  bool contig[U];   // KMAJ: the unit's VEC output indices are consecutive in memory
  bool fast;        // every unit of every thread of the block may use 16-byte loads
  int klim[U];      // load_v: leading elements of the unit inside the reduction range
  bool kall;        // load_v: the whole k-step lies inside the reduction range

  // mn0: first output index of the tile; n_mn, lo, s_lo, s_hi: extent and
  // two-level strides of the output dimension.  Units wholly outside the
  // operand read the tile's first row instead: those values reach only
  // outputs that are never written.
  __device__ __forceinline__ void init(int tid, int64_t mn0, int64_t n_mn, int64_t lo, int64_t s_mn,
                                       int64_t s_hi, bool vec_ok) {
    const int64_t off0 = two_level(mn0, lo, s_mn, s_hi);
    bool base_ok = true;
    if (KMAJ) base_ok = mn0 + VEC <= n_mn && (lo <= 0 || (mn0 % lo) + VEC <= lo);
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const int u = tid + e * NT;
      int mn;
      if (KMAJ) {
        row[e] = u / (BMN / VEC);
        mn = (u % (BMN / VEC)) * VEC;
        col[e] = mn;
      } else {
        mn = u / (BK / VEC);
        row[e] = mn;
        col[e] = (u % (BK / VEC)) * VEC;
      }
      const int64_t i = mn0 + mn;
      ok[e] = i < n_mn;
      off[e] = ok[e] ? two_level(i, lo, s_mn, s_hi) : off0;
      if (KMAJ) {
        bool c = i + VEC <= n_mn;
        if (c && lo > 0) c = (i % lo) + VEC <= lo;
        contig[e] = c;
        if (c) vec[e] = vec_ok;
        else vec[e] = vec_ok && !ok[e] && base_ok;  // straddling units are never vectorised
      } else {
        contig[e] = true;
        vec[e] = vec_ok;
      }
    }
    bool all = true;
#pragma unroll
    for (int e = 0; e < U; ++e) all = all && vec[e];
    fast = __syncthreads_and(all) != 0;
  }

  // VONLY: the host has checked that every unit of every tile is a 16-byte
  // group (unit stride, no group cut by the two-level index, and any group
  // that runs past the operand's end inside a library allocation); units
  // outside the operand read the tile's first group and k beyond K is
  // masked, so every load is unconditional.
  __device__ __forceinline__ void init_v(int tid, int64_t mn0, int64_t lo, int64_t s_mn,
                                         int64_t n_mn, int64_t s_hi) {
    const int64_t off0 = two_level(mn0, lo, s_mn, s_hi);
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const int u = tid + e * NT;
      int mn;
      if (KMAJ) {
        row[e] = u / (BMN / VEC);
        mn = (u % (BMN / VEC)) * VEC;
        col[e] = mn;
      } else {
        mn = u / (BK / VEC);
        row[e] = mn;
        col[e] = (u % (BK / VEC)) * VEC;
      }
      const int64_t i = mn0 + mn;
      off[e] = i < n_mn ? two_level(i, lo, s_mn, s_hi) : off0;
    }
  }
  // The loaded values are not masked here: a select on them would make the
  // k-step wait for its loads at once, before the MFMAs of the current step
  // that they are meant to overlap.  klim records how many leading elements
  // of each unit lie inside the reduction range; mask() applies it when the
  // registers go to LDS, after the MFMAs.
  __device__ __forceinline__ void load_v(T (&rg)[U][VEC], const T *X, int64_t k0, int64_t K,
                                         int64_t s_k) {
    typedef typename Tr<T>::g16 v16;
    kall = k0 + BK <= K;
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const int64_t k = k0 + (KMAJ ? row[e] : col[e]);
      const bool in = k < K;
      const int64_t kc = in ? k : 0;
      const T *src = KMAJ ? X + off[e] + kc * s_k : X + off[e] + kc;
      const v16 v = *reinterpret_cast<const v16 *>(src);
#pragma unroll
      for (int q = 0; q < VEC; ++q) rg[e][q] = v[q];
      klim[e] = KMAJ ? (in ? VEC : 0) : (int)min<int64_t>(max<int64_t>(K - k, 0), VEC);
    }
  }
  __device__ __forceinline__ void mask(T (&rg)[U][VEC]) const {
    if (kall) return;  // uniform: every step but a partial last one
#pragma unroll
    for (int e = 0; e < U; ++e)
#pragma unroll
      for (int q = 0; q < VEC; ++q) rg[e][q] = q < klim[e] ? rg[e][q] : T(0);
  }

  // a k-step of the block's interior: every unit in range and aligned, so
  // the loads are unconditional and issue back to back
  __device__ __forceinline__ void load_fast(T (&rg)[U][VEC], const T *X, int64_t k0,
                                            int64_t s_k) const {
    typedef typename Tr<T>::g16 v16;
#pragma unroll
    for (int e = 0; e < U; ++e) {
      const T *src = KMAJ ? X + off[e] + (k0 + row[e]) * s_k : X + off[e] + k0 + col[e];
      const v16 v = *reinterpret_cast<const v16 *>(src);
#pragma unroll
      for (int q = 0; q < VEC; ++q) rg[e][q] = v[q];
    }
  }

  // general k-step (tile edges, a partial last k-step, unaligned operands):
  // element by element, every load unconditional from a valid address (the
  // slice's first element when out of range) and its value selected after,
  // so no branch splits the loads of a step.
  __device__ __forceinline__ void load(T (&rg)[U][VEC], const T *X, int64_t k0, int64_t K,
                                       int64_t s_k, int64_t mn0, int64_t n_mn, int64_t lo,
                                       int64_t s_mn, int64_t s_hi) const {
#pragma unroll
    for (int e = 0; e < U; ++e) {
#pragma unroll
      for (int q = 0; q < VEC; ++q) {
        int64_t o;
        bool valid;
        if (KMAJ) {
          const int64_t k = k0 + row[e];
          const int64_t i = mn0 + col[e] + q;
          valid = k < K && i < n_mn;
          const int64_t oi = contig[e] ? off[e] + q * s_mn : two_level(i, lo, s_mn, s_hi);
          o = valid ? oi + k * s_k : 0;
        } else {
          const int64_t k = k0 + col[e] + q;
          valid = ok[e] && k < K;
          o = valid ? off[e] + k * s_k : 0;
        }
        const T x = X[o];
        rg[e][q] = valid ? x : T(0);
      }
    }
  }

  __device__ __forceinline__ void store(T (*L)[LEN], const T (&rg)[U][VEC]) const {
#pragma unroll
    for (int e = 0; e < U; ++e) {
      T *dst = &L[row[e]][col[e]];
      if (sizeof(T) == 4 && KMAJ) {
        // [k][m] FP32 rows are 8-byte aligned only
        *reinterpret_cast<f2 *>(dst) = f2{(float)rg[e][0], (float)rg[e][1]};
        *reinterpret_cast<f2 *>(dst + 2) = f2{(float)rg[e][2], (float)rg[e][3]};
      } else {
        typename Tr<T>::v16 v;
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[q] = rg[e][q];
        *reinterpret_cast<typename Tr<T>::v16 *>(dst) = v;
      }
    }
  }
};

// fragment (16 rows, S k-values of group g) of an operand tile in LDS
template <typename T, int LEN, bool KMAJ>
__device__ __forceinline__ void frag(T (&f)[Tr<T>::S], const T (*L)[LEN], int mn, int g) {
  constexpr int S = Tr<T>::S;
  if (KMAJ) {
#pragma unroll
    for (int s = 0; s < S; ++s) f[s] = L[g * S + s][mn];
  } else {
    typedef typename Tr<T>::v16 v16;
    constexpr int VEC = Tr<T>::VEC;
#pragma unroll
    for (int h = 0; h < S / VEC; ++h) {
      const v16 v = *reinterpret_cast<const v16 *>(&L[mn][g * S + h * VEC]);
#pragma unroll
      for (int q = 0; q < VEC; ++q) f[h * VEC + q] = v[q];
    }
  }
}

// output position of accumulator element e of lane l within a 16x16 fragment
template <typename T, bool ROTA> struct OutMap;
template <> struct OutMap<float, false> {
  static __device__ __forceinline__ int row(int l, int e) { return 4 * (l >> 4) + e; }
  static __device__ __forceinline__ int col(int l, int) { return l & 15; }
};
template <> struct OutMap<double, false> {
  static __device__ __forceinline__ int row(int l, int) { return 4 * ((l & 15) >> 2) + (l >> 4); }
  static __device__ __forceinline__ int col(int l, int r) {
    return 4 * ((((l & 15) >> 2) + r) & 3) + (l & 3);
  }
};
// A read rotated: block b of instruction r multiplies rows 4((b+r)%4)..+3
// with columns 4b..4b+3
template <> struct OutMap<double, true> {
  static __device__ __forceinline__ int row(int l, int r) {
    return 4 * ((((l & 15) >> 2) + r) & 3) + (l >> 4);
  }
  static __device__ __forceinline__ int col(int l, int) { return 4 * ((l & 15) >> 2) + (l & 3); }
};

// Write a block's accumulators: alpha * acc + beta * Cin into C, or the raw
// partial sums into the split workspace.
template <typename T, typename TC, int FM, int FN, int WTM, int WTN, bool ROTA, typename Acc4>
__device__ __forceinline__ void epilogue(const KParams &kp, const Acc4 (&acc)[FM][FN], int64_t m0,
                                         int64_t n0, int64_t z, int split, int lane, int wm,
                                         int wn) {
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type acc_t;
  const GemmArgs &p = kp.a;
  int64_t coff[FN][4];
  bool cok[FN][4];
#pragma unroll
  for (int j = 0; j < FN; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t col = n0 + wn * WTN + j * 16 + OutMap<T, ROTA>::col(lane, e);
      cok[j][e] = col < p.N;
      coff[j][e] = cok[j][e] ? two_level(col, p.Nlo, p.sCn, p.sCn_hi) : 0;
    }
  if (kp.splits == 1) {
    TC *C = static_cast<TC *>(p.C) + z * p.sCz;
    const TC *Cin = static_cast<const TC *>(p.Cin) + z * p.sCz;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * WTM + i * 16 + OutMap<T, ROTA>::row(lane, e);
        if (row >= p.M) continue;
        const int64_t roff = two_level(row, p.Mlo, p.sCm, p.sCm_hi);
        const double dr = p.den_row ? p.den_row[row] + p.den_shift : 0.0;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (!cok[j][e]) continue;
          const int64_t o = roff + coff[j][e];
          double out = p.alpha * (double)acc[i][j][e];
          if (p.beta != 0.0) out += p.beta * (double)Cin[o];
          if (p.den_row) out /= dr + p.den_col[n0 + wn * WTN + j * 16 + OutMap<T, ROTA>::col(lane, e)];
          C[o] = (TC)out;
        }
      }
  } else {
    acc_t *wk = static_cast<acc_t *>(kp.work) + (((int64_t)split * p.Z + z) * p.M) * p.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * WTM + i * 16 + OutMap<T, ROTA>::row(lane, e);
        if (row >= p.M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int64_t col = n0 + wn * WTN + j * 16 + OutMap<T, ROTA>::col(lane, e);
          if (col < p.N) wk[row * p.N + col] = acc[i][j][e];
        }
      }
  }
}

// Output tile of work item w: (batch, split) planes outermost; inside a plane
// the tiles go in bands of kGroupM tile rows, column by column within a band,
// so that the blocks resident on one XCD at a time (a contiguous range of w)
// share a few A row panels and a few B column panels in that XCD's L2.
constexpr int64_t kGroupM = 8;
__device__ __forceinline__ void tile_of(const KParams &kp, int64_t w, int64_t &tm, int64_t &tn,
                                        int64_t &zs) {
  const int64_t plane = (int64_t)kp.tiles_m * kp.tiles_n;
  zs = w / plane;
  const int64_t q = w - zs * plane, band = kGroupM * kp.tiles_n;
  const int64_t grp = q / band, first = grp * kGroupM;
  const int64_t gm = min(kGroupM, (int64_t)kp.tiles_m - first);
  const int64_t r = q - grp * band;
  tm = first + r % gm;
  tn = r / gm;
}

template <typename T, typename TC, int BM, int BN, bool AKM, bool BKN, bool VONLY>
__global__ __launch_bounds__((WaveGrid<BM, BN>::NT)) void k_gemm(KParams kp) {
  typedef WaveGrid<BM, BN> WG;
  constexpr int S = Tr<T>::S, VEC = Tr<T>::VEC, NT = WG::NT;
  constexpr int WTM = BM / WG::WM, WTN = BN / WG::WN, FM = WTM / 16, FN = WTN / 16;
  constexpr bool ROTA = sizeof(T) == 8 && FM < FN;
  typedef Stage<T, BM, AKM, VONLY, NT> SA;
  typedef Stage<T, BN, BKN, VONLY, NT> SB;
  __shared__ __attribute__((aligned(16))) T As[2][SA::ROWS][SA::LEN];
  __shared__ __attribute__((aligned(16))) T Bs[2][SB::ROWS][SB::LEN];

  const GemmArgs &p = kp.a;
  // XCD-aware work index
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

  const T *Az = static_cast<const T *>(p.A) + z * p.sAz;
  const T *Bz = static_cast<const T *>(p.B) + z * p.sBz;

  SA sa;
  SB sb;
  if constexpr (VONLY) {
    sa.init_v(tid, m0, p.Mlo, p.sAm, p.M, p.sAm_hi);
    sb.init_v(tid, n0, p.Nlo, p.sBn, p.N, p.sBn_hi);
  } else {
    sa.init(tid, m0, p.M, p.Mlo, p.sAm, p.sAm_hi, kp.vec_a);
    sb.init(tid, n0, p.N, p.Nlo, p.sBn, p.sBn_hi, kp.vec_b);
  }

  // FP32: acc[i][j][e] = element e of the 16x16x4 fragment accumulator;
  // FP64: acc[i][j][r] = the 4x4x4 accumulator of rotation r
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type acc_t;
  typedef acc_t acc4 __attribute__((ext_vector_type(4)));
  acc4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc4{0, 0, 0, 0};

  T ra[SA::U][VEC], rb[SB::U][VEC];
  // position (slice r, k0) of the next k-step to load, advanced step by step
  constexpr int BK = Tr<T>::BK;
  int64_t lr = s_begin / kp.ktiles;
  int64_t lk0 = (s_begin - lr * kp.ktiles) * BK;
  auto load_next = [&]() {
    const T *Ar = Az + lr * p.sAr;
    const T *Br = Bz + lr * p.sBr;
    if constexpr (VONLY) {
      sa.load_v(ra, Ar, lk0, p.K, p.sAk);
      sb.load_v(rb, Br, lk0, p.K, p.sBk);
    } else {
      const bool kfull = lk0 + BK <= p.K;
      if (sa.fast && kfull) sa.load_fast(ra, Ar, lk0, p.sAk);
      else sa.load(ra, Ar, lk0, p.K, p.sAk, m0, p.M, p.Mlo, p.sAm, p.sAm_hi);
      if (sb.fast && kfull) sb.load_fast(rb, Br, lk0, p.sBk);
      else sb.load(rb, Br, lk0, p.K, p.sBk, n0, p.N, p.Nlo, p.sBn, p.sBn_hi);
    }
    lk0 += BK;
    if (lk0 >= kp.ktiles * BK) {
      lk0 = 0;
      ++lr;
    }
  };

  auto store_next = [&](int buf) {
    if constexpr (VONLY) {
      sa.mask(ra);
      sb.mask(rb);
    }
    sa.store(As[buf], ra);
    sb.store(Bs[buf], rb);
  };

  int cur = 0;
  if (s_begin < s_end) {
    load_next();
    store_next(0);
  }
  __syncthreads();
  for (int64_t step = s_begin; step < s_end; ++step) {
    const bool more = step + 1 < s_end;
    if (more) load_next();
    if constexpr (sizeof(T) == 4) {
      T af[FM][S];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        frag<T, SA::LEN, AKM>(af[i], As[cur], wm * WTM + i * 16 + l16, g);
      T bf[FN][S];
#pragma unroll
      for (int j = 0; j < FN; ++j)
        frag<T, SB::LEN, BKN>(bf[j], Bs[cur], wn * WTN + j * 16 + l16, g);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s], bf[j][s], acc[i][j], 0, 0, 0);
    } else if constexpr (ROTA) {
      T bf[FN][S];
#pragma unroll
      for (int j = 0; j < FN; ++j)
        frag<T, SB::LEN, BKN>(bf[j], Bs[cur], wn * WTN + j * 16 + l16, g);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          T af[S];
          frag<T, SA::LEN, AKM>(af, As[cur], wm * WTM + i * 16 + ((l16 + 4 * r) & 15), g);
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int j = 0; j < FN; ++j)
              acc[i][j][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[s], bf[j][s], acc[i][j][r], 0, 0, 0);
        }
    } else {
      T af[FM][S];
#pragma unroll
      for (int i = 0; i < FM; ++i)
        frag<T, SA::LEN, AKM>(af[i], As[cur], wm * WTM + i * 16 + l16, g);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          T bf[S];
          frag<T, SB::LEN, BKN>(bf, Bs[cur], wn * WTN + j * 16 + ((l16 + 4 * r) & 15), g);
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int i = 0; i < FM; ++i)
              acc[i][j][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[i][s], bf[s], acc[i][j][r], 0, 0, 0);
        }
    }
    if (more) store_next(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  epilogue<T, TC, FM, FN, WTM, WTN, ROTA>(kp, acc, m0, n0, z, split, lane, wm, wn);
}


// The split-BF16 kernel (FP32 operands on the BF16 matrix cores; PLAIN: one
// product of the operands rounded to BF16); defined in gemm_split.h, which
// the FP32 instantiation units include.
template <typename TC, int BM, int BN, bool PLAIN>
__global__ __launch_bounds__((WaveGrid<BM, BN>::NT)) void k_gemm_split(KParams kp);

template <typename TA, typename TC>
__global__ void k_split_reduce(KParams kp) {
  const GemmArgs &p = kp.a;
  const int64_t MN = p.M * p.N;
  const int64_t total = p.Z * MN;
  const TA *w = static_cast<const TA *>(kp.work);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = t / MN;
    const int64_t rem = t - z * MN;
    const int64_t row = rem / p.N, col = rem - row * p.N;
    double s = 0.0;
    for (int sp = 0; sp < kp.splits; ++sp) s += (double)w[(int64_t)sp * total + t];
    const int64_t off = z * p.sCz + two_level(row, p.Mlo, p.sCm, p.sCm_hi) +
                        two_level(col, p.Nlo, p.sCn, p.sCn_hi);
    double out = p.alpha * s;
    if (p.beta != 0.0) out += p.beta * (double)static_cast<const TC *>(p.Cin)[off];
    if (p.den_row) out /= p.den_row[row] + p.den_col[col] + p.den_shift;
    static_cast<TC *>(p.C)[off] = (TC)out;
  }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// 16-byte loads need a unit-stride contiguous dimension (bounds are checked
// per unit in the kernel).
inline bool vec_ok(int64_t s_fast) { return s_fast == 1; }

// Every unit of one operand is a 16-byte group: unit stride along the
// contiguous dimension and no group cut by a two-level index.  A group may
// run past the operand's last element (an m/n extent or K not a multiple of
// the group) only when the operand lies in a library allocation, which has
// spare bytes past its end: elements past K are masked, elements past M or N
// reach only outputs that are never written.
inline bool operand_vec(bool kmaj, int64_t s_mn, int64_t s_k, int64_t n_mn, int64_t K, int64_t lo,
                        int vec, bool slack) {
  if (kmaj)
    return s_mn == 1 && (lo <= 0 || lo % vec == 0) && (n_mn % vec == 0 || slack);
  return s_k == 1 && (K % vec == 0 || slack);
}

inline bool gemm_vonly(const GemmArgs &a, int vec) {
  const bool akm = std::llabs(a.sAm) < std::llabs(a.sAk);
  const bool bkn = std::llabs(a.sBn) < std::llabs(a.sBk);
  return a.K > 0 && operand_vec(akm, a.sAm, a.sAk, a.M, a.K, a.Mlo, vec, a.slack) &&
         operand_vec(bkn, a.sBn, a.sBk, a.N, a.K, a.Nlo, vec, a.slack);
}

// The split BF16 kernel: vector-only operands that are both k-contiguous.
inline bool gemm_split_ok(const GemmArgs &a) {
  const bool akm = std::llabs(a.sAm) < std::llabs(a.sAk);
  const bool bkn = std::llabs(a.sBn) < std::llabs(a.sBk);
  return a.bf16x3 && !akm && !bkn && gemm_vonly(a, Tr<float>::VEC);
}

// SPLIT: 0 the FP64 / FP32 MFMA kernel, 1 split BF16 products, 2 plain BF16
template <typename T, typename TC, int BM, int BN, bool VONLY, int SPLIT = 0>
void launch_tile(Exec &ex, const GemmArgs &a, int splits) {
  constexpr int BK = Tr<T>::BK, VEC = Tr<T>::VEC;
  KParams kp;
  kp.a = a;
  kp.splits = splits;
  kp.ktiles = cdiv(a.K, BK);
  const int64_t total = a.R * kp.ktiles;
  kp.steps_per_split = cdiv(total, splits);
  kp.tiles_m = (int)cdiv(a.M, BM);
  kp.tiles_n = (int)cdiv(a.N, BN);
  kp.nwork = (int64_t)kp.tiles_m * kp.tiles_n * a.Z * splits;
  kp.per_xcd = cdiv(kp.nwork, kXcd);
  MLCC_REQUIRE(kp.per_xcd * kXcd < (int64_t)1 << 31, MLCC_E_ARG, "gemm: grid too large");
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type acc_t;
  kp.work = nullptr;
  if (splits > 1) {
    const size_t need = sizeof(acc_t) * (size_t)splits * a.Z * a.M * a.N;
    if (a.work) {
      MLCC_REQUIRE(need <= a.work_cap, MLCC_E_ARG, "gemm: split partials exceed the workspace");
      kp.work = a.work;
    } else {
      kp.work = ex.scratch(need);
    }
  }
  // layouts: an operand is staged [k][m] when m has the smaller stride
  const bool akm = std::llabs(a.sAm) < std::llabs(a.sAk);
  const bool bkn = std::llabs(a.sBn) < std::llabs(a.sBk);
  kp.vec_a = vec_ok(akm ? a.sAm : a.sAk);
  kp.vec_b = vec_ok(bkn ? a.sBn : a.sBk);
  const dim3 grid((unsigned)(kp.per_xcd * kXcd)), block(WaveGrid<BM, BN>::NT);
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (ex.prof && ex.prof->on) {
    ev = ex.prof->next();
    MLCC_HIP(hipEventRecord(ev.first, ex.stream));
  }
  if constexpr (SPLIT) {
    static_assert(sizeof(T) == 4, "split products take FP32 operands");
    MLCC_REQUIRE(!akm && !bkn, MLCC_E_ARG, "gemm: split products need k-contiguous operands");
    hipLaunchKernelGGL((k_gemm_split<TC, BM, BN, SPLIT == 2>), grid, block, 0, ex.stream, kp);
  } else if (akm && bkn)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, true, true, VONLY>), grid, block, 0, ex.stream, kp);
  else if (akm)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, true, false, VONLY>), grid, block, 0, ex.stream, kp);
  else if (bkn)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, false, true, VONLY>), grid, block, 0, ex.stream, kp);
  else
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, false, false, VONLY>), grid, block, 0, ex.stream, kp);
  MLCC_HIP(hipGetLastError());
  if (ev.first) {
    MLCC_HIP(hipEventRecord(ev.second, ex.stream));
    ex.prof->recs.push_back({a.tag, ev.first, ev.second,
                             2.0 * (double)a.M * a.N * a.K * a.R * a.Z});
  }
  if (splits > 1) {
    const int64_t n = a.Z * a.M * a.N;
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((k_split_reduce<acc_t, TC>), dim3(blocks), dim3(256), 0, ex.stream, kp);
    MLCC_HIP(hipGetLastError());
  }
}

// Resident blocks per CU of the kernel launch_tile runs for this layout (the
// compiled register and LDS use decide it), queried once per variant.
template <typename T, typename TC, int BM, int BN, bool VONLY, int SPLIT = 0>
int tile_occupancy(const GemmArgs &a) {
  static std::atomic<int> cache[4];
  const bool akm = std::llabs(a.sAm) < std::llabs(a.sAk);
  const bool bkn = std::llabs(a.sBn) < std::llabs(a.sBk);
  const int v = SPLIT ? 0 : (akm ? 2 : 0) + (bkn ? 1 : 0);
  int nb = cache[v].load(std::memory_order_relaxed);
  if (nb > 0) return nb;
  const void *f;
  if constexpr (SPLIT) f = reinterpret_cast<const void *>(&k_gemm_split<TC, BM, BN, SPLIT == 2>);
  else if (akm && bkn) f = reinterpret_cast<const void *>(&k_gemm<T, TC, BM, BN, true, true, VONLY>);
  else if (akm) f = reinterpret_cast<const void *>(&k_gemm<T, TC, BM, BN, true, false, VONLY>);
  else if (bkn) f = reinterpret_cast<const void *>(&k_gemm<T, TC, BM, BN, false, true, VONLY>);
  else f = reinterpret_cast<const void *>(&k_gemm<T, TC, BM, BN, false, false, VONLY>);
  MLCC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, WaveGrid<BM, BN>::NT, 0));
  nb = std::max(nb, 1);
  cache[v].store(nb, std::memory_order_relaxed);
  return nb;
}

// The tile menus: (BM, BN) multiples of 32 (two waves along each
// dimension); the general (element-wise fallback) kernel is built for fewer
// shapes.  Tiles of 80 (one wave along that dimension, FM or FN = 5) were
// measured slower on every contraction here: at one wave per SIMD the MFMA
// pipeline idles more than the padding they save.
#define MLCC_GEMM_TILES_GENERAL(X) \
  X(128, 128) X(128, 64) X(64, 128) X(64, 64) X(128, 32) X(32, 128) X(64, 32) X(32, 64) X(32, 32) \
  X(96, 160)
#define MLCC_GEMM_TILES(X) \
  X(128, 128) X(128, 96) X(96, 128) X(128, 64) X(64, 128) X(96, 96) X(96, 64) X(64, 96) \
  X(64, 64) X(128, 32) X(32, 128) X(96, 32) X(32, 96) X(64, 32) X(32, 64) X(32, 32)    \
  X(96, 160) X(160, 96) X(64, 160) X(160, 64) X(32, 160) X(160, 32)

typedef void (*LaunchFn)(Exec &, const GemmArgs &, int);
typedef int (*OccFn)(const GemmArgs &);
struct Tile {
  int bm, bn;
  LaunchFn fn;
  OccFn occ;
};

// Compute units of the device (queried once; the library runs on one GPU model).
inline int cu_count() {
  static std::atomic<int> n{0};
  int c = n.load(std::memory_order_relaxed);
  if (c > 0) return c;
  int dev = 0;
  MLCC_HIP(hipGetDevice(&dev));
  MLCC_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
  c = std::max(c, 1);
  n.store(c, std::memory_order_relaxed);
  return c;
}

// Forced tile of the lane (mlcc_gemm_tile): index of bm x bn in the menu, or -1.
inline int forced_tile(const Exec &ex, const Tile *tiles, int ntiles) {
  for (int t = 0; t < ntiles; ++t)
    if (tiles[t].bm == ex.force_bm && tiles[t].bn == ex.force_bn) return t;
  return -1;  // none, or one this menu lacks: the cost model decides
}

inline void launch_chosen(Exec &ex, const GemmArgs &a, const Tile &t, int splits) {
  ex.last_bm = t.bm;
  ex.last_bn = t.bn;
  t.fn(ex, a, splits);
}

// With a caller workspace the split count is bounded by what fits in it.
template <typename T> inline int64_t cap_splits(const GemmArgs &a, int64_t s) {
  if (!a.work || s <= 1) return s;
  typedef typename std::conditional<sizeof(T) == 8, double, float>::type acc_t;
  const double per = (double)sizeof(acc_t) * (double)a.Z * (double)a.M * (double)a.N;
  const int64_t fit = (int64_t)std::floor((double)a.work_cap / per);
  return std::max<int64_t>(1, std::min<int64_t>(s, fit));
}

// FP64 MFMA kernels: pick the tile (and split count) with the lowest modelled
// time.  Per k-step a wave issues (bm/32)(bn/32) groups of sixteen 4x4x4
// products of 16 cycles, W cycles in all, and waits about kStepLatency cycles
// (global load, LDS store, barrier, LDS read) that only the other resident
// blocks of its CU can hide: r resident blocks take max(r W, W + kStepLatency)
// cycles per k-step.  r is at most the kernel's occupancy; the split count is
// the largest that keeps every block resident at once; a split reduction adds
// its partial sums' traffic (16 bytes each at ~5 TB/s) and a launch.  On top
// of that, the operand panels every tile streams through L2 (Z R M N K
// sizeof(T) (1/bm + 1/bn) bytes) at about 18 TB/s: the term that separates
// the tiles of large products, fitted to a tile sweep of the 3601 x 5000 x
// 5000 (x 5) doubles-to-singles product, where 96 x 128 runs 13% faster than
// 64 x 64.  The other constants were fitted to tile sweeps of the MLCC2
// Jacobian's contractions (10 to 2800 us) and checked on a 4096^3 product.
// The FP32 kernels keep the load-coefficient model below: on them this one
// picked slower large tiles.
template <typename T, typename TC>
void dispatch(Exec &ex, const GemmArgs &a, const Tile *tiles, int ntiles) {
  constexpr int BK = Tr<T>::BK;
  constexpr double kStepLatency = 3000.0, kClockMHz = 2400.0, kUsPerPartialByte = 0.2e-6;
  constexpr double kL2BytesPerUs = 18e6;
  const int64_t steps = a.R * cdiv(a.K, BK);
  const int64_t ncu = cu_count();
  const int forced = forced_tile(ex, tiles, ntiles);
  int best = -1, best_s = 1;
  double best_us = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    if (forced >= 0 && t != forced) continue;
    const int bm = tiles[t].bm, bn = tiles[t].bn;
    const int64_t occ = tiles[t].occ(a);
    const int64_t blocks = cdiv(a.M, bm) * cdiv(a.N, bn) * a.Z;
    int64_t s = 1;
    if (blocks < occ * ncu && steps >= 8)
      s = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(occ * ncu / blocks, steps / 4), 128));
    s = cap_splits<T>(a, s);
    const int64_t nb = blocks * s;
    const int64_t r = std::min<int64_t>(occ, cdiv(nb, ncu));
    const int64_t rounds = cdiv(nb, ncu * r);
    const double W = 256.0 * (bm / 32) * (bn / 32);
    double us = (double)rounds * (double)cdiv(steps, s) * std::max((double)r * W, W + kStepLatency) / kClockMHz;
    if (s > 1) us += kUsPerPartialByte * 16.0 * (double)s * a.Z * a.M * a.N + 3.0;
    us += (double)a.Z * a.R * a.M * a.N * a.K * sizeof(T) * (1.0 / bm + 1.0 / bn) / kL2BytesPerUs;
    if (best < 0 || us < best_us) {
      best = t;
      best_s = (int)s;
      best_us = us;
    }
  }
  launch_chosen(ex, a, tiles[best], best_s);
}

// FP32 MFMA and split BF16 kernels: pick the tile with the lowest modelled
// time: padded MACs, an operand-load overhead that grows as the tile shrinks
// (coefficient load_coef, 16 for FP32 MFMA), the number of rounds of ~2048
// resident waves, and the split reduction's traffic.  The
// split BF16 kernel takes a larger coefficient: its per-k-step work (the
// hi/lo split, two LDS rows per element) grows with the tile's perimeter, and
// with 48 the model picks the measured best tile on each of the shapes swept
// (a 4096^3 product, the batch-reduced 400 x 160 x 480000, 2250 x 9000 x
// 1200, 14400 x 144 x 14400).
template <typename T, typename TC>
void dispatch_load(Exec &ex, const GemmArgs &a, const Tile *tiles, int ntiles, double load_coef) {
  constexpr int BK = Tr<T>::BK;
  const int64_t steps = a.R * cdiv(a.K, BK);
  auto waves_of = [](int bm, int bn) { return (bm % 32 == 0 ? 2 : 1) * (bn % 32 == 0 ? 2 : 1); };
  // splits: as many as fit one round of ~2048 resident waves.  Rounding up
  // instead would leave a few blocks to run alone in a second round (7 tiles
  // x 74 splits = 518 blocks of 4 waves).
  auto splits_for = [&](int64_t blocks, int nw) {
    const int64_t target = 2048 / nw;
    int s = 1;
    if (blocks < target && steps >= 8) {
      s = (int)std::min<int64_t>(target / blocks, steps / 4);
      s = std::max(1, std::min(s, 128));
    }
    return (int)cap_splits<T>(a, s);
  };
  const int forced = forced_tile(ex, tiles, ntiles);
  int best = -1;
  double best_cost = 0.0;
  for (int t = 0; t < ntiles; ++t) {
    const int bm = tiles[t].bm, bn = tiles[t].bn, nw = waves_of(bm, bn);
    if (forced >= 0 && t != forced) continue;
    const int64_t blocks = cdiv(a.M, bm) * cdiv(a.N, bn) * a.Z;
    const int s = splits_for(blocks, nw);
    const double rounds = std::ceil((double)(blocks * s * nw) / 2048.0);
    const double f = 1.0 + load_coef * (1.0 / bm + 1.0 / bn);
    const double per_block = (double)bm * bn * ((double)cdiv(steps, s) * BK * f + 16.0);
    double cost = rounds * per_block * 4.0 / nw;
    if (s > 1) cost += 2.0 * (double)s * a.Z * a.M * a.N;
    if (best < 0 || cost < best_cost) {
      best = t;
      best_cost = cost;
    }
  }
  const int bm = tiles[best].bm, bn = tiles[best].bn;
  launch_chosen(ex, a, tiles[best], splits_for(cdiv(a.M, bm) * cdiv(a.N, bn) * a.Z, waves_of(bm, bn)));
}

}  // namespace gk

// per operand-type entry points (one translation unit each for the
// vector-only and the general kernels)
void gemm_f64(Exec &ex, const GemmArgs &a);
void gemm_f32(Exec &ex, const GemmArgs &a);
void gemm_f32_out64(Exec &ex, const GemmArgs &a);
void gemm_f64_general(Exec &ex, const GemmArgs &a);
void gemm_f32_general(Exec &ex, const GemmArgs &a);
void gemm_f32_out64_general(Exec &ex, const GemmArgs &a);

}  // namespace mlcc
