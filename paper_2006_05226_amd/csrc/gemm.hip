// Batched, batch-reduced, strided GEMM on CDNA4 matrix cores (MFMA).
//
//   C_z[m][n] = alpha * sum_{r<R} sum_{k<K} A_zr[m][k] * B_zr[k][n] + beta * Cin_z[m][n]
//
// Every Cholesky-index contraction of the method is one call of this engine:
// the X1 transformation (batched over Cholesky vectors), the Fock exchange
// term (reduced over Cholesky vectors and occupied orbitals), g~_aibj, the
// u-contractions of the Omega vector and the Jacobian terms (batched over
// trial vectors through two-level row/column indices).
//
// Design (64-wide wavefronts, one 16x16 output tile per MFMA):
// * 256 threads = 4 waves in a 2x2 grid; a block owns a BM x BN tile of C and
//   each wave a (BM/2) x (BN/2) sub-tile of (BM/32) x (BN/32) MFMA tiles.
// * FP64: v_mfma_f64_16x16x4_f64; FP32: v_mfma_f32_16x16x4_f32.  Inputs of
//   both: A[i = lane%16][k = lane/16], B[k = lane/16][j = lane%16].  Output
//   element e = 0..3 of a lane is D[i][j = lane%16] with i = 4*(lane/16) + e
//   for FP32 but i = 4*e + lane/16 for FP64 (measured with a one-wave probe).
// * A and B tiles are staged through double-buffered LDS as [k][m] / [k][n]
//   rows, padded so that the four k-rows read by one fragment load fall into
//   different banks; one barrier per k-step.  The next tile's global loads are
//   issued before the MFMAs of the current one.  Global loads are mapped so
//   that consecutive lanes read consecutive addresses along whichever of
//   (m, k) has the smaller stride; per-thread row/column offsets (including
//   the two-level index) are computed once, outside the k loop.
// * The reduction range (R x ceil(K/BK) tile steps) can be split over blocks;
//   split partials go to a workspace and are summed in a fixed order, so the
//   result is deterministic.
#include <cstdlib>

#include "mlcc_internal.h"

namespace mlcc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef d4 vec;
  typedef double acc;
  static __device__ __forceinline__ int row(int lane, int e) { return 4 * e + (lane >> 4); }
  static __device__ __forceinline__ vec op(double a, double b, vec c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mma<float> {
  typedef f4 vec;
  typedef float acc;
  static __device__ __forceinline__ int row(int lane, int e) { return 4 * (lane >> 4) + e; }
  static __device__ __forceinline__ vec op(float a, float b, vec c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// LDS row padding (elements): row stride in bytes = 128 mod 256 (f64) or
// 64 mod 256 (f32), so that the 4 k-rows of a fragment load hit disjoint banks.
template <typename T, int W> struct Pad {
  static constexpr int bytes = W * (int)sizeof(T);
  static constexpr int want = sizeof(T) == 8 ? 128 : 64;
  static constexpr int v = (((want - bytes % 256) % 256) + 256) % 256 / (int)sizeof(T);
};

struct KParams {
  GemmArgs a;
  int splits;
  int64_t steps_per_split;
  int64_t ktiles;
  void *work;  // [splits][Z][M][N] accumulators when splits > 1
};

__device__ __forceinline__ int64_t two_level(int64_t i, int64_t lo_n, int64_t s_lo, int64_t s_hi) {
  if (lo_n <= 0) return i * s_lo;
  const int64_t hi = i / lo_n;
  return hi * s_hi + (i - hi * lo_n) * s_lo;
}

template <typename T, typename TC, int BM, int BN, int BK, bool AKF, bool BKF>
__global__ __launch_bounds__(256) void k_gemm(KParams kp) {
  typedef typename Mma<T>::vec vec;
  typedef typename Mma<T>::acc acc_t;
  constexpr int PA = Pad<T, BM>::v, PB = Pad<T, BN>::v;
  __shared__ T As[2][BK][BM + PA];
  __shared__ T Bs[2][BK][BN + PB];
  constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
  constexpr int AE = BM * BK / 256, BE = BN * BK / 256;
  static_assert(AE * 256 == BM * BK && BE * 256 == BN * BK, "tile");

  const GemmArgs &p = kp.a;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  const int64_t z = blockIdx.z / kp.splits;
  const int split = blockIdx.z % kp.splits;
  const int64_t total = p.R * kp.ktiles;
  const int64_t s_begin = split * kp.steps_per_split;
  const int64_t s_end = min(total, s_begin + kp.steps_per_split);

  const T *Az = static_cast<const T *>(p.A) + z * p.sAz;
  const T *Bz = static_cast<const T *>(p.B) + z * p.sBz;

  // per-thread load coordinates: row/column offsets are fixed for the block
  int64_t aoff[AE], boff[BE];
  int akk[AE], bkk[BE];
  bool aok[AE], bok[BE];
#pragma unroll
  for (int e = 0; e < AE; ++e) {
    const int idx = tid + e * 256;
    const int mm = AKF ? idx / BK : idx % BM;
    akk[e] = AKF ? idx % BK : idx / BM;
    const int64_t m = m0 + mm;
    aok[e] = m < p.M;
    aoff[e] = aok[e] ? two_level(m, p.Mlo, p.sAm, p.sAm_hi) : 0;
  }
#pragma unroll
  for (int e = 0; e < BE; ++e) {
    const int idx = tid + e * 256;
    const int nn = BKF ? idx / BK : idx % BN;
    bkk[e] = BKF ? idx % BK : idx / BN;
    const int64_t n = n0 + nn;
    bok[e] = n < p.N;
    boff[e] = bok[e] ? two_level(n, p.Nlo, p.sBn, p.sBn_hi) : 0;
  }

  vec acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = vec{0, 0, 0, 0};

  T ra[AE], rb[BE];
  auto load = [&](int64_t step) {
    const int64_t r = step / kp.ktiles;
    const int64_t k0 = (step - r * kp.ktiles) * BK;
    const T *Ar = Az + r * p.sAr;
    const T *Br = Bz + r * p.sBr;
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int64_t k = k0 + akk[e];
      ra[e] = (aok[e] && k < p.K) ? Ar[aoff[e] + k * p.sAk] : T(0);
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int64_t k = k0 + bkk[e];
      rb[e] = (bok[e] && k < p.K) ? Br[boff[e] + k * p.sBk] : T(0);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < AE; ++e) {
      const int idx = tid + e * 256;
      const int mm = AKF ? idx / BK : idx % BM;
      As[buf][akk[e]][mm] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < BE; ++e) {
      const int idx = tid + e * 256;
      const int nn = BKF ? idx / BK : idx % BN;
      Bs[buf][bkk[e]][nn] = rb[e];
    }
  };

  int cur = 0;
  if (s_begin < s_end) {
    load(s_begin);
    store(0);
  }
  __syncthreads();
  for (int64_t step = s_begin; step < s_end; ++step) {
    const bool more = step + 1 < s_end;
    if (more) load(step + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[FM], bf[FN];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = As[cur][kr][wm * WTM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = Bs[cur][kr][wn * WTN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mma<T>::op(af[i], bf[j], acc[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

  // epilogue: row and column offsets once per fragment
  int64_t coff[FN];
  bool cok[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int64_t col = n0 + wn * WTN + j * 16 + (lane & 15);
    cok[j] = col < p.N;
    coff[j] = cok[j] ? two_level(col, p.Nlo, p.sCn, p.sCn_hi) : 0;
  }
  if (kp.splits == 1) {
    TC *C = static_cast<TC *>(p.C) + z * p.sCz;
    const TC *Cin = static_cast<const TC *>(p.Cin) + z * p.sCz;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * WTM + i * 16 + Mma<T>::row(lane, e);
        if (row >= p.M) continue;
        const int64_t roff = two_level(row, p.Mlo, p.sCm, p.sCm_hi);
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (!cok[j]) continue;
          const int64_t off = roff + coff[j];
          double out = p.alpha * (double)acc[i][j][e];
          if (p.beta != 0.0) out += p.beta * (double)Cin[off];
          C[off] = (TC)out;
        }
      }
  } else {
    acc_t *w = static_cast<acc_t *>(kp.work) + (((int64_t)split * p.Z + z) * p.M) * p.N;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm * WTM + i * 16 + Mma<T>::row(lane, e);
        if (row >= p.M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          const int64_t col = n0 + wn * WTN + j * 16 + (lane & 15);
          if (col < p.N) w[row * p.N + col] = acc[i][j][e];
        }
      }
  }
}

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
    static_cast<TC *>(p.C)[off] = (TC)out;
  }
}

template <typename T, typename TC, int BM, int BN, int BK>
void launch_tile(Exec &ex, const GemmArgs &a, int splits) {
  KParams kp;
  kp.a = a;
  kp.splits = splits;
  kp.ktiles = (a.K + BK - 1) / BK;
  const int64_t total = a.R * kp.ktiles;
  kp.steps_per_split = (total + splits - 1) / splits;
  typedef typename Mma<T>::acc acc_t;
  kp.work = nullptr;
  if (splits > 1)
    kp.work = ex.scratch(sizeof(acc_t) * (size_t)splits * a.Z * a.M * a.N);
  dim3 grid((unsigned)((a.N + BN - 1) / BN), (unsigned)((a.M + BM - 1) / BM),
            (unsigned)(a.Z * splits));
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  if (ex.prof && ex.prof->on) {
    ev = ex.prof->next();
    MLCC_HIP(hipEventRecord(ev.first, ex.stream));
  }
  // coalescing: let threads run along the smaller stride
  const bool akf = std::llabs(a.sAk) <= std::llabs(a.sAm);
  const bool bkf = std::llabs(a.sBk) <= std::llabs(a.sBn);
  if (akf && bkf)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, BK, true, true>), grid, dim3(256), 0, ex.stream, kp);
  else if (akf)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, BK, true, false>), grid, dim3(256), 0, ex.stream, kp);
  else if (bkf)
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, BK, false, true>), grid, dim3(256), 0, ex.stream, kp);
  else
    hipLaunchKernelGGL((k_gemm<T, TC, BM, BN, BK, false, false>), grid, dim3(256), 0, ex.stream, kp);
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

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, typename TC>
void dispatch(Exec &ex, const GemmArgs &a) {
  constexpr int BK = sizeof(T) == 8 ? 16 : 32;
  // Tile shape: 128 along a dimension that is large, 64 or 32 along a small
  // one; the reduction is split when the tiles alone cannot fill the chip.
  auto pick = [](int64_t x) -> int { return x >= 96 ? 128 : (x >= 48 ? 64 : 32); };
  int bm = pick(a.M), bn = pick(a.N);
  const int64_t steps = a.R * cdiv(a.K, BK);
  // few large tiles and a reduction too short to split: use 64 x 64
  if (bm == 128 && bn == 128 && cdiv(a.M, 128) * cdiv(a.N, 128) * a.Z < 160 && steps < 64)
    bm = bn = 64;
  // tuning knob: MLCC_GEMM_TILE=BMxBN forces the tile of every launch
  static const char *forced = std::getenv("MLCC_GEMM_TILE");
  if (forced) {
    int fm = 0, fn = 0;
    if (std::sscanf(forced, "%dx%d", &fm, &fn) == 2) {
      bm = fm;
      bn = fn;
    }
  }
  const int64_t blocks = cdiv(a.M, bm) * cdiv(a.N, bn) * a.Z;
  int splits = 1;
  const int64_t want = 512;
  if (blocks < want && steps >= 8) {
    splits = (int)std::min<int64_t>(cdiv(want, blocks), steps / 4);
    splits = std::max(1, std::min(splits, 128));
    while (splits > 1 && a.Z * splits > 65535) --splits;
  }
#define MLCC_TILE(BMv, BNv)                          \
  if (bm == BMv && bn == BNv) {                      \
    launch_tile<T, TC, BMv, BNv, BK>(ex, a, splits); \
    return;                                          \
  }
  MLCC_TILE(128, 128)
  MLCC_TILE(128, 64)
  MLCC_TILE(64, 128)
  MLCC_TILE(128, 32)
  MLCC_TILE(32, 128)
  MLCC_TILE(64, 64)
  MLCC_TILE(64, 32)
  MLCC_TILE(32, 64)
#undef MLCC_TILE
  launch_tile<T, TC, 32, 32, BK>(ex, a, splits);
}

}  // namespace

std::pair<hipEvent_t, hipEvent_t> Profiler::next() {
  if (used == pool.size()) {
    hipEvent_t a, b;
    MLCC_HIP(hipEventCreate(&a));
    MLCC_HIP(hipEventCreate(&b));
    pool.push_back({a, b});
  }
  return pool[used++];
}

void gemm(Exec &ex, Prec prec, const GemmArgs &a, bool out_f64) {
  if (a.M <= 0 || a.N <= 0 || a.Z <= 0) return;
  MLCC_REQUIRE(a.Z <= 65535, MLCC_E_ARG, "gemm: batch count above 65535");
  MLCC_REQUIRE((a.M + 31) / 32 <= 65535, MLCC_E_ARG, "gemm: M too large for the grid");
  if (a.K <= 0 || a.R <= 0) {
    // empty reduction: C = beta * Cin (a strided copy / scale); no A, B reads
    GemmArgs b = a;
    b.K = 0;
    b.R = 1;
    b.alpha = 0.0;
    if (prec == Prec::F64) launch_tile<double, double, 32, 32, 16>(ex, b, 1);
    else if (out_f64) launch_tile<float, double, 32, 32, 32>(ex, b, 1);
    else launch_tile<float, float, 32, 32, 32>(ex, b, 1);
    return;
  }
  if (prec == Prec::F64) dispatch<double, double>(ex, a);
  else if (out_f64) dispatch<float, double>(ex, a);
  else dispatch<float, float>(ex, a);
}

}  // namespace mlcc
