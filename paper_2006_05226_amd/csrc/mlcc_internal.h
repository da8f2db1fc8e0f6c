// Internal declarations shared by the translation units of libmlcc.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mlcc.h"
#include "../../include/mlcc_engine.h"

namespace mlcc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
  mlcc_status code;
  std::string msg;
};

#define MLCC_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::mlcc::Error{e_ == hipErrorOutOfMemory ? MLCC_E_OOM : MLCC_E_DEVICE,        \
                          std::string(#expr) + ": " + hipGetErrorString(e_)};            \
  } while (0)

#define MLCC_REQUIRE(cond, code, msg)                          \
  do {                                                         \
    if (!(cond)) throw ::mlcc::Error{(code), std::string(msg)}; \
  } while (0)

// ---------------------------------------------------------------------------
// device memory accounting
// ---------------------------------------------------------------------------
// Device allocations of a context, cached.  Every allocation has kSlack
// readable bytes past its end, so a 16-byte load that runs past a row's last
// element stays inside it; owns() tells whether a pointer lies in a live
// allocation.
//
// Freeing device memory synchronises the whole device, which stalls every
// stream, so blocks are not returned to the device when released but kept:
// * each allocator serves one stream (the context's, or one serving lane's,
//   with the context's allocator as root); a block released on it goes to
//   its own cache and is reused only by it, which stream order makes safe;
// * once the stream has finished all its work (quiesce(), called after the
//   stream is synchronised), its cached blocks become idle in the root,
//   where any allocator may take them;
// * idle blocks are returned to the device only when an allocation would
//   pass the budget or the device is out of memory (trim()), and at the end.
// The root keeps the accounting: used = bytes of live blocks, held = bytes
// taken from the device (live, cached and idle), budget bounds held.
constexpr size_t kSlack = 256;
struct Alloc {
  int device = 0;
  uint64_t budget = 0;  // root: bound on held bytes (0: unlimited)
  uint64_t used = 0;    // root: bytes of live blocks (their capacity)
  uint64_t held = 0;    // root: bytes allocated from the device
  Alloc *root = this;   // a lane's allocator points to the context's
  hipStream_t stream = nullptr;  // the stream this allocator serves
  std::mutex mu;
  std::map<uintptr_t, size_t> live;         // root: base -> capacity
  std::multimap<size_t, void *> cache;      // capacity -> block, released on this stream
  std::multimap<size_t, void *> idle;       // root: capacity -> block no pending work uses
  std::vector<Alloc *> lanes;               // root: the attached lanes' allocators
  void *get(size_t bytes);
  void put(void *p, size_t bytes);
  bool owns(const void *p);
  void quiesce();  // this allocator's stream is idle: cached blocks become idle in the root
  // root: idle blocks back to the device, the largest first, until at least
  // need bytes are freed (0: all of them)
  void trim(size_t need = 0);
  // under memory pressure: wait for this stream, then quiesce and trim
  void reclaim(size_t need = 0);
  // root, when reclaim() did not free enough: every attached lane's cached
  // blocks (and the root's own), each after its stream has finished the work
  // enqueued before, become idle; then trim
  void reclaim_all(size_t need = 0);
  // a block that this allocator's stream no longer needs and that nothing
  // later on this stream is expected to reuse (a one-off staging copy):
  // idle in the root at once, after the stream has finished the work
  // enqueued before, so that every lane may reuse it (or trim free it)
  void put_idle(void *p);
  // root: bytes of its idle blocks and of the blocks cached on its own stream
  // (device memory that reclaim returns on demand)
  size_t reusable();
  void attach(Alloc *lane);  // root: a lane whose cache reclaim_all may empty
  void detach(Alloc *lane);  // root: before the lane's stream is destroyed
  void release_all();  // root, at the end: every cached and idle block back to the device
  Alloc() = default;
  Alloc(const Alloc &) = delete;
  Alloc &operator=(const Alloc &) = delete;
};

// RAII device buffer accounted against an Alloc.
struct DBuf {
  Alloc *al = nullptr;
  void *p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept { *this = std::move(o); }
  DBuf &operator=(DBuf &&o) noexcept {
    if (this != &o) {
      release();
      al = o.al; p = o.p; bytes = o.bytes;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(Alloc *a, size_t nbytes) {
    release();
    al = a;
    bytes = nbytes;
    p = nbytes ? a->get(nbytes) : nullptr;
  }
  // grow-only
  void ensure(Alloc *a, size_t nbytes) {
    if (nbytes > bytes) alloc(a, nbytes);
  }
  void release() {
    if (p && al) al->put(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  void release_idle() {
    if (p && al) al->put_idle(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Event-based timing of GEMM-engine launches, grouped by contraction name.
struct Profiler {
  struct Rec {
    const char *tag;
    hipEvent_t a, b;
    double flops;
  };
  bool on = false;
  std::vector<Rec> recs;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
  std::pair<hipEvent_t, hipEvent_t> next();
  void clear() { recs.clear(); used = 0; }
};

// An execution lane: a stream plus its scratch for split reductions.
// Largest packed operand planes of one BF16 product (larger ones run
// without packing).
constexpr size_t kPlaneBytesMax = (size_t)3 << 30;

struct Exec {
  Profiler *prof = nullptr;
  Alloc *al = nullptr;
  hipStream_t stream = nullptr;
  DBuf work;      // split-K partials
  DBuf red;       // reduction partials (dot products)
  DBuf planes;    // packed BF16 operand planes of the large split / plain BF16 products
  // Packed planes: 0 where the cost rule says they pay, 1 wherever the
  // product allows them, -1 never (tests and tuning); at most planes_cap bytes.
  int planes_mode = 0;
  size_t planes_cap = kPlaneBytesMax;
  double *pinned = nullptr;    // pinned host scalars (512 doubles) for results
  // Tile override of the contraction engine on this lane (parity tests,
  // tuning): a forced bm x bn is used by every call whose menu has it; the
  // tile of the lane's last dispatched call is kept.
  int force_bm = 0, force_bn = 0, last_bm = 0, last_bn = 0;
  // contraction tags that run plain BF16 products under Prec::BF16 (the
  // context's map; set before problems or servers are created)
  const std::vector<std::string> *bf16_map = nullptr;
  void *scratch(size_t bytes) {
    work.ensure(al, bytes);
    return work.p;
  }
};

// ---------------------------------------------------------------------------
// GEMM engine (gemm.hip)
// ---------------------------------------------------------------------------
// F32: FP32 operands on FP32 MFMA; BF16X3: FP32 operands on the BF16 matrix
// cores as hi*hi + hi*lo + lo*hi where the operand layout allows it, FP32
// MFMA elsewhere.
// BF16: as BF16X3, except the contractions named in the lane's BF16 map,
// which run one BF16 product of operands rounded to BF16 (FP32 accumulation).
enum class Prec : int { F64 = 0, F32 = 1, BF16X3 = 2, BF16 = 3 };

struct GemmArgs {
  int64_t M = 0, N = 0, K = 0, R = 1, Z = 1;
  const void *A = nullptr;
  int64_t sAm = 0, sAk = 0, sAr = 0, sAz = 0;
  const void *B = nullptr;
  int64_t sBk = 0, sBn = 0, sBr = 0, sBz = 0;
  const void *Cin = nullptr;  // may alias C; read only if beta != 0
  void *C = nullptr;
  int64_t sCm = 0, sCn = 0, sCz = 0;
  double alpha = 1.0, beta = 0.0;
  const char *tag = "gemm";  // contraction name for the profiler
  // Optional two-level row / column index: when Mlo > 0, row m is
  // (m / Mlo, m % Mlo) and its offset is (m / Mlo) * s_hi + (m % Mlo) * s_lo,
  // where s_lo is the ordinary stride (sAm, sCm) and s_hi is sAm_hi / sCm_hi.
  // Likewise Nlo for columns (sBn, sCn with sBn_hi, sCn_hi).  This lets one
  // launch cover a batch of trial vectors stored back to back.
  int64_t Mlo = 0, sAm_hi = 0, sCm_hi = 0;
  int64_t Nlo = 0, sBn_hi = 0, sCn_hi = 0;
  // set by gemm(): A and B lie in library allocations (kSlack bytes past the end)
  bool slack = false;
  // set by gemm(): FP32 operands may run on the BF16 matrix cores (split products)
  bool bf16x3 = false;
  // set by gemm(): a plain BF16 product (Prec::BF16 and a tag of the BF16 map)
  bool bf16_plain = false;
  // Optional orbital-energy denominator applied in FP64 by the epilogue:
  //   C[m][n] = (alpha * acc + beta * Cin[m][n]) / (den_row[m] + den_col[n] + den_shift)
  // (m, n: output row and column indices, before any two-level mapping).
  const double *den_row = nullptr, *den_col = nullptr;
  double den_shift = 0.0;
  // Caller-provided workspace for split partial sums (work_cap bytes): when
  // set, the engine allocates nothing and uses only as many reduction splits
  // as fit in it.
  void *work = nullptr;
  size_t work_cap = 0;
};

// prec selects the operand type (double or float) and the MFMA; out_f64
// selects the type of C (only meaningful for F32: FP32 operands with an FP32
// accumulator written out as double).
void gemm(Exec &ex, Prec prec, const GemmArgs &a, bool out_f64);


// ---------------------------------------------------------------------------
// element-wise and reduction kernels (kernels.hip)
// ---------------------------------------------------------------------------
namespace k {
// dst[z][r*cols + c] = src[z*sz + (r)*ld + c] for r<rows, c<cols (convert type)
template <typename TD, typename TS>
void pack2d(Exec &ex, TD *dst, const TS *src, int64_t Z, int64_t sz, int64_t rows, int64_t cols,
            int64_t ld);
// dst[z][c*rows + r] = src[z*sz + r*ld + c]   (transposing pack)
template <typename TD, typename TS>
void pack2d_t(Exec &ex, TD *dst, const TS *src, int64_t Z, int64_t sz, int64_t rows,
              int64_t cols, int64_t ld);
template <typename TD, typename TS> void convert(Exec &ex, TD *dst, const TS *src, int64_t n);
// y = a*x + b*y
void axpby(Exec &ex, int64_t n, double a, const double *x, double b, double *y);
void scale(Exec &ex, int64_t n, double a, double *x);
// out = a*x + b*y (element type T, arithmetic in double)
template <typename T>
void lincomb(Exec &ex, int64_t n, double a, const T *x, double b, const T *y, T *out);
void fill(Exec &ex, double *x, int64_t n, double v);
// deterministic dot products into a device scalar array (res[i])
void dot(Exec &ex, int64_t n, const double *x, const double *y, double *res);
template <typename TA, typename TB>
void dot_mixed(Exec &ex, int64_t n, const TA *x, const TB *y, double *res);
// u = 2x - x(i<->j) of full doubles arrays (TU output); nz arrays, x[z] at
// x + z*ldx and u[z] at u + z*ldu.  occ_rows: row (a,i) of u is stored at
// row index i*v + a (columns keep the pair order b*o + j).
template <typename TU>
void u_of(Exec &ex, int o, int v, const double *x, TU *u, int nz = 1, int64_t ldx = 0,
          int64_t ldu = 0, bool occ_rows = false);
// out = G + G^T + d .* c  (M x M, f64 out); G type TG; nz arrays with
// G[z] at G + z*sGz, c[z] at c + z*ldc, out[z] at out + z*ldo
template <typename TG>
void sym_plus_diag(Exec &ex, int64_t M, const TG *G, int64_t ldg, const double *eps_ai,
                   const double *c, double *out, int nz = 1, int64_t sGz = 0, int64_t ldc = 0,
                   int64_t ldo = 0);
// x <- (x + x^T) / 2 in place, nz M x M arrays at x + z*ld
void symmetrize(Exec &ex, int64_t M, double *x, int nz = 1, int64_t ld = 0);
// CC2-level rows of three-level MLCCSD: out = G (+ G^T when addT) + d .* x on
// the entries (ai, bj) with ai or bj outside the CCSD space (a < vt, i < ot);
// the entries with both inside are not touched
template <typename TG>
void cc2_rows(Exec &ex, int64_t M, int o, int ot, int vt, const TG *G, int64_t ldg, bool addT,
              const double *eps_ai, const double *x, int64_t ldx, double *out);
// x[ai][bj] = (G + G^T)[ai][bj] / (w - eps_aibj)  (effective singles); nz arrays
template <typename TG, typename TO>
void sym_div(Exec &ex, int64_t M, const TG *G, int64_t ldg, const double *eps_ai, double w,
             TO *out, int nz = 1, int64_t sGz = 0, int64_t ldo = 0);
// u = 2x - x(i<->j) of an occupied-pair block (rows (i, a), i in [i0, i0+ni);
// columns (j, b), j in [j0, j0+nj); see kernels.hip): u1 the block, u2 (or
// NULL) its transpose, xs (or NULL) x scattered to a full a-major [ai][bj];
// nz blocks at strides sxz (x) and suz (u1, u2)
template <typename TU>
void u_pairblock(Exec &ex, int o, int v, int ni, int nj, const double *x, int64_t ldx,
                 int64_t sxz, TU *u1, int64_t ldu1, TU *u2, int64_t ldu2, int64_t suz, int nz,
                 double *xs, int i0, int j0);
// dst[z*d_z + r*d_r + c] += alpha * src[z*s_z + r*s_r + c*s_c]
template <typename TS>
void acc3d(Exec &ex, int64_t nz, int64_t rows, int64_t cols, double alpha, const TS *src,
           int64_t s_z, int64_t s_r, int64_t s_c, double *dst, int64_t d_z, int64_t d_r);
// Delta t = -Omega / denominators
void qn_step_singles(Exec &ex, int V, int O, const double *eps, const double *om, double *t);
void qn_step_doubles(Exec &ex, int64_t M, const double *eps_ai, const double *om, double *t);
// Davidson preconditioner r / (w - D) with clamp
void precond(Exec &ex, int64_t n1, int64_t M, const double *eps_vo, const double *eps_ai,
             double w, const double *r, double *out);
// eps_ai[a*o+i] = e_a - e_i (active) and eps_vo[A*O+I] = e_A - e_I
void denominators(Exec &ex, int O, int V, int o, int v, const double *eps, double *eps_ai,
                  double *eps_vo);
// d^K = sum_I X^K_II (trace over occupied) , X stacked [J][n][n]
template <typename T>
void occ_trace(Exec &ex, int64_t J, int64_t n, int O, const T *X, double *d);
// singles energy: E1 = 2 sum_K (tr Q^K)^2 - sum_K tr(Q^K Q^K),  Q^K = Lt_oo - L_oo
template <typename T>
void energy_singles(Exec &ex, int64_t J, int64_t n, int O, const T *Lt, const T *L, double *res);
// NaN/Inf check, result count into res (double)
void nonfinite(Exec &ex, int64_t n, const double *x, double *res);
// Omega2 (MLCC2) = g~ + eps_aibj s ; elementwise
template <typename TG>
void mlcc2_omega2(Exec &ex, int64_t M, const TG *g, const double *eps_ai, const double *s,
                  double *out);
// dst[j0][j1][j2][j3] (contiguous, dims n[]) = a * src[sum_k j_k s[k]] + b * dst
template <typename TD, typename TS>
void permute4(Exec &ex, TD *dst, const TS *src, const int64_t n[4], const int64_t s[4], double a,
              double b);
// out += R + R^T (M x M)
void sym_accum(Exec &ex, int64_t M, const double *R, double *out);
// synthetic Cholesky vectors on the device (see MLCC_SYNTH_L in mlcc.h)
void synth_cholesky(Exec &ex, double *L, int64_t J, int64_t n, int O, int V, uint64_t seed);
}  // namespace k

}  // namespace mlcc
