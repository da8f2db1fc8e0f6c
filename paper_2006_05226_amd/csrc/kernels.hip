// Element-wise and reduction kernels of the MLCC path: packing of Cholesky
// blocks, the orbital-energy denominator updates of the doubles (Sec. 2.1: the
// MLCC2 doubles equation has the analytic solution s = -g~/eps in the
// semicanonical basis), the u = 2x - x(i<->j) combinations, symmetrisation of
// the doubles part of the Jacobian transformation, quasi-Newton steps, the
// Davidson preconditioner and FP64 dot products.
//
// These are HBM-bound: grid-stride loops with consecutive lanes on consecutive
// addresses; reductions are two-pass with a fixed order (deterministic).
#include <algorithm>

#include "mlcc_internal.h"

namespace mlcc {
namespace k {
namespace {

constexpr int TPB = 256;

inline unsigned blocks_for(int64_t n, int64_t cap = 16384) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

#define GRID_STRIDE(i, n)                                                   \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

template <typename TD, typename TS>
__global__ void k_pack2d(TD *dst, const TS *src, int64_t Z, int64_t sz, int64_t rows,
                         int64_t cols, int64_t ld) {
  const int64_t per = rows * cols;
  GRID_STRIDE(t, Z * per) {
    const int64_t z = t / per, rem = t - z * per;
    const int64_t r = rem / cols, c = rem - r * cols;
    dst[t] = (TD)src[z * sz + r * ld + c];
  }
}

// transposing pack through a 32x32 LDS tile per (z, tile)
template <typename TD, typename TS>
__global__ void k_pack2d_t(TD *dst, const TS *src, int64_t sz, int64_t rows, int64_t cols,
                           int64_t ld) {
  __shared__ TD tile[32][33];
  const int64_t z = blockIdx.z;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, c = c0 + tx;
    if (r < rows && c < cols) tile[y][tx] = (TD)src[z * sz + r * ld + c];
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t c = c0 + y, r = r0 + tx;
    if (r < rows && c < cols) dst[z * rows * cols + c * rows + r] = tile[tx][y];
  }
}

template <typename TD, typename TS>
__global__ void k_convert(TD *dst, const TS *src, int64_t n) {
  GRID_STRIDE(i, n) dst[i] = (TD)src[i];
}

__global__ void k_axpby(int64_t n, double a, const double *x, double b, double *y) {
  GRID_STRIDE(i, n) y[i] = a * x[i] + b * y[i];
}
template <typename T>
__global__ void k_lincomb(int64_t n, double a, const T *x, double b, const T *y, T *out) {
  GRID_STRIDE(i, n) out[i] = (T)(a * (double)x[i] + b * (double)y[i]);
}
__global__ void k_scale(int64_t n, double a, double *x) {
  GRID_STRIDE(i, n) x[i] *= a;
}
__global__ void k_fill(double *x, int64_t n, double v) {
  GRID_STRIDE(i, n) x[i] = v;
}

// block-level sum in fixed order
__device__ double block_sum(double v) {
  __shared__ double sh[TPB];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename TA, typename TB>
__global__ void k_dot_partial(int64_t n, const TA *x, const TB *y, double *part) {
  double s = 0.0;
  GRID_STRIDE(i, n) s += (double)x[i] * (double)y[i];
  const double b = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}
__global__ void k_sum_final(int nb, const double *part, double *res) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += TPB) s += part[i];
  const double b = block_sum(s);
  if (threadIdx.x == 0) *res = b;
}

__global__ void k_nonfinite_partial(int64_t n, const double *x, double *part) {
  double s = 0.0;
  GRID_STRIDE(i, n) s += (isfinite(x[i]) ? 0.0 : 1.0);
  const double b = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

template <typename TU>
__global__ void k_u_of(int o, int v, const double *x, TU *u, int nz, int64_t ldx, int64_t ldu,
                       bool occ_rows) {
  const int64_t M = (int64_t)o * v, MM = M * M;
  GRID_STRIDE(tt, MM * nz) {
    const int64_t z = tt / MM, t = tt - z * MM;
    const int64_t ai = t / M, bj = t - ai * M;
    const int64_t a = ai / o, i = ai - a * o, b = bj / o, j = bj - b * o;
    const double *xz = x + z * ldx;
    const int64_t row = occ_rows ? i * v + a : ai;
    u[z * ldu + row * M + bj] = (TU)(2.0 * xz[t] - xz[(a * o + j) * M + (b * o + i)]);
  }
}

// The same through LDS: a workgroup takes the o x (nb*o) slab of rows (a, i)
// and columns (b, j) for nb consecutive b, where both x_aibj and x_ajbi live,
// so the loads and the stores run along contiguous (b, j).
template <typename TU>
__global__ void k_u_of_tiled(int o, int v, const double *x, TU *u, int64_t ldx, int64_t ldu,
                             bool occ_rows, int bchunk) {
  extern __shared__ double slab[];  // [o][bchunk*o + 1]
  const int64_t M = (int64_t)o * v;
  const int S = bchunk * o + 1;
  const int z = blockIdx.z, a = blockIdx.y, b0 = blockIdx.x * bchunk;
  const int nb = min(bchunk, v - b0);
  const int W = nb * o;
  const double *xz = x + z * ldx;
  TU *uz = u + z * ldu;
  for (int t = threadIdx.x; t < o * W; t += blockDim.x) {
    const int i = t / W, c = t - i * W;
    slab[i * S + c] = xz[((int64_t)a * o + i) * M + (int64_t)b0 * o + c];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < o * W; t += blockDim.x) {
    const int i = t / W, c = t - i * W;
    const int bl = c / o, j = c - bl * o;
    const double val = 2.0 * slab[i * S + c] - slab[j * S + bl * o + i];
    const int64_t row = occ_rows ? (int64_t)i * v + a : (int64_t)a * o + i;
    uz[row * M + (int64_t)b0 * o + c] = (TU)val;
  }
}

// u = 2x - x(i<->j) on one occupied-pair block of a doubles array.  The block
// holds rows (i, a) for i in an occupied range I (row (i - i0) v + a) and
// columns (j, b) for j in a range J (column (j - j0) v + b).  x_ajbi = x_biaj
// lies in the same block, at row (i, b) and column (j, a), so each v x v
// sub-block (i, j) is combined with its own transpose: u_ij = 2 x_ij - x_ij^T.
// A workgroup takes a 32 x 32 tile of a sub-block and the mirrored tile into
// LDS, so that loads and stores run along contiguous addresses.  u1 receives
// the block (rows (i, a), leading dimension ldu1); u2, unless NULL, the
// mirrored block (J, I) of the symmetric u, u2 = u1^T (rows (j, b), ldu2).
// xs, unless NULL, receives x itself at its a-major place in a full [ai][bj]
// array (ai = a o + i) and the mirrored place.
template <typename TU>
__global__ void k_u_pairblock(int o, int v, int nj, const double *x, int64_t ldx, int64_t sxz,
                              TU *u1, int64_t ldu1, TU *u2, int64_t ldu2, int64_t suz,
                              double *xs, int i0, int j0) {
  __shared__ double t1[32][33], t2[32][33];
  const int nt = (v + 31) / 32;
  const int ta = blockIdx.x / nt, tb = blockIdx.x - ta * nt;
  const int il = blockIdx.y / nj, jl = blockIdx.y - il * nj;
  const int64_t z = blockIdx.z;
  x += z * sxz;
  u1 += z * suz;
  if (u2) u2 += z * suz;
  const int a0 = ta * 32, b0 = tb * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t rI = (int64_t)il * v, cJ = (int64_t)jl * v;
  // t1[a][b] = x[(i, a)][(j, b)],  t2[b][a] = x[(i, b)][(j, a)]
  for (int y = ty; y < 32; y += 8) {
    const int a = a0 + y, b = b0 + tx;
    t1[y][tx] = (a < v && b < v) ? x[(rI + a) * ldx + cJ + b] : 0.0;
    const int bb = b0 + y, aa = a0 + tx;
    t2[y][tx] = (bb < v && aa < v) ? x[(rI + bb) * ldx + cJ + aa] : 0.0;
  }
  __syncthreads();
  const int64_t M = (int64_t)o * v;
  const int i = i0 + il, j = j0 + jl;
  for (int y = ty; y < 32; y += 8) {
    const int a = a0 + y, b = b0 + tx;
    if (a < v && b < v) {
      u1[(rI + a) * ldu1 + cJ + b] = (TU)(2.0 * t1[y][tx] - t2[tx][y]);
      if (xs) {
        xs[((int64_t)a * o + i) * M + (int64_t)b * o + j] = t1[y][tx];
        xs[((int64_t)b * o + j) * M + (int64_t)a * o + i] = t1[y][tx];
      }
    }
  }
  if (u2) {
    for (int y = ty; y < 32; y += 8) {
      const int b = b0 + y, a = a0 + tx;
      if (a < v && b < v) u2[(cJ + b) * ldu2 + rI + a] = (TU)(2.0 * t1[tx][y] - t2[y][tx]);
    }
  }
}

template <typename TS>
__global__ void k_acc3d(int64_t nz, int64_t rows, int64_t cols, double alpha, const TS *src,
                        int64_t s_z, int64_t s_r, int64_t s_c, double *dst, int64_t d_z,
                        int64_t d_r) {
  const int64_t per = rows * cols;
  GRID_STRIDE(t, nz * per) {
    const int64_t z = t / per, rc = t - z * per, r = rc / cols, c = rc - r * cols;
    dst[z * d_z + r * d_r + c] += alpha * (double)src[z * s_z + r * s_r + c * s_c];
  }
}

// out = G + G^T + eps_aibj * c  through 32x32 LDS tiles (coalesced transpose)
template <typename TG>
__global__ void k_sym_plus_diag(int64_t M, const TG *G, int64_t ldg, const double *eps_ai,
                                const double *c, double *out, int64_t sGz, int64_t ldc,
                                int64_t ldo) {
  __shared__ double tile[32][33];
  G += blockIdx.z * sGz;
  if (c) c += blockIdx.z * ldc;
  out += blockIdx.z * ldo;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // load G[c0.., r0..] transposed into tile
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = c0 + y, cc = r0 + tx;
    tile[y][tx] = (rr < M && cc < M) ? (double)G[rr * ldg + cc] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, cc = c0 + tx;
    if (r < M && cc < M) {
      const int64_t off = r * M + cc;
      double v = (double)G[r * ldg + cc] + tile[tx][y];
      if (c) v += (eps_ai[r] + eps_ai[cc]) * c[off];
      out[off] = v;
    }
  }
}

// x <- (x + x^T) / 2 in place for nz M x M arrays at x + z*ld: each unordered
// pair (p, q), p < q, belongs to one thread.
__global__ void k_symmetrize(int64_t M, double *x, int nz, int64_t ld) {
  const int64_t per = M * M, total = per * nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t z = t / per, e = t - z * per, p = e / M, q = e - p * M;
    if (p >= q) continue;
    double *xz = x + z * ld;
    const double a = 0.5 * (xz[p * M + q] + xz[q * M + p]);
    xz[p * M + q] = a;
    xz[q * M + p] = a;
  }
}

// CC2-level rows of three-level MLCCSD: out[ai][bj] = G[ai][bj] (+ G[bj][ai]
// when addT) + eps_aibj x[ai][bj] for every pair of pairs not both inside the
// CCSD space (a < vt and i < ot; pair index a*o + i); the other entries are
// left alone.  32x32 LDS tiles as in k_sym_plus_diag.
template <typename TG>
__global__ void k_cc2_rows(int64_t M, int o, int ot, int vt, const TG *G, int64_t ldg, int addT,
                           const double *eps_ai, const double *x, int64_t ldx, double *out) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (addT) {
    for (int y = ty; y < 32; y += 8) {
      const int64_t rr = c0 + y, cc = r0 + tx;
      tile[y][tx] = (rr < M && cc < M) ? (double)G[rr * ldg + cc] : 0.0;
    }
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, cc = c0 + tx;
    if (r < M && cc < M) {
      const bool rin = r / o < vt && r % o < ot, cin = cc / o < vt && cc % o < ot;
      if (rin && cin) continue;
      double v = (double)G[r * ldg + cc];
      if (addT) v += tile[tx][y];
      out[r * M + cc] = v + (eps_ai[r] + eps_ai[cc]) * x[r * ldx + cc];
    }
  }
}

template <typename TG, typename TO>
__global__ void k_sym_div(int64_t M, const TG *G, int64_t ldg, const double *eps_ai, double w,
                          TO *out, int64_t sGz, int64_t ldo) {
  __shared__ double tile[32][33];
  G += blockIdx.z * sGz;
  out += blockIdx.z * ldo;
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = c0 + y, cc = r0 + tx;
    tile[y][tx] = (rr < M && cc < M) ? (double)G[rr * ldg + cc] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, cc = c0 + tx;
    if (r < M && cc < M) {
      const int64_t off = r * M + cc;
      out[off] = (TO)(((double)G[r * ldg + cc] + tile[tx][y]) / (w - (eps_ai[r] + eps_ai[cc])));
    }
  }
}

template <typename TG>
__global__ void k_mlcc2_omega2(int64_t M, const TG *g, const double *eps_ai, const double *s,
                               double *out) {
  GRID_STRIDE(t, M * M) {
    const int64_t ai = t / M, bj = t - ai * M;
    out[t] = (double)g[t] + (eps_ai[ai] + eps_ai[bj]) * s[t];
  }
}

__global__ void k_qn_singles(int V, int O, const double *eps, const double *om, double *t) {
  GRID_STRIDE(x, (int64_t)V * O) {
    const int64_t A = x / O, I = x - A * O;
    t[x] -= om[x] / (eps[O + A] - eps[I]);
  }
}
__global__ void k_qn_doubles(int64_t M, const double *eps_ai, const double *om, double *t) {
  GRID_STRIDE(x, M * M) {
    const int64_t ai = x / M, bj = x - ai * M;
    t[x] -= om[x] / (eps_ai[ai] + eps_ai[bj]);
  }
}

__global__ void k_precond(int64_t n1, int64_t M, const double *eps_vo, const double *eps_ai,
                          double w, const double *r, double *out) {
  GRID_STRIDE(x, n1 + M * M) {
    double d;
    if (x < n1) {
      d = eps_vo[x];
    } else {
      const int64_t y = x - n1, ai = y / M, bj = y - ai * M;
      d = eps_ai[ai] + eps_ai[bj];
    }
    double den = w - d;
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    out[x] = r[x] / den;
  }
}

__global__ void k_denominators(int O, int V, int o, int v, const double *eps, double *eps_ai,
                               double *eps_vo) {
  GRID_STRIDE(x, (int64_t)V * O) {
    const int64_t A = x / O, I = x - A * O;
    eps_vo[x] = eps[O + A] - eps[I];
  }
  GRID_STRIDE(x, (int64_t)v * o) {
    const int64_t a = x / o, i = x - a * o;
    eps_ai[x] = eps[O + a] - eps[i];
  }
}

template <typename T>
__global__ void k_occ_trace(int64_t J, int64_t n, int O, const T *X, double *d) {
  GRID_STRIDE(K, J) {
    double s = 0.0;
    const T *x = X + K * n * n;
    for (int I = 0; I < O; ++I) s += (double)x[(int64_t)I * n + I];
    d[K] = s;
  }
}

// per Cholesky vector: 2 (tr Q)^2 - tr(Q Q), Q = Lt_oo - L_oo; one block per K
template <typename T>
__global__ void k_energy_singles(int64_t n, int O, const T *Lt, const T *L, double *part) {
  const int64_t K = blockIdx.x;
  const T *a = Lt + K * n * n;
  const T *b = L + K * n * n;
  double tr = 0.0, qq = 0.0;
  for (int64_t x = threadIdx.x; x < (int64_t)O * O; x += TPB) {
    const int64_t I = x / O, J = x - I * O;
    const double qij = (double)a[I * n + J] - (double)b[I * n + J];
    const double qji = (double)a[J * n + I] - (double)b[J * n + I];
    qq += qij * qji;
    if (I == J) tr += qij;
  }
  const double trs = block_sum(tr);
  __syncthreads();
  const double qqs = block_sum(qq);
  if (threadIdx.x == 0) part[K] = 2.0 * trs * trs - qqs;
}

// Tile geometry of k_permute4_tiled: extents of dst dimension 3 and d (the
// one along which src is contiguous) and of the outer pair (a, b), their
// src strides (s*) and dst strides (d*), tile counts along 3 and d.
struct P4 {
  int64_t n3, nd, nb, t3, td;
  int64_t s3, sd, sa, sb;
  int64_t dd, da, db;
};

// dst[j0][j1][j2][j3] (contiguous, dims n0..n3) = a * src[sum j_k s_k] + b * dst
// Element by element in dst order (IT: the index type, 32-bit when the
// array allows it); coalesced on both sides when s3 is 1.
template <typename TD, typename TS, typename IT>
__global__ void k_permute4(TD *dst, const TS *src, IT n0, IT n1, IT n2, IT n3, int64_t s0,
                           int64_t s1, int64_t s2, int64_t s3, double a, double b) {
  const IT total = n0 * n1 * n2 * n3;
  for (IT t = (IT)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (IT)gridDim.x * blockDim.x) {
    IT r = t;
    const IT j3 = r % n3;
    r /= n3;
    const IT j2 = r % n2;
    r /= n2;
    const IT j1 = r % n1;
    const IT j0 = r / n1;
    double v = a * (double)src[j0 * s0 + j1 * s1 + j2 * s2 + j3 * s3];
    if (b != 0.0) v += b * (double)dst[t];
    dst[t] = (TD)v;
  }
}

// The same when src is contiguous along dst dimension d < 3 instead: 32 x 32
// tiles over (j_d, j3) through LDS, read along j_d and written along j3, so
// that both sides are coalesced.  Block q: tile (q3, qd) of the pair of
// indices (ja, jb) over the other two dimensions (a < b).
template <typename TD, typename TS>
__global__ __launch_bounds__(256) void k_permute4_tiled(TD *dst, const TS *src, P4 p, double a,
                                                          double b) {
  __shared__ double tile[32][33];
  int64_t q = blockIdx.x;
  const int64_t q3 = q % p.t3;
  q /= p.t3;
  const int64_t qd = q % p.td;
  q /= p.td;
  const int64_t jb = q % p.nb, ja = q / p.nb;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t sbase = ja * p.sa + jb * p.sb, dbase = ja * p.da + jb * p.db;
  const int64_t jd0 = qd * 32, j30 = q3 * 32;
#pragma unroll
  for (int k = ty; k < 32; k += 8) {
    const int64_t j3 = j30 + k, jd = jd0 + tx;
    if (j3 < p.n3 && jd < p.nd) tile[k][tx] = (double)src[sbase + jd * p.sd + j3 * p.s3];
  }
  __syncthreads();
#pragma unroll
  for (int k = ty; k < 32; k += 8) {
    const int64_t jd = jd0 + k, j3 = j30 + tx;
    if (j3 < p.n3 && jd < p.nd) {
      const int64_t o = dbase + jd * p.dd + j3;
      double v = a * tile[tx][k];
      if (b != 0.0) v += b * (double)dst[o];
      dst[o] = (TD)v;
    }
  }
}

// out += R + R^T  (M x M) through 32x32 LDS tiles
__global__ void k_sym_accum(int64_t M, const double *R, double *out) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = c0 + y, cc = r0 + tx;
    tile[y][tx] = (rr < M && cc < M) ? R[rr * M + cc] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int64_t r = r0 + y, cc = c0 + tx;
    if (r < M && cc < M) out[r * M + cc] += R[r * M + cc] + tile[tx][y];
  }
}

}  // namespace

template <typename TD, typename TS>
void pack2d(Exec &ex, TD *dst, const TS *src, int64_t Z, int64_t sz, int64_t rows, int64_t cols,
            int64_t ld) {
  const int64_t n = Z * rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL((k_pack2d<TD, TS>), dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, dst, src,
                     Z, sz, rows, cols, ld);
  MLCC_HIP(hipGetLastError());
}

template <typename TD, typename TS>
void pack2d_t(Exec &ex, TD *dst, const TS *src, int64_t Z, int64_t sz, int64_t rows, int64_t cols,
              int64_t ld) {
  if (Z * rows * cols <= 0) return;
  MLCC_REQUIRE(Z <= 65535, MLCC_E_ARG, "pack2d_t: batch too large");
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32), (unsigned)Z);
  hipLaunchKernelGGL((k_pack2d_t<TD, TS>), grid, dim3(256), 0, ex.stream, dst, src, sz, rows,
                     cols, ld);
  MLCC_HIP(hipGetLastError());
}

template <typename TD, typename TS> void convert(Exec &ex, TD *dst, const TS *src, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert<TD, TS>), dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, dst, src,
                     n);
  MLCC_HIP(hipGetLastError());
}

void axpby(Exec &ex, int64_t n, double a, const double *x, double b, double *y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, n, a, x, b, y);
  MLCC_HIP(hipGetLastError());
}
template <typename T>
void lincomb(Exec &ex, int64_t n, double a, const T *x, double b, const T *y, T *out) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_lincomb<T>), dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, n, a, x, b, y,
                     out);
  MLCC_HIP(hipGetLastError());
}
template void lincomb<double>(Exec &, int64_t, double, const double *, double, const double *,
                              double *);
template void lincomb<float>(Exec &, int64_t, double, const float *, double, const float *,
                             float *);
void scale(Exec &ex, int64_t n, double a, double *x) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, n, a, x);
  MLCC_HIP(hipGetLastError());
}
void fill(Exec &ex, double *x, int64_t n, double v) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(TPB), 0, ex.stream, x, n, v);
  MLCC_HIP(hipGetLastError());
}

static double *red_part(Exec &ex, int nb) {
  ex.red.ensure(ex.al, sizeof(double) * (size_t)(nb + 8));
  return ex.red.as<double>();
}

template <typename TA, typename TB>
void dot_mixed(Exec &ex, int64_t n, const TA *x, const TB *y, double *res) {
  const unsigned nb = blocks_for(n, 1024);
  double *part = red_part(ex, nb);
  hipLaunchKernelGGL((k_dot_partial<TA, TB>), dim3(nb), dim3(TPB), 0, ex.stream, n, x, y, part);
  MLCC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, ex.stream, (int)nb, part, res);
  MLCC_HIP(hipGetLastError());
}
void dot(Exec &ex, int64_t n, const double *x, const double *y, double *res) {
  dot_mixed<double, double>(ex, n, x, y, res);
}

void nonfinite(Exec &ex, int64_t n, const double *x, double *res) {
  const unsigned nb = blocks_for(n, 1024);
  double *part = red_part(ex, nb);
  hipLaunchKernelGGL(k_nonfinite_partial, dim3(nb), dim3(TPB), 0, ex.stream, n, x, part);
  MLCC_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, ex.stream, (int)nb, part, res);
  MLCC_HIP(hipGetLastError());
}

template <typename TU>
void u_of(Exec &ex, int o, int v, const double *x, TU *u, int nz, int64_t ldx, int64_t ldu,
          bool occ_rows) {
  const int64_t M = (int64_t)o * v;
  if (M == 0 || nz <= 0) return;
  if (o <= 64 && v <= 65535 && nz <= 65535) {
    // slabs of at most 4096 doubles (+ padding) of LDS
    const int bchunk = std::max(1, std::min(v, 4096 / (o * o)));
    const size_t lds = (size_t)o * (bchunk * o + 1) * sizeof(double);
    const dim3 grid((unsigned)((v + bchunk - 1) / bchunk), (unsigned)v, (unsigned)nz);
    hipLaunchKernelGGL((k_u_of_tiled<TU>), grid, dim3(TPB), lds, ex.stream, o, v, x, u,
                       nz > 1 ? ldx : 0, nz > 1 ? ldu : 0, occ_rows, bchunk);
  } else {
    hipLaunchKernelGGL((k_u_of<TU>), dim3(blocks_for(M * M * nz)), dim3(TPB), 0, ex.stream, o, v,
                       x, u, nz, ldx, ldu, occ_rows);
  }
  MLCC_HIP(hipGetLastError());
}

template <typename TU>
void u_pairblock(Exec &ex, int o, int v, int ni, int nj, const double *x, int64_t ldx,
                 int64_t sxz, TU *u1, int64_t ldu1, TU *u2, int64_t ldu2, int64_t suz, int nz,
                 double *xs, int i0, int j0) {
  if (v <= 0 || ni <= 0 || nj <= 0 || nz <= 0) return;
  const int64_t nt = (v + 31) / 32;
  MLCC_REQUIRE(nt * nt <= 2147483647 && (int64_t)ni * nj <= 65535 && nz <= 65535, MLCC_E_ARG,
               "u_pairblock: block too large");
  const dim3 grid((unsigned)(nt * nt), (unsigned)(ni * nj), (unsigned)nz);
  hipLaunchKernelGGL((k_u_pairblock<TU>), grid, dim3(256), 0, ex.stream, o, v, nj, x, ldx, sxz,
                     u1, ldu1, u2, ldu2, suz, xs, i0, j0);
  MLCC_HIP(hipGetLastError());
}

template <typename TS>
void acc3d(Exec &ex, int64_t nz, int64_t rows, int64_t cols, double alpha, const TS *src,
           int64_t s_z, int64_t s_r, int64_t s_c, double *dst, int64_t d_z, int64_t d_r) {
  if (nz <= 0 || rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL((k_acc3d<TS>), dim3(blocks_for(nz * rows * cols)), dim3(TPB), 0, ex.stream,
                     nz, rows, cols, alpha, src, s_z, s_r, s_c, dst, d_z, d_r);
  MLCC_HIP(hipGetLastError());
}

template <typename TG>
void sym_plus_diag(Exec &ex, int64_t M, const TG *G, int64_t ldg, const double *eps_ai,
                   const double *c, double *out, int nz, int64_t sGz, int64_t ldc, int64_t ldo) {
  if (M == 0 || nz <= 0) return;
  dim3 grid((unsigned)((M + 31) / 32), (unsigned)((M + 31) / 32), (unsigned)nz);
  hipLaunchKernelGGL((k_sym_plus_diag<TG>), grid, dim3(256), 0, ex.stream, M, G, ldg, eps_ai, c,
                     out, sGz, ldc, ldo);
  MLCC_HIP(hipGetLastError());
}

void symmetrize(Exec &ex, int64_t M, double *x, int nz, int64_t ld) {
  if (M == 0 || nz <= 0) return;
  hipLaunchKernelGGL(k_symmetrize, dim3(blocks_for(M * M * nz)), dim3(TPB), 0, ex.stream, M, x,
                     nz, ld);
  MLCC_HIP(hipGetLastError());
}

template <typename TG>
void cc2_rows(Exec &ex, int64_t M, int o, int ot, int vt, const TG *G, int64_t ldg, bool addT,
              const double *eps_ai, const double *x, int64_t ldx, double *out) {
  if (M == 0 || o <= 0) return;
  dim3 grid((unsigned)((M + 31) / 32), (unsigned)((M + 31) / 32));
  hipLaunchKernelGGL((k_cc2_rows<TG>), grid, dim3(256), 0, ex.stream, M, o, ot, vt, G, ldg,
                     addT ? 1 : 0, eps_ai, x, ldx, out);
  MLCC_HIP(hipGetLastError());
}

template <typename TG, typename TO>
void sym_div(Exec &ex, int64_t M, const TG *G, int64_t ldg, const double *eps_ai, double w,
             TO *out, int nz, int64_t sGz, int64_t ldo) {
  if (M == 0 || nz <= 0) return;
  dim3 grid((unsigned)((M + 31) / 32), (unsigned)((M + 31) / 32), (unsigned)nz);
  hipLaunchKernelGGL((k_sym_div<TG, TO>), grid, dim3(256), 0, ex.stream, M, G, ldg, eps_ai, w,
                     out, sGz, ldo);
  MLCC_HIP(hipGetLastError());
}

template <typename TG>
void mlcc2_omega2(Exec &ex, int64_t M, const TG *g, const double *eps_ai, const double *s,
                  double *out) {
  if (M == 0) return;
  hipLaunchKernelGGL((k_mlcc2_omega2<TG>), dim3(blocks_for(M * M)), dim3(TPB), 0, ex.stream, M,
                     g, eps_ai, s, out);
  MLCC_HIP(hipGetLastError());
}

void qn_step_singles(Exec &ex, int V, int O, const double *eps, const double *om, double *t) {
  hipLaunchKernelGGL(k_qn_singles, dim3(blocks_for((int64_t)V * O)), dim3(TPB), 0, ex.stream, V,
                     O, eps, om, t);
  MLCC_HIP(hipGetLastError());
}
void qn_step_doubles(Exec &ex, int64_t M, const double *eps_ai, const double *om, double *t) {
  if (M == 0) return;
  hipLaunchKernelGGL(k_qn_doubles, dim3(blocks_for(M * M)), dim3(TPB), 0, ex.stream, M, eps_ai,
                     om, t);
  MLCC_HIP(hipGetLastError());
}
void precond(Exec &ex, int64_t n1, int64_t M, const double *eps_vo, const double *eps_ai,
             double w, const double *r, double *out) {
  hipLaunchKernelGGL(k_precond, dim3(blocks_for(n1 + M * M)), dim3(TPB), 0, ex.stream, n1, M,
                     eps_vo, eps_ai, w, r, out);
  MLCC_HIP(hipGetLastError());
}
void denominators(Exec &ex, int O, int V, int o, int v, const double *eps, double *eps_ai,
                  double *eps_vo) {
  hipLaunchKernelGGL(k_denominators, dim3(blocks_for((int64_t)V * O)), dim3(TPB), 0, ex.stream,
                     O, V, o, v, eps, eps_ai, eps_vo);
  MLCC_HIP(hipGetLastError());
}

template <typename T>
void occ_trace(Exec &ex, int64_t J, int64_t n, int O, const T *X, double *d) {
  hipLaunchKernelGGL((k_occ_trace<T>), dim3(blocks_for(J)), dim3(TPB), 0, ex.stream, J, n, O, X,
                     d);
  MLCC_HIP(hipGetLastError());
}

template <typename T>
void energy_singles(Exec &ex, int64_t J, int64_t n, int O, const T *Lt, const T *L, double *res) {
  MLCC_REQUIRE(J <= 2147483647, MLCC_E_ARG, "too many Cholesky vectors");
  double *part = red_part(ex, (int)J + 1024);
  double *part2 = part + J;
  hipLaunchKernelGGL((k_energy_singles<T>), dim3((unsigned)J), dim3(TPB), 0, ex.stream, n, O, Lt,
                     L, part);
  MLCC_HIP(hipGetLastError());
  // sum the J partials in a fixed order
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, ex.stream, (int)J, part, res);
  MLCC_HIP(hipGetLastError());
  (void)part2;
}

template <typename TD, typename TS>
void permute4(Exec &ex, TD *dst, const TS *src, const int64_t n[4], const int64_t s[4], double a,
              double b) {
  const int64_t total = n[0] * n[1] * n[2] * n[3];
  if (total <= 0) return;
  // the dst dimension along which src is contiguous, if not the last one
  int d = -1;
  if (std::llabs(s[3]) != 1 && n[3] > 1)
    for (int k = 2; k >= 0; --k)
      if (std::llabs(s[k]) == 1 && n[k] > 1) {
        d = k;
        break;
      }
  if (d >= 0) {
    const int64_t dstride[4] = {n[1] * n[2] * n[3], n[2] * n[3], n[3], 1};
    int o2[2], m = 0;
    for (int k = 0; k < 3; ++k)
      if (k != d) o2[m++] = k;
    P4 p;
    p.n3 = n[3];
    p.nd = n[d];
    p.nb = n[o2[1]];
    p.t3 = (n[3] + 31) / 32;
    p.td = (n[d] + 31) / 32;
    p.s3 = s[3];
    p.sd = s[d];
    p.sa = s[o2[0]];
    p.sb = s[o2[1]];
    p.dd = dstride[d];
    p.da = dstride[o2[0]];
    p.db = dstride[o2[1]];
    const int64_t blocks = p.t3 * p.td * n[o2[0]] * n[o2[1]];
    MLCC_REQUIRE(blocks < ((int64_t)1 << 31), MLCC_E_ARG, "permute4: array too large");
    hipLaunchKernelGGL((k_permute4_tiled<TD, TS>), dim3((unsigned)blocks), dim3(256), 0, ex.stream,
                       dst, src, p, a, b);
  } else if (total < ((int64_t)1 << 30)) {  // t + grid stride stays below 2^31
    hipLaunchKernelGGL((k_permute4<TD, TS, int32_t>), dim3(blocks_for(total)), dim3(TPB), 0,
                       ex.stream, dst, src, (int32_t)n[0], (int32_t)n[1], (int32_t)n[2],
                       (int32_t)n[3], s[0], s[1], s[2], s[3], a, b);
  } else {
    hipLaunchKernelGGL((k_permute4<TD, TS, int64_t>), dim3(blocks_for(total)), dim3(TPB), 0,
                       ex.stream, dst, src, n[0], n[1], n[2], n[3], s[0], s[1], s[2], s[3], a, b);
  }
  MLCC_HIP(hipGetLastError());
}
template void permute4<double, double>(Exec &, double *, const double *, const int64_t *,
                                       const int64_t *, double, double);
template void permute4<float, float>(Exec &, float *, const float *, const int64_t *,
                                     const int64_t *, double, double);
template void permute4<float, double>(Exec &, float *, const double *, const int64_t *,
                                      const int64_t *, double, double);
template void permute4<double, float>(Exec &, double *, const float *, const int64_t *,
                                      const int64_t *, double, double);

void sym_accum(Exec &ex, int64_t M, const double *R, double *out) {
  if (M == 0) return;
  dim3 grid((unsigned)((M + 31) / 32), (unsigned)((M + 31) / 32));
  hipLaunchKernelGGL(k_sym_accum, grid, dim3(256), 0, ex.stream, M, R, out);
  MLCC_HIP(hipGetLastError());
}

// explicit instantiations
#define INST_PACK(TD, TS)                                                                      \
  template void pack2d<TD, TS>(Exec &, TD *, const TS *, int64_t, int64_t, int64_t, int64_t,   \
                               int64_t);                                                       \
  template void pack2d_t<TD, TS>(Exec &, TD *, const TS *, int64_t, int64_t, int64_t, int64_t, \
                                 int64_t);                                                     \
  template void convert<TD, TS>(Exec &, TD *, const TS *, int64_t);
INST_PACK(double, double)
INST_PACK(float, double)
INST_PACK(float, float)
INST_PACK(double, float)
template void dot_mixed<double, double>(Exec &, int64_t, const double *, const double *, double *);
template void dot_mixed<float, float>(Exec &, int64_t, const float *, const float *, double *);
template void dot_mixed<double, float>(Exec &, int64_t, const double *, const float *, double *);
template void u_of<double>(Exec &, int, int, const double *, double *, int, int64_t, int64_t,
                           bool);
template void u_of<float>(Exec &, int, int, const double *, float *, int, int64_t, int64_t, bool);
template void u_pairblock<double>(Exec &, int, int, int, int, const double *, int64_t, int64_t,
                                  double *, int64_t, double *, int64_t, int64_t, int, double *,
                                  int, int);
template void u_pairblock<float>(Exec &, int, int, int, int, const double *, int64_t, int64_t,
                                 float *, int64_t, float *, int64_t, int64_t, int, double *, int,
                                 int);
template void acc3d<double>(Exec &, int64_t, int64_t, int64_t, double, const double *, int64_t,
                            int64_t, int64_t, double *, int64_t, int64_t);
template void acc3d<float>(Exec &, int64_t, int64_t, int64_t, double, const float *, int64_t,
                           int64_t, int64_t, double *, int64_t, int64_t);
template void sym_plus_diag<double>(Exec &, int64_t, const double *, int64_t, const double *,
                                    const double *, double *, int, int64_t, int64_t, int64_t);
template void sym_plus_diag<float>(Exec &, int64_t, const float *, int64_t, const double *,
                                   const double *, double *, int, int64_t, int64_t, int64_t);
template void cc2_rows<double>(Exec &, int64_t, int, int, int, const double *, int64_t, bool,
                               const double *, const double *, int64_t, double *);
template void cc2_rows<float>(Exec &, int64_t, int, int, int, const float *, int64_t, bool,
                              const double *, const double *, int64_t, double *);
template void sym_div<double, double>(Exec &, int64_t, const double *, int64_t, const double *,
                                      double, double *, int, int64_t, int64_t);
template void sym_div<double, float>(Exec &, int64_t, const double *, int64_t, const double *,
                                     double, float *, int, int64_t, int64_t);
template void mlcc2_omega2<double>(Exec &, int64_t, const double *, const double *,
                                   const double *, double *);
template void occ_trace<double>(Exec &, int64_t, int64_t, int, const double *, double *);
template void occ_trace<float>(Exec &, int64_t, int64_t, int, const float *, double *);
template void energy_singles<double>(Exec &, int64_t, int64_t, int, const double *,
                                     const double *, double *);
template void energy_singles<float>(Exec &, int64_t, int64_t, int, const float *, const float *,
                                    double *);

}  // namespace k
}  // namespace mlcc
