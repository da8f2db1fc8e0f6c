// Cholesky vectors in the MO basis from AO integrals (Sec. 2.4 of Folkestad
// et al.): the two-step Cholesky decomposition.
//
// First step (mlcc_cholesky_basis): the Cholesky basis by pivoted Cholesky
// decomposition of the AO integral matrix over packed pairs ab (a >= b), with
// the updated diagonal D_ab = (ab|ab) - sum_J (L^J_ab)^2 screened by the MO
// weights, D~_ab = nu_a D_ab nu_b (eq. cd_screening; nu_a = max_p (C^a_ap)^2,
// eq. mo_screening).  Each pivot is one device argmax of D~, one engine GEMV
// (the new column minus its projection on the earlier vectors) and one update
// of the vector and the diagonal; only the pivot's index and diagonal come to
// the host, for the termination test max D~ < tau.  S = Q Q^T over the basis
// is the decomposition's own vectors at the pivots (Q lower triangular), and
// Q^-T comes from a device triangular inversion (rocSOLVER).
//
// Second step (mlcc_mo_cholesky, Algorithm 1): for each batch P of MO
// indices p,
//   for each chunk of the basis: (ab|K) unpacked from the integral columns
//   at the pivots, W_pbK = sum_a C_ap (ab|K), X_pqK = sum_b W_pbK C_bq;
//   then L^J_pq = sum_K [Q^-T]_KJ X_pqK for p in P.
// The three contractions run on the GEMM engine with both operands
// contiguous along the reduction index (C and Q^-T are stored transposed
// once), so the split BF16 products apply in MLCC_BF16X3.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "api_util.h"

namespace mlcc {
namespace {

constexpr int TPB = 256;
inline unsigned blocks_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 16384));
}
#define GRID_STRIDE(i, n)                                                   \
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); \
       i += (int64_t)gridDim.x * blockDim.x)

// packed pair index of (a, b), a >= b
__device__ __forceinline__ int64_t pair_of(int64_t a, int64_t b) {
  return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
}

__global__ void k_diag(const double *G, int64_t npair, double *D) {
  GRID_STRIDE(i, npair) D[i] = G[i * npair + i];
}

// w_ab = nu_a nu_b over packed pairs
__global__ void k_pair_weights(const double *nu, int64_t n_ao, double *w) {
  GRID_STRIDE(a, n_ao) {
    for (int64_t b = 0; b <= a; ++b) w[a * (a + 1) / 2 + b] = nu[a] * nu[b];
  }
}

// Largest w_i D_i (w NULL: D_i); ties go to the lower index, so the choice
// does not depend on the launch.  Partial results per block, then one block.
__global__ void k_argmax_partial(const double *w, const double *D, int64_t n, double *pv,
                                 int64_t *pi) {
  __shared__ double sv[TPB];
  __shared__ int64_t si[TPB];
  double best = -1.0;
  int64_t bi = -1;
  GRID_STRIDE(i, n) {
    const double x = w ? w[i] * D[i] : D[i];
    if (x > best || (x == best && i < bi)) {
      best = x;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double v2 = sv[threadIdx.x + s];
      const int64_t i2 = si[threadIdx.x + s];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 >= 0 &&
                                   (si[threadIdx.x] < 0 || i2 < si[threadIdx.x]))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}

// res = {max w D, its index (as double), D at that index}
__global__ void k_argmax_final(int nb, const double *pv, const int64_t *pi, const double *D,
                               double *res) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double best = -1.0;
  int64_t bi = -1;
  for (int b = 0; b < nb; ++b)
    if (pi[b] >= 0 && (pv[b] > best || (pv[b] == best && pi[b] < bi))) {
      best = pv[b];
      bi = pi[b];
    }
  res[0] = best;
  res[1] = (double)bi;
  res[2] = bi >= 0 ? D[bi] : 0.0;
}

// L = col / sqrt(dK) in place; D -= L^2, the pivot's diagonal set to zero
__global__ void k_chol_update(double *L, int64_t npair, int64_t K, double dK, double *D) {
  const double r = 1.0 / sqrt(dK);
  GRID_STRIDE(i, npair) {
    const double l = L[i] * r;
    L[i] = l;
    D[i] = i == K ? 0.0 : D[i] - l * l;
  }
}

// Q[J][J'] = L^{J'} at pivot J (J' <= J), zero above the diagonal
__global__ void k_gather_q(const double *L, int64_t npair, const int *piv, int64_t n,
                           double *Q) {
  GRID_STRIDE(t, n * n) {
    const int64_t J = t / n, Jp = t - J * n;
    Q[t] = Jp <= J ? L[Jp * npair + piv[J]] : 0.0;
  }
}

// out[c][r] = in[r][c]   (n x n)
template <typename TO, typename TI>
__global__ void k_transpose(const TI *in, int64_t rows, int64_t cols, TO *out) {
  GRID_STRIDE(t, rows * cols) {
    const int64_t r = t / cols, c = t - r * cols;
    out[c * rows + r] = (TO)in[t];
  }
}

// (ab|K) for the kc basis elements K = piv[k0 + k]: ao3[k][a][b] from row
// piv[K] of the symmetric pair matrix G
template <typename T>
__global__ void k_unpack_columns(const double *G, int64_t npair, const int *piv, int64_t k0,
                                 int64_t kc, int64_t n_ao, T *ao3) {
  const int64_t nn = n_ao * n_ao;
  GRID_STRIDE(t, kc * nn) {
    const int64_t k = t / nn, ab = t - k * nn, a = ab / n_ao, b = ab - a * n_ao;
    ao3[t] = (T)G[(int64_t)piv[k0 + k] * npair + pair_of(a, b)];
  }
}

struct Solver {
  rocblas_handle h = nullptr;
  explicit Solver(hipStream_t s) {
    MLCC_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, MLCC_E_DEVICE,
                 "rocblas_create_handle failed");
    rocblas_set_stream(h, s);
  }
  ~Solver() {
    if (h) rocblas_destroy_handle(h);
  }
};

// a caller array (host or device) as a device pointer
const double *device_view(mlcc_context *ctx, DBuf &tmp, const double *src, int64_t n) {
  if (is_device_ptr(src)) return src;
  tmp.alloc(&ctx->al, n * sizeof(double));
  MLCC_HIP(hipMemcpyAsync(tmp.p, src, n * sizeof(double), hipMemcpyHostToDevice, ctx->ex.stream));
  return tmp.as<double>();
}

void write_out(mlcc_context *ctx, double *dst, const double *src, int64_t n) {
  MLCC_HIP(hipMemcpyAsync(dst, src, n * sizeof(double),
                          is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          ctx->ex.stream));
}

void cholesky_basis(mlcc_context *ctx, int32_t n_ao, const double *G_in, const double *nu_in,
                    double tau, int32_t max_vectors, int32_t *pivots, int32_t *n_vectors,
                    double *QinvT) {
  Exec &x = ctx->ex;
  Alloc *al = &ctx->al;
  const int64_t npair = (int64_t)n_ao * (n_ao + 1) / 2;
  DBuf Gt, nut, D, w, Lp, red, res, Q;
  const double *Gd = device_view(ctx, Gt, G_in, npair * npair);
  D.alloc(al, npair * sizeof(double));
  hipLaunchKernelGGL(k_diag, dim3(blocks_for(npair)), dim3(TPB), 0, x.stream, Gd, npair,
                     D.as<double>());
  if (nu_in) {
    const double *nu = device_view(ctx, nut, nu_in, n_ao);
    w.alloc(al, npair * sizeof(double));
    hipLaunchKernelGGL(k_pair_weights, dim3(blocks_for(n_ao)), dim3(TPB), 0, x.stream, nu,
                       (int64_t)n_ao, w.as<double>());
  }
  MLCC_HIP(hipGetLastError());
  Lp.alloc(al, (size_t)max_vectors * npair * sizeof(double));
  const unsigned nb = std::min<unsigned>(blocks_for(npair), 1024);
  red.alloc(al, nb * (sizeof(double) + sizeof(int64_t)));
  res.alloc(al, 4 * sizeof(double));
  double *pv = red.as<double>();
  int64_t *pi = reinterpret_cast<int64_t *>(pv + nb);
  std::vector<int> piv;
  for (int32_t J = 0; J < max_vectors; ++J) {
    hipLaunchKernelGGL(k_argmax_partial, dim3(nb), dim3(TPB), 0, x.stream,
                       w.p ? w.as<double>() : nullptr, D.as<double>(), npair, pv, pi);
    hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(64), 0, x.stream, (int)nb, pv, pi,
                       D.as<double>(), res.as<double>());
    MLCC_HIP(hipGetLastError());
    MLCC_HIP(hipMemcpyAsync(x.pinned, res.p, 3 * sizeof(double), hipMemcpyDeviceToHost,
                            x.stream));
    MLCC_HIP(hipStreamSynchronize(x.stream));
    const double best = x.pinned[0], dK = x.pinned[2];
    const int64_t K = (int64_t)x.pinned[1];
    MLCC_REQUIRE(std::isfinite(best) && std::isfinite(dK), MLCC_E_NUMERIC,
                 "non-finite integral diagonal");
    if (!(best >= tau) || K < 0) break;
    MLCC_REQUIRE(dK > 0.0, MLCC_E_NUMERIC, "the integral matrix is not positive semidefinite");
    double *LJ = Lp.as<double>() + (int64_t)J * npair;
    // L^J = G[K] - sum_{J' < J} L^{J'}_K L^{J'} (an empty reduction copies G[K])
    G(1, npair, J).A(Lp.as<double>() + K, 0, npair).B(Lp.p, npair, 1)
        .C(LJ, 0, 1, 0, -1.0, 1.0, Gd + K * npair).tag("chol_column").run(x, Prec::F64, true);
    hipLaunchKernelGGL(k_chol_update, dim3(blocks_for(npair)), dim3(TPB), 0, x.stream, LJ, npair,
                       K, dK, D.as<double>());
    MLCC_HIP(hipGetLastError());
    piv.push_back((int)K);
  }
  const int64_t n = (int64_t)piv.size();
  *n_vectors = (int32_t)n;
  for (int64_t J = 0; J < n; ++J) pivots[J] = piv[J];
  if (n == 0 || !QinvT) {
    MLCC_HIP(hipStreamSynchronize(x.stream));
    return;
  }
  // Q (row major, lower) from the vectors at the pivots; its inverse by
  // rocSOLVER on the column-major view (upper), then Q^-T = (Q^-1)^T
  DBuf dpiv, Qi, info;
  dpiv.alloc(al, n * sizeof(int));
  MLCC_HIP(hipMemcpyAsync(dpiv.p, piv.data(), n * sizeof(int), hipMemcpyHostToDevice, x.stream));
  Q.alloc(al, n * n * sizeof(double));
  hipLaunchKernelGGL(k_gather_q, dim3(blocks_for(n * n)), dim3(TPB), 0, x.stream, Lp.as<double>(),
                     npair, dpiv.as<int>(), n, Q.as<double>());
  MLCC_HIP(hipGetLastError());
  info.alloc(al, sizeof(rocblas_int));
  {
    Solver sv(x.stream);
    const rocblas_status st = rocsolver_dtrtri(sv.h, rocblas_fill_upper, rocblas_diagonal_non_unit,
                                               (rocblas_int)n, Q.as<double>(), (rocblas_int)n,
                                               info.as<rocblas_int>());
    MLCC_REQUIRE(st == rocblas_status_success, MLCC_E_DEVICE, "rocsolver_dtrtri failed");
    rocblas_int inf = 0;
    MLCC_HIP(hipMemcpyAsync(&inf, info.p, sizeof(rocblas_int), hipMemcpyDeviceToHost, x.stream));
    MLCC_HIP(hipStreamSynchronize(x.stream));
    MLCC_REQUIRE(inf == 0, MLCC_E_NUMERIC, "singular Cholesky factor of the basis");
  }
  Qi.alloc(al, n * n * sizeof(double));
  hipLaunchKernelGGL((k_transpose<double, double>), dim3(blocks_for(n * n)), dim3(TPB), 0,
                     x.stream, Q.as<double>(), n, n, Qi.as<double>());
  MLCC_HIP(hipGetLastError());
  write_out(ctx, QinvT, Qi.as<double>(), n * n);
  MLCC_HIP(hipStreamSynchronize(x.stream));
}

template <typename T>
void mo_cholesky_t(mlcc_context *ctx, Prec prec, int32_t n_ao, int32_t n_mo, const double *G_in,
                   int32_t n_vec, const int32_t *pivots, const double *QinvT_in,
                   const double *C_in, int32_t p_batch, double *L_out) {
  Exec &x = ctx->ex;
  Alloc *al = &ctx->al;
  const int64_t npair = (int64_t)n_ao * (n_ao + 1) / 2, na = n_ao, nm = n_mo, nJ = n_vec;
  DBuf Gt, Qt, Ct, dpiv, CT, Qinv, ao3, W, X, Lt;
  const double *Gd = device_view(ctx, Gt, G_in, npair * npair);
  const double *QiT = device_view(ctx, Qt, QinvT_in, nJ * nJ);
  const double *C = device_view(ctx, Ct, C_in, na * nm);
  std::vector<int> hp(pivots, pivots + n_vec);
  for (int p : hp) MLCC_REQUIRE(p >= 0 && p < npair, MLCC_E_ARG, "pivot outside the pair range");
  dpiv.alloc(al, nJ * sizeof(int));
  MLCC_HIP(hipMemcpyAsync(dpiv.p, hp.data(), nJ * sizeof(int), hipMemcpyHostToDevice, x.stream));
  // C^T [n_mo][n_ao] and Q^-1 = (Q^-T)^T [J][K] in the operand type
  CT.alloc(al, nm * na * sizeof(T));
  hipLaunchKernelGGL((k_transpose<T, double>), dim3(blocks_for(na * nm)), dim3(TPB), 0, x.stream,
                     C, na, nm, CT.as<T>());
  Qinv.alloc(al, nJ * nJ * sizeof(T));
  hipLaunchKernelGGL((k_transpose<T, double>), dim3(blocks_for(nJ * nJ)), dim3(TPB), 0, x.stream,
                     QiT, nJ, nJ, Qinv.as<T>());
  MLCC_HIP(hipGetLastError());
  // batch of p and chunk of the basis within 2 GB of scratch
  const int64_t kc = std::min<int64_t>(nJ, 128);
  const double ts = sizeof(T);
  int64_t nb = p_batch > 0 ? std::min<int64_t>(p_batch, nm) : nm;
  if (p_batch <= 0) {
    const double per_p = ts * ((double)nJ * nm + (double)kc * na);
    nb = std::max<int64_t>(1, std::min<int64_t>(nm, (int64_t)((2e9 - ts * kc * na * na) / per_p)));
  }
  ao3.alloc(al, (size_t)kc * na * na * sizeof(T));
  W.alloc(al, (size_t)kc * nb * na * sizeof(T));
  X.alloc(al, (size_t)nJ * nb * nm * sizeof(T));
  double *Ld = L_out;
  if (!is_device_ptr(L_out)) {
    Lt.alloc(al, (size_t)nJ * nm * nm * sizeof(double));
    Ld = Lt.as<double>();
  }
  for (int64_t p0 = 0; p0 < nm; p0 += nb) {
    const int64_t np = std::min<int64_t>(nb, nm - p0);
    for (int64_t k0 = 0; k0 < nJ; k0 += kc) {
      const int64_t nk = std::min<int64_t>(kc, nJ - k0);
      // (ab|K) for this chunk of the basis
      hipLaunchKernelGGL((k_unpack_columns<T>), dim3(blocks_for(nk * na * na)), dim3(TPB), 0,
                         x.stream, Gd, npair, dpiv.as<int>(), k0, nk, na, ao3.as<T>());
      MLCC_HIP(hipGetLastError());
      // W[k][p][b] = sum_a C_ap (ab|K)   ((ab|K) read as [b][a]: symmetric)
      G(np, na, na, 1, nk).A(CT.as<T>() + p0 * na, na, 1, 0, 0).B(ao3.p, 1, na, 0, na * na)
          .C(W.p, na, 1, np * na).tag("mo_chol_W").run(x, prec, sizeof(T) == 8);
      // X[K][p][q] = sum_b W[k][p][b] C_bq
      G(np, nm, na, 1, nk).A(W.p, na, 1, 0, np * na).B(CT.p, 1, na, 0, 0)
          .C(X.as<T>() + k0 * np * nm, nm, 1, np * nm).tag("mo_chol_X").run(x, prec, sizeof(T) == 8);
    }
    // L^J_pq = sum_K [Q^-T]_KJ X[K][p][q] for p in the batch
    G(nJ, np * nm, nJ).A(Qinv.p, nJ, 1).B(X.p, np * nm, 1).C(Ld + p0 * nm, nm * nm, 1)
        .tag("mo_chol_L").run(x, prec, true);
  }
  if (Ld != L_out) write_out(ctx, L_out, Ld, nJ * nm * nm);
  MLCC_HIP(hipStreamSynchronize(x.stream));
}

}  // namespace
}  // namespace mlcc

using namespace mlcc;

extern "C" {

mlcc_status mlcc_cholesky_basis(mlcc_context *ctx, int32_t n_ao, const double *G, const double *nu,
                                double tau, int32_t max_vectors, int32_t *pivots,
                                int32_t *n_vectors, double *QinvT) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(n_ao >= 1 && n_ao <= 4096, MLCC_E_ARG, "n_ao out of range");
    const int64_t npair = (int64_t)n_ao * (n_ao + 1) / 2;
    MLCC_REQUIRE(max_vectors >= 1 && max_vectors <= npair, MLCC_E_ARG, "bad max_vectors");
    MLCC_REQUIRE(G && pivots && n_vectors, MLCC_E_ARG, "NULL argument");
    MLCC_REQUIRE(tau > 0.0 && std::isfinite(tau), MLCC_E_ARG, "tau must be positive");
    MLCC_HIP(hipSetDevice(ctx->device));
    cholesky_basis(ctx, n_ao, G, nu, tau, max_vectors, pivots, n_vectors, QinvT);
    return MLCC_OK;
  });
}

mlcc_status mlcc_mo_cholesky(mlcc_context *ctx, int32_t precision, int32_t n_ao, int32_t n_mo,
                             const double *G, int32_t n_vec, const int32_t *pivots,
                             const double *QinvT, const double *C, int32_t p_batch,
                             double *L_out) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(precision == MLCC_FP64 || precision == MLCC_FP32 || precision == MLCC_BF16X3 ||
                     precision == MLCC_BF16,
                 MLCC_E_ARG, "unknown precision");
    MLCC_REQUIRE(n_ao >= 1 && n_ao <= 4096 && n_mo >= 1 && n_mo <= n_ao, MLCC_E_ARG,
                 "bad orbital counts");
    const int64_t npair = (int64_t)n_ao * (n_ao + 1) / 2;
    MLCC_REQUIRE(n_vec >= 1 && n_vec <= npair, MLCC_E_ARG, "bad number of vectors");
    MLCC_REQUIRE(G && pivots && QinvT && C && L_out, MLCC_E_ARG, "NULL argument");
    MLCC_REQUIRE(p_batch >= 0, MLCC_E_ARG, "negative batch");
    MLCC_HIP(hipSetDevice(ctx->device));
    if (precision == MLCC_FP64)
      mo_cholesky_t<double>(ctx, Prec::F64, n_ao, n_mo, G, n_vec, pivots, QinvT, C, p_batch, L_out);
    else
      mo_cholesky_t<float>(ctx, engine_prec(precision), n_ao, n_mo, G, n_vec, pivots, QinvT, C,
                           p_batch, L_out);
    return MLCC_OK;
  });
}

}  // extern "C"
