// Correlated natural transition orbitals (CNTOs) from CCS excitation vectors
// and the semicanonical basis the multilevel models run in (Sec. 2.2: eqs. M,
// N, approx_double_1, approx_double_2 and select_CNTOs).
//
// For each excitation (R, w), over the full orbital space (pair p = a*O + i):
//   Z^K_ai    = sum_c L^K_ac R_ci - sum_k R_ak L^K_ki
//   gbar_aibj = sum_K (Z^K_ai L^K_bj + L^K_ai Z^K_bj)            (eq. approx_double_2)
//   R_aibj    = -gbar_aibj / ((1 + d_ai,bj)(e_a + e_b - e_i - e_j - w))  (eq. approx_double_1)
//   M        += R^T R + 1/2 sum_a R_a. R_a.^T + 1/2 diag_i(sum_a R_aiai^2)  (eq. M)
//   N        += R R^T + 1/2 sum_i R_.i R_.i^T + 1/2 diag_a(sum_i R_aiai^2)  (eq. N)
// (the P^{ab}_{ij} symmetrisation of eq. approx_double_2 folds into the two
// products of gbar).  gbar is one GEMM over the two slices [Z | L] x [L | Z],
// both pair-major so the reduction index is contiguous; M and N are batch-
// reduced GEMMs over a and over i.  The eigenvectors of the largest
// eigenvalues of M and N span the active occupied and virtual spaces; each of
// the four blocks is then rotated to diagonalise its Fock block.  The
// symmetric eigenproblems run on the device (rocSOLVER syevd); the Cholesky
// vectors are rotated on the device, L'^K = C^T L^K C.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "problem.h"

namespace mlcc {
namespace {

constexpr int kTPB = 256;
inline unsigned nblocks(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kTPB - 1) / kTPB, 16384));
}

// g[p][q] <- -g[p][q] / ((1 + d_pq)(e_a + e_b - e_i - e_j - w)), p = (a,i), q = (b,j)
template <typename T>
__global__ void k_cnto_doubles(int64_t O, int64_t V, const double *eps, double w, T *g) {
  const int64_t n1 = O * V, total = n1 * n1;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = t / n1, q = t - p * n1;
    const int64_t a = p / O, i = p - a * O, b = q / O, j = q - b * O;
    double den = eps[O + a] + eps[O + b] - eps[i] - eps[j] - w;
    if (p == q) den *= 2.0;
    g[t] = (T)(-(double)g[t] / den);
  }
}

// delta terms of eqs. M and N: M_ii += 1/2 sum_a R_aiai^2, N_aa += 1/2 sum_i R_aiai^2
template <typename T>
__global__ void k_cnto_diag(int64_t O, int64_t V, const T *R2, double *M, double *N) {
  const int64_t n1 = O * V;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < O + V;
       t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    if (t < O) {
      for (int64_t a = 0; a < V; ++a) {
        const int64_t p = a * O + t;
        const double r = (double)R2[p * n1 + p];
        s += r * r;
      }
      M[t * O + t] += 0.5 * s;
    } else {
      const int64_t a = t - O;
      for (int64_t i = 0; i < O; ++i) {
        const int64_t p = a * O + i;
        const double r = (double)R2[p * n1 + p];
        s += r * r;
      }
      N[a * V + a] += 0.5 * s;
    }
  }
}

// Symmetric eigenproblems on the device through rocSOLVER.
struct SymEig {
  rocblas_handle h = nullptr;
  explicit SymEig(hipStream_t s) {
    MLCC_REQUIRE(rocblas_create_handle(&h) == rocblas_status_success, MLCC_E_DEVICE,
                 "rocblas_create_handle failed");
    rocblas_set_stream(h, s);
  }
  ~SymEig() {
    if (h) rocblas_destroy_handle(h);
  }
  // A: symmetric m x m (row major).  On return w holds the eigenvalues in
  // ascending order and row k of A the unit eigenvector of w[k].
  void run(Exec &ex, Alloc *al, int64_t m, std::vector<double> &A, std::vector<double> &w) {
    w.assign(m, 0.0);
    if (m == 0) return;
    DBuf dA, dW, dE, dI;
    dA.alloc(al, m * m * sizeof(double));
    dW.alloc(al, m * sizeof(double));
    dE.alloc(al, m * sizeof(double));
    dI.alloc(al, sizeof(rocblas_int));
    MLCC_HIP(hipMemcpyAsync(dA.p, A.data(), m * m * sizeof(double), hipMemcpyHostToDevice,
                            ex.stream));
    // a symmetric row-major matrix is its own column-major form; the
    // column-major eigenvector k is row k of the row-major result
    const rocblas_status st =
        rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)m,
                         dA.as<double>(), (rocblas_int)m, dW.as<double>(), dE.as<double>(),
                         dI.as<rocblas_int>());
    MLCC_REQUIRE(st == rocblas_status_success, MLCC_E_DEVICE, "rocsolver_dsyevd failed");
    rocblas_int info = 0;
    MLCC_HIP(hipMemcpyAsync(A.data(), dA.p, m * m * sizeof(double), hipMemcpyDeviceToHost,
                            ex.stream));
    MLCC_HIP(hipMemcpyAsync(w.data(), dW.p, m * sizeof(double), hipMemcpyDeviceToHost, ex.stream));
    MLCC_HIP(hipMemcpyAsync(&info, dI.p, sizeof(rocblas_int), hipMemcpyDeviceToHost, ex.stream));
    MLCC_HIP(hipStreamSynchronize(ex.stream));
    MLCC_REQUIRE(info == 0, MLCC_E_NUMERIC, "symmetric eigensolver did not converge");
  }
};

// Columns [c0, c0 + k) of U (m x m, row major) rotated so that the Fock block
// F (m x m) is diagonal on them; writes the rotated columns into C and their
// orbital energies (ascending) into e.
void semicanonical(Exec &ex, Alloc *al, SymEig &se, int64_t m, const std::vector<double> &U,
                   const std::vector<double> &F, int64_t c0, int64_t k, std::vector<double> &C,
                   double *e) {
  if (k == 0) return;
  // B = U_blk^T F U_blk (k x k), with every inner loop over contiguous memory
  std::vector<double> FU(m * k, 0.0), B(k * k, 0.0);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t s = 0; s < m; ++s) {
      const double f = F[r * m + s];
      if (f == 0.0) continue;
      const double *us = &U[s * m + c0];
      double *fu = &FU[r * k];
      for (int64_t c = 0; c < k; ++c) fu[c] += f * us[c];
    }
  for (int64_t r = 0; r < m; ++r) {
    const double *ur = &U[r * m + c0];
    const double *fu = &FU[r * k];
    for (int64_t c = 0; c < k; ++c) {
      const double uc = ur[c];
      double *b = &B[c * k];
      for (int64_t d = 0; d < k; ++d) b[d] += uc * fu[d];
    }
  }
  for (int64_t c = 0; c < k; ++c)  // exact symmetry for the solver
    for (int64_t d = 0; d < c; ++d) B[c * k + d] = B[d * k + c] = 0.5 * (B[c * k + d] + B[d * k + c]);
  std::vector<double> w;
  se.run(ex, al, k, B, w);
  for (int64_t c = 0; c < k; ++c) {
    e[c] = w[c];
    // column c0 + c of C = U_blk * (eigenvector c), largest entry positive
    int64_t imax = 0;
    double vmax = -1.0;
    for (int64_t r = 0; r < m; ++r) {
      double s = 0.0;
      for (int64_t l = 0; l < k; ++l) s += U[r * m + c0 + l] * B[c * k + l];
      C[r * m + c0 + c] = s;
      if (std::fabs(s) > vmax) {
        vmax = std::fabs(s);
        imax = r;
      }
    }
    if (C[imax * m + c0 + c] < 0.0)
      for (int64_t r = 0; r < m; ++r) C[r * m + c0 + c] = -C[r * m + c0 + c];
  }
}

}  // namespace
}  // namespace mlcc

using namespace mlcc;

template <typename T>
void mlcc_problem::cnto_t(int ns, const double *R, const double *w, int o_act, int v_act,
                          double *m_eig, double *n_eig, double *C_out, double *eps_out,
                          double *fock_out, double *L_out, bool L_out_dev) {
  Exec &x = *ex;
  Alloc *al = ex->al;
  const int64_t O = d.O, V = d.V, J = d.J, n = d.n, n2 = d.n2, n1 = d.n1;
  const Prec p = gemm_prec<T>();
  const bool o64 = sizeof(T) == 8;
  const T *Lp = off<T>(L);

  // W = [Z | L_vo | Z], each pair-major [n1][K]
  DBuf W;
  W.alloc(al, (size_t)3 * n1 * J * sizeof(T));
  T *Zp = off<T>(W), *Lvo = Zp + n1 * J, *Zp2 = Lvo + n1 * J;
  {
    const int64_t nn[4] = {1, V, O, J}, ss[4] = {0, n, 1, n2};  // L_vo[(a,i)][K] = L^K[O+a][i]
    k::permute4<T, T>(x, Lvo, Lp + O * n, nn, ss, 1.0, 0.0);
  }
  DBuf Rd, Rt, Zt, Gb, Md, Nd;
  Rd.alloc(al, n1 * sizeof(double));
  Rt.alloc(al, n1 * sizeof(T));
  Zt.alloc(al, (size_t)J * n1 * sizeof(T));
  Gb.alloc(al, (size_t)n1 * n1 * sizeof(T));
  Md.alloc(al, O * O * sizeof(double));
  Nd.alloc(al, V * V * sizeof(double));
  k::fill(x, Md.as<double>(), O * O, 0.0);
  k::fill(x, Nd.as<double>(), V * V, 0.0);
  const double *epsd = eps.as<double>();
  for (int s = 0; s < ns; ++s) {
    MLCC_HIP(hipMemcpyAsync(Rd.p, R + (int64_t)s * n1, n1 * sizeof(double),
                            hipMemcpyDeviceToDevice, x.stream));
    k::convert<T, double>(x, off<T>(Rt), Rd.as<double>(), n1);
    // Z^K_ai = sum_c L^K_ac R_ci - sum_k R_ak L^K_ki   ([K][V][O])
    G(V, O, V, 1, J).A(Lp + O * n + O, n, 1, 0, n2).B(Rt.p, O, 1, 0, 0).C(Zt.p, O, 1, n1)
        .tag("cnto_Z").run(x, p, o64);
    G(V, O, O, 1, J).A(Rt.p, O, 1, 0, 0).B(Lp, n, 1, 0, n2).C(Zt.p, O, 1, n1, -1.0, 1.0)
        .tag("cnto_Z").run(x, p, o64);
    {
      const int64_t nn[4] = {1, V, O, J}, ss[4] = {0, O, 1, n1};
      k::permute4<T, T>(x, Zp, off<T>(Zt), nn, ss, 1.0, 0.0);
    }
    MLCC_HIP(hipMemcpyAsync(Zp2, Zp, (size_t)n1 * J * sizeof(T), hipMemcpyDeviceToDevice,
                            x.stream));
    // gbar = Z L^T + L Z^T: slice 0 pairs Z with L, slice 1 L with Z
    G(n1, n1, J, 2).A(Zp, J, 1, n1 * J).B(Lvo, 1, J, n1 * J).C(Gb.p, n1, 1).tag("cnto_gbar")
        .run(x, p, o64);
    hipLaunchKernelGGL((k_cnto_doubles<T>), dim3(nblocks(n1 * n1)), dim3(kTPB), 0, x.stream, O,
                       V, epsd, w[s], off<T>(Gb));
    MLCC_HIP(hipGetLastError());
    // M += 1/2 sum_a R[(a,i)][.] R[(a,j)][.], N += 1/2 sum_i R[(a,i)][.] R[(b,i)][.]
    G(O, O, n1, V).A(Gb.p, n1, 1, O * n1).B(Gb.p, 1, n1, O * n1).C(Md.p, O, 1, 0, 0.5, 1.0)
        .tag("cnto_MN").run(x, p, true);
    G(V, V, n1, O).A(Gb.p, O * n1, 1, n1).B(Gb.p, 1, O * n1, n1).C(Nd.p, V, 1, 0, 0.5, 1.0)
        .tag("cnto_MN").run(x, p, true);
    hipLaunchKernelGGL((k_cnto_diag<T>), dim3(nblocks(O + V)), dim3(kTPB), 0, x.stream, O, V,
                       off<T>(Gb), Md.as<double>(), Nd.as<double>());
    MLCC_HIP(hipGetLastError());
    // singles: M += R^T R, N += R R^T (FP64)
    G(O, O, V).A(Rd.p, 1, O).B(Rd.p, O, 1).C(Md.p, O, 1, 0, 1.0, 1.0).run(x, Prec::F64, true);
    G(V, V, O).A(Rd.p, O, 1).B(Rd.p, 1, O).C(Nd.p, V, 1, 0, 1.0, 1.0).run(x, Prec::F64, true);
  }
  W.release();
  Zt.release();
  Gb.release();

  std::vector<double> Mh(O * O), Nh(V * V);
  MLCC_HIP(hipMemcpyAsync(Mh.data(), Md.p, O * O * sizeof(double), hipMemcpyDeviceToHost, x.stream));
  MLCC_HIP(hipMemcpyAsync(Nh.data(), Nd.p, V * V * sizeof(double), hipMemcpyDeviceToHost, x.stream));
  MLCC_HIP(hipStreamSynchronize(x.stream));
  for (int64_t i = 0; i < O; ++i)
    for (int64_t j = 0; j < i; ++j) Mh[i * O + j] = Mh[j * O + i] = 0.5 * (Mh[i * O + j] + Mh[j * O + i]);
  for (int64_t a = 0; a < V; ++a)
    for (int64_t b = 0; b < a; ++b) Nh[a * V + b] = Nh[b * V + a] = 0.5 * (Nh[a * V + b] + Nh[b * V + a]);
  SymEig se(x.stream);
  std::vector<double> mw, nw;
  se.run(x, al, O, Mh, mw);
  se.run(x, al, V, Nh, nw);
  // U: columns = eigenvectors, largest eigenvalue first
  auto columns_desc = [](int64_t m, const std::vector<double> &rows, std::vector<double> &U) {
    U.assign(m * m, 0.0);
    for (int64_t c = 0; c < m; ++c)
      for (int64_t r = 0; r < m; ++r) U[r * m + c] = rows[(m - 1 - c) * m + r];
  };
  std::vector<double> Uo, Uv;
  columns_desc(O, Mh, Uo);
  columns_desc(V, Nh, Uv);
  if (m_eig)
    for (int64_t c = 0; c < O; ++c) m_eig[c] = mw[O - 1 - c];
  if (n_eig)
    for (int64_t c = 0; c < V; ++c) n_eig[c] = nw[V - 1 - c];

  // the Fock matrix of this problem: the given one, or diag(eps)
  std::vector<double> F(n2, 0.0), e(n);
  MLCC_HIP(hipMemcpyAsync(e.data(), eps.p, n * sizeof(double), hipMemcpyDeviceToHost, x.stream));
  if (fock.p)
    MLCC_HIP(hipMemcpyAsync(F.data(), fock.p, n2 * sizeof(double), hipMemcpyDeviceToHost, x.stream));
  MLCC_HIP(hipStreamSynchronize(x.stream));
  if (!fock.p)
    for (int64_t q = 0; q < n; ++q) F[q * n + q] = e[q];
  std::vector<double> Foo(O * O), Fvv(V * V);
  for (int64_t i = 0; i < O; ++i)
    for (int64_t j = 0; j < O; ++j) Foo[i * O + j] = F[i * n + j];
  for (int64_t a = 0; a < V; ++a)
    for (int64_t b = 0; b < V; ++b) Fvv[a * V + b] = F[(O + a) * n + O + b];
  std::vector<double> Co(O * O), Cv(V * V), enew(n);
  semicanonical(x, al, se, O, Uo, Foo, 0, o_act, Co, enew.data());
  semicanonical(x, al, se, O, Uo, Foo, o_act, O - o_act, Co, enew.data() + o_act);
  semicanonical(x, al, se, V, Uv, Fvv, 0, v_act, Cv, enew.data() + O);
  semicanonical(x, al, se, V, Uv, Fvv, v_act, V - v_act, Cv, enew.data() + O + v_act);
  std::vector<double> C(n2, 0.0);
  for (int64_t i = 0; i < O; ++i)
    for (int64_t j = 0; j < O; ++j) C[i * n + j] = Co[i * O + j];
  for (int64_t a = 0; a < V; ++a)
    for (int64_t b = 0; b < V; ++b) C[(O + a) * n + O + b] = Cv[a * V + b];
  if (C_out) std::copy(C.begin(), C.end(), C_out);
  if (eps_out) std::copy(enew.begin(), enew.end(), eps_out);
  if (fock_out) {
    // C^T F C (block diagonal C, host)
    std::vector<double> FC(n2, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t s = 0; s < n; ++s) {
        const double f = F[r * n + s];
        if (f == 0.0) continue;
        for (int64_t c = 0; c < n; ++c) FC[r * n + c] += f * C[s * n + c];
      }
    std::fill(fock_out, fock_out + n2, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int64_t q = 0; q < n; ++q) {
        const double cr = C[r * n + q];
        if (cr == 0.0) continue;
        const double *x = &FC[r * n];
        double *y = &fock_out[q * n];
        for (int64_t c = 0; c < n; ++c) y[c] += cr * x[c];
      }
  }
  if (L_out) {
    // L'^K = C^T L^K C on the device; FP64 result
    std::vector<T> Ch(C.begin(), C.end());
    DBuf Ct, T1, Lo;
    Ct.alloc(al, n2 * sizeof(T));
    T1.alloc(al, (size_t)J * n2 * sizeof(T));
    double *dst = L_out;
    if (!L_out_dev) {
      Lo.alloc(al, (size_t)J * n2 * sizeof(double));
      dst = Lo.as<double>();
    }
    MLCC_HIP(hipMemcpyAsync(Ct.p, Ch.data(), n2 * sizeof(T), hipMemcpyHostToDevice, x.stream));
    G(n, n, n, 1, J).A(Lp, n, 1, 0, n2).B(Ct.p, n, 1, 0, 0).C(T1.p, n, 1, n2).tag("cnto_L")
        .run(x, p, o64);
    G(n, n, n, 1, J).A(Ct.p, 1, n, 0, 0).B(T1.p, n, 1, 0, n2).C(dst, n, 1, n2).tag("cnto_L")
        .run(x, p, true);
    if (!L_out_dev)
      MLCC_HIP(hipMemcpyAsync(L_out, dst, (size_t)J * n2 * sizeof(double), hipMemcpyDeviceToHost,
                              x.stream));
    MLCC_HIP(hipStreamSynchronize(x.stream));
  }
}

void mlcc_problem::cnto(int ns, const double *R, const double *w, int o_act, int v_act,
                        double *m_eig, double *n_eig, double *C, double *eps_out, double *fock_out,
                        double *L_out, bool L_out_dev) {
  if (prec == MLCC_FP64)
    cnto_t<double>(ns, R, w, o_act, v_act, m_eig, n_eig, C, eps_out, fock_out, L_out, L_out_dev);
  else
    cnto_t<float>(ns, R, w, o_act, v_act, m_eig, n_eig, C, eps_out, fock_out, L_out, L_out_dev);
}
