// Solver drivers: DIIS-accelerated quasi-Newton ground state and the
// nonsymmetric Davidson excitation solver (Sec. 2.1).  All vectors live on the
// device in FP64; only scalars and the small reduced matrices come to the host.
#include "drivers.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>

#include "dense.h"

namespace mlcc {

namespace {

// C[1][N] = a (device, 1 x K) * B (K x N, row stride ldb)
void rowvec_times(Exec &ex, int64_t K, int64_t N, const double *a, const double *B, int64_t ldb,
                  double *C, double alpha = 1.0, double beta = 0.0) {
  G(1, N, K).A(a, 0, 1).B(B, ldb, 1).C(C, 0, 1, 0, alpha, beta).run(ex, Prec::F64, true);
}

// C[m][n] = sum_x X[m][x] Y[n][x]   (X: mX rows, Y: nY rows, both stride ld)
void gram(Exec &ex, int64_t mX, int64_t nY, int64_t len, const double *X, const double *Y,
          int64_t ld, double *C) {
  G(mX, nY, len).A(X, ld, 1).B(Y, 1, ld).C(C, nY, 1).run(ex, Prec::F64, true);
}

}  // namespace

// ---------------------------------------------------------------------------
// Ground state
// ---------------------------------------------------------------------------
mlcc_status ground_state(mlcc_problem &P, const mlcc_solver_opts &o, mlcc_info &info) {
  Exec &ex = *P.ex;
  Alloc *al = P.ex->al;
  const bool diis_doubles = P.model == MLCC_MLCCSD && P.has_doubles();
  const int64_t len = P.d.n1 + (diis_doubles ? P.d.M * P.d.M : 0);
  const int m = o.diis_dim > 0 ? o.diis_dim : 8;
  const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
  DBuf Xh, Eh, cdev;
  Xh.alloc(al, (size_t)m * len * sizeof(double));
  Eh.alloc(al, (size_t)m * len * sizeof(double));
  cdev.alloc(al, (size_t)(m + 1) * sizeof(double));
  std::vector<double> B((size_t)m * m, 0.0), row(m);
  int count = 0;
  info = mlcc_info{};
  double *amp = P.amp.as<double>();
  double *om = P.om.as<double>();
  bool converged = false;
  int it = 0;
  for (it = 1; it <= max_iter; ++it) {
    P.compute_state(false);
    info.energy = P.e_corr;
    info.residual = P.omega_norm;
    if (!std::isfinite(P.omega_norm) || !std::isfinite(P.e_corr))
      throw Error{MLCC_E_NUMERIC, "non-finite residual or energy in the ground-state iteration"};
    if (P.omega_norm < o.tol) {
      converged = true;
      break;
    }
    if (it == max_iter) break;
    const int slot = (it - 1) % m;
    double *xs = Xh.as<double>() + (int64_t)slot * len;
    double *es = Eh.as<double>() + (int64_t)slot * len;
    MLCC_HIP(hipMemcpyAsync(xs, amp, len * sizeof(double), hipMemcpyDeviceToDevice, ex.stream));
    MLCC_HIP(hipMemcpyAsync(es, om, len * sizeof(double), hipMemcpyDeviceToDevice, ex.stream));
    k::qn_step_singles(ex, P.d.V, P.d.O, P.eps.as<double>(), om, xs);
    if (diis_doubles)
      k::qn_step_doubles(ex, P.d.M, P.eps_ai.as<double>(), om + P.d.n1, xs + P.d.n1);
    count = std::min(count + 1, m);
    // B[slot][j] = e_slot . e_j
    G(1, count, len).A(es, 0, 1).B(Eh.p, 1, len).C(P.res.p, 0, 1).run(ex, Prec::F64, true);
    P.fetch_n(P.res.as<double>(), row.data(), count);
    for (int j = 0; j < count; ++j) {
      B[(size_t)slot * m + j] = row[j];
      B[(size_t)j * m + slot] = row[j];
    }
    // solve [B -1; -1 0] [c; l] = [0; -1] over the stored entries
    const int nb = count + 1;
    std::vector<double> A((size_t)nb * nb, 0.0), rhs(nb, 0.0);
    double scale = 0.0;
    for (int i = 0; i < count; ++i) scale = std::max(scale, std::fabs(B[(size_t)i * m + i]));
    if (scale == 0.0) scale = 1.0;
    for (int i = 0; i < count; ++i) {
      for (int j = 0; j < count; ++j) A[(size_t)i * nb + j] = B[(size_t)i * m + j] / scale;
      A[(size_t)i * nb + count] = -1.0;
      A[(size_t)count * nb + i] = -1.0;
    }
    rhs[count] = -1.0;
    std::vector<double> c(count, 0.0);
    if (dense::lu_solve(nb, A, rhs)) {
      for (int i = 0; i < count; ++i) c[i] = rhs[i];
    } else {
      c[slot] = 1.0;  // singular history: plain quasi-Newton step
    }
    MLCC_HIP(hipMemcpyAsync(cdev.p, c.data(), count * sizeof(double), hipMemcpyHostToDevice,
                            ex.stream));
    rowvec_times(ex, count, len, cdev.as<double>(), Xh.as<double>(), len, amp);
    MLCC_HIP(hipStreamSynchronize(ex.stream));
  }
  P.have_amp = true;
  P.jac_ready = false;
  info.iterations = it > max_iter ? max_iter : it;
  info.converged = converged ? 1 : 0;
  return converged ? MLCC_OK : MLCC_E_NOCONV;
}

// ---------------------------------------------------------------------------
// Davidson
// ---------------------------------------------------------------------------
DavidsonResult davidson(Exec &ex, Alloc *al, int64_t dim, int n_roots, int n_guess,
                        int max_space, int max_iter, double tol,
                        const std::vector<int64_t> &guess_idx, const TransformFn &apply,
                        const PrecondFn &precond, const double *start, int n_start,
                        int target_near, double target_w) {
  DavidsonResult out;
  max_space = std::max(max_space, n_guess + 2 * n_roots);
  max_space = std::max(max_space, 2 * n_roots + 2);
  DBuf Vb, AVb, Wb, Xb, AXb, Yd, Cb, small;
  Vb.alloc(al, (size_t)max_space * dim * sizeof(double));
  AVb.alloc(al, (size_t)max_space * dim * sizeof(double));
  const int wmax = std::max(n_guess, n_roots) + std::max(n_start, 0);
  Wb.alloc(al, (size_t)wmax * dim * sizeof(double));
  Xb.alloc(al, (size_t)n_roots * dim * sizeof(double));
  AXb.alloc(al, (size_t)n_roots * dim * sizeof(double));
  Yd.alloc(al, (size_t)max_space * max_space * sizeof(double));
  Cb.alloc(al, (size_t)max_space * wmax * sizeof(double));
  small.alloc(al, (size_t)std::max(64, max_space * wmax + 64) * sizeof(double));
  double *V = Vb.as<double>(), *AV = AVb.as<double>(), *W = Wb.as<double>();
  std::vector<double> R;  // reduced matrix k x k, R[i][j] = v_i . A v_j
  std::vector<double> hbuf((size_t)max_space * wmax + 64);
  auto fetch = [&](const double *dev, int n) {
    MLCC_HIP(hipMemcpyAsync(hbuf.data(), dev, n * sizeof(double), hipMemcpyDeviceToHost,
                            ex.stream));
    MLCC_HIP(hipStreamSynchronize(ex.stream));
  };

  // start vectors
  int nw = 0;
  MLCC_HIP(hipMemsetAsync(W, 0, (size_t)wmax * dim * sizeof(double), ex.stream));
  if (start && n_start > 0) {
    MLCC_HIP(hipMemcpyAsync(W, start, (size_t)n_start * dim * sizeof(double),
                            hipMemcpyDeviceToDevice, ex.stream));
    nw = n_start;
  }
  for (int g = 0; g < n_guess && nw < wmax; ++g) {
    k::fill(ex, W + (int64_t)nw * dim + guess_idx[g], 1, 1.0);
    ++nw;
  }
  MLCC_HIP(hipStreamSynchronize(ex.stream));

  int k = 0;
  std::vector<double> omega(n_roots, 0.0), resn(n_roots, 0.0);
  std::vector<int> is_complex(n_roots, 0);
  std::vector<double> Yh;
  for (int it = 1; it <= max_iter; ++it) {
    out.iterations = it;
    // --- orthonormalise the new block against V and within itself; a
    // direction that loses all but 1e-8 of its norm is dropped
    const int k_old = k;
    std::vector<double> n0(nw, 0.0);
    for (int w = 0; w < nw; ++w)
      k::dot(ex, dim, W + (int64_t)w * dim, W + (int64_t)w * dim, small.as<double>() + w);
    if (nw > 0) {
      fetch(small.as<double>(), nw);
      for (int w = 0; w < nw; ++w) n0[w] = std::sqrt(hbuf[w]);
    }
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      double *C = Cb.as<double>();
      gram(ex, k, nw, dim, V, W, dim, C);  // C[i][w] = v_i . w
      // W[w] -= sum_i C[i][w] v_i
      G(nw, dim, k).A(C, 1, nw).B(V, dim, 1).C(W, dim, 1, 0, -1.0, 1.0).run(ex, Prec::F64, true);
    }
    for (int w = 0; w < nw; ++w) {
      double *wv = W + (int64_t)w * dim;
      double nrm = 0.0;
      // against the vectors this block has added so far: c = V_new w and
      // w -= V_new^T c on the device (two passes), one fetch for the norm
      const int nn = k - k_old;
      double *cv = small.as<double>() + 32;
      for (int pass = 0; pass < 2 && nn > 0; ++pass) {
        G(nn, 1, dim).A(V + (int64_t)k_old * dim, dim, 1).B(wv, 1, 0).C(cv, 1, 0)
            .run(ex, Prec::F64, true);
        G(1, dim, nn).A(cv, 0, 1).B(V + (int64_t)k_old * dim, dim, 1).C(wv, 0, 1, 0, -1.0, 1.0)
            .run(ex, Prec::F64, true);
      }
      k::dot(ex, dim, wv, wv, small.as<double>());
      fetch(small.as<double>(), 1);
      nrm = std::sqrt(hbuf[0]);
      if (!(nrm > 1e-10) || nrm < 1e-8 * n0[w] || k >= max_space) continue;
      MLCC_HIP(hipMemcpyAsync(V + (int64_t)k * dim, wv, dim * sizeof(double),
                              hipMemcpyDeviceToDevice, ex.stream));
      k::scale(ex, dim, 1.0 / nrm, V + (int64_t)k * dim);
      ++k;
    }
    if (k == k_old) {
      out.stalled = true;
      break;
    }
    // --- transform the new vectors
    apply(k - k_old, V + (int64_t)k_old * dim, AV + (int64_t)k_old * dim);
    out.transforms += k - k_old;
    // --- extend the reduced matrix
    {
      std::vector<double> Rn((size_t)k * k, 0.0);
      for (int i = 0; i < k_old; ++i)
        for (int j = 0; j < k_old; ++j) Rn[(size_t)i * k + j] = R[(size_t)i * k_old + j];
      double *C = Cb.as<double>();
      const int nn = k - k_old;
      // rows of the new vectors: v_i . A v_j, i >= k_old, all j
      gram(ex, nn, k, dim, V + (int64_t)k_old * dim, AV, dim, C);
      fetch(C, nn * k);
      for (int i = 0; i < nn; ++i)
        for (int j = 0; j < k; ++j) Rn[(size_t)(k_old + i) * k + j] = hbuf[(size_t)i * k + j];
      if (k_old > 0) {
        gram(ex, k_old, nn, dim, V, AV + (int64_t)k_old * dim, dim, C);
        fetch(C, k_old * nn);
        for (int i = 0; i < k_old; ++i)
          for (int j = 0; j < nn; ++j) Rn[(size_t)i * k + k_old + j] = hbuf[(size_t)i * nn + j];
      }
      R.swap(Rn);
    }
    // --- reduced eigenproblem
    std::vector<std::complex<double>> ev;
    if (!dense::eigenvalues(k, R.data(), ev)) throw Error{MLCC_E_NUMERIC, "reduced eigenproblem failed"};
    std::vector<int> ord(k);
    std::iota(ord.begin(), ord.end(), 0);
    if (target_near) {
      std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        return std::fabs(ev[a].real() - target_w) < std::fabs(ev[b].real() - target_w);
      });
    } else {
      std::sort(ord.begin(), ord.end(), [&](int a, int b) { return ev[a].real() < ev[b].real(); });
    }
    const int nr = std::min(n_roots, k);
    Yh.assign((size_t)k * n_roots, 0.0);
    for (int r = 0; r < nr; ++r) {
      const std::complex<double> lam = ev[ord[r]];
      omega[r] = lam.real();
      is_complex[r] = std::fabs(lam.imag()) > 1e-10 * std::max(1.0, std::fabs(lam.real()));
      std::vector<double> y;
      if (!dense::eigenvector_real(k, R.data(), lam.real(), y))
        throw Error{MLCC_E_NUMERIC, "Ritz vector failed"};
      for (int i = 0; i < k; ++i) Yh[(size_t)i * n_roots + r] = y[i];
    }
    MLCC_HIP(hipMemcpyAsync(Yd.p, Yh.data(), (size_t)k * n_roots * sizeof(double),
                            hipMemcpyHostToDevice, ex.stream));
    // X = Y^T V, AX = Y^T AV
    double *X = Xb.as<double>(), *AX = AXb.as<double>();
    G(nr, dim, k).A(Yd.p, 1, n_roots).B(V, dim, 1).C(X, dim, 1).run(ex, Prec::F64, true);
    G(nr, dim, k).A(Yd.p, 1, n_roots).B(AV, dim, 1).C(AX, dim, 1).run(ex, Prec::F64, true);
    // residuals r = AX - w X (into AX)
    for (int r = 0; r < nr; ++r) {
      k::axpby(ex, dim, -omega[r], X + (int64_t)r * dim, 1.0, AX + (int64_t)r * dim);
      k::dot(ex, dim, AX + (int64_t)r * dim, AX + (int64_t)r * dim, small.as<double>() + r);
    }
    fetch(small.as<double>(), nr);
    bool all = true;
    for (int r = 0; r < nr; ++r) {
      resn[r] = std::sqrt(hbuf[r]);
      if (!std::isfinite(resn[r])) throw Error{MLCC_E_NUMERIC, "non-finite Davidson residual"};
      if (resn[r] >= tol) all = false;
    }
    if (all && nr == n_roots) {
      out.converged = true;
      break;
    }
    if (it == max_iter) break;
    // --- new directions: preconditioned residuals of unconverged roots
    nw = 0;
    for (int r = 0; r < nr; ++r) {
      if (resn[r] < tol) continue;
      precond(omega[r], AX + (int64_t)r * dim, W + (int64_t)nw * dim);
      ++nw;
    }
    // --- collapse onto the Ritz vectors when the space is full
    if (k + nw > max_space) {
      // orthonormalise the Ritz vectors: Gram = Y^T Y, Yn = Y L^-T
      std::vector<double> Gm((size_t)nr * nr, 0.0);
      for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nr; ++b) {
          double s = 0.0;
          for (int i = 0; i < k; ++i) s += Yh[(size_t)i * n_roots + a] * Yh[(size_t)i * n_roots + b];
          Gm[(size_t)a * nr + b] = s;
        }
      std::vector<double> Li;
      if (!dense::cholesky(nr, Gm)) throw Error{MLCC_E_NUMERIC, "collapse: dependent Ritz vectors"};
      dense::lower_inverse(nr, Gm, Li);
      std::vector<double> Yn((size_t)k * nr, 0.0);  // Yn = Y Li^T
      for (int i = 0; i < k; ++i)
        for (int a = 0; a < nr; ++a) {
          double s = 0.0;
          for (int b = 0; b < nr; ++b) s += Yh[(size_t)i * n_roots + b] * Li[(size_t)a * nr + b];
          Yn[(size_t)i * nr + a] = s;
        }
      // R_new = Yn^T R Yn
      std::vector<double> RY((size_t)k * nr, 0.0), Rnew((size_t)nr * nr, 0.0);
      for (int i = 0; i < k; ++i)
        for (int a = 0; a < nr; ++a) {
          double s = 0.0;
          for (int j = 0; j < k; ++j) s += R[(size_t)i * k + j] * Yn[(size_t)j * nr + a];
          RY[(size_t)i * nr + a] = s;
        }
      for (int a = 0; a < nr; ++a)
        for (int b = 0; b < nr; ++b) {
          double s = 0.0;
          for (int i = 0; i < k; ++i) s += Yn[(size_t)i * nr + a] * RY[(size_t)i * nr + b];
          Rnew[(size_t)a * nr + b] = s;
        }
      MLCC_HIP(hipMemcpyAsync(Yd.p, Yn.data(), (size_t)k * nr * sizeof(double),
                              hipMemcpyHostToDevice, ex.stream));
      G(nr, dim, k).A(Yd.p, 1, nr).B(V, dim, 1).C(X, dim, 1).run(ex, Prec::F64, true);
      G(nr, dim, k).A(Yd.p, 1, nr).B(AV, dim, 1).C(AX + 0, dim, 1).run(ex, Prec::F64, true);
      // AX held residuals; they were consumed by precond above
      MLCC_HIP(hipMemcpyAsync(V, X, (size_t)nr * dim * sizeof(double), hipMemcpyDeviceToDevice,
                              ex.stream));
      MLCC_HIP(hipMemcpyAsync(AV, AX, (size_t)nr * dim * sizeof(double), hipMemcpyDeviceToDevice,
                              ex.stream));
      k = nr;
      R.swap(Rnew);
      out.collapses++;
    }
  }
  out.omega = omega;
  out.residual = resn;
  out.complex = is_complex;
  // final Ritz vectors stay in X (first n_roots rows)
  out.X = std::move(Xb);
  return out;
}

}  // namespace mlcc
