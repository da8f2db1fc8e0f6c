// Small dense linear algebra on the host (FP64): the DIIS linear system and
// the reduced nonsymmetric eigenproblem of the Davidson method (a few hundred
// rows at most).
//
// Eigenvalues: Householder reduction to upper Hessenberg form followed by the
// single-shift QR iteration in complex arithmetic (Wilkinson shifts, Givens
// rotations, deflation on negligible subdiagonals; Golub & Van Loan, "Matrix
// Computations", Ch. 7).  Working in complex arithmetic handles complex
// conjugate pairs without the real double-shift bookkeeping.
// Eigenvectors: inverse iteration with the original matrix, LU with partial
// pivoting.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "dense.h"

namespace mlcc {
namespace dense {

typedef std::complex<double> cd;

bool lu_solve(int n, std::vector<double> A, std::vector<double> &b) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > best) {
        best = std::fabs(A[i * n + k]);
        p = i;
      }
    if (best == 0.0 || !std::isfinite(best)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  return true;
}

static void hessenberg(int n, std::vector<cd> &H) {
  // Householder: for column k zero rows k+2.. of H
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += std::norm(H[i * n + k]);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    std::vector<cd> v(n, 0.0);
    const cd x0 = H[(k + 1) * n + k];
    const cd phase = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
    for (int i = k + 1; i < n; ++i) v[i] = H[i * n + k];
    v[k + 1] += phase * alpha;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    // H <- (I - 2 v v^H / vn) H (I - 2 v v^H / vn)
    for (int j = 0; j < n; ++j) {
      cd s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * H[i * n + j];
      s *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) H[i * n + j] -= v[i] * s;
    }
    for (int i = 0; i < n; ++i) {
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += H[i * n + j] * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) H[i * n + j] -= s * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) H[i * n + k] = 0.0;
  }
}

static cd wilkinson_shift(cd a, cd b, cd c, cd d) {
  // eigenvalue of [[a b][c d]] closer to d
  const cd tr = a + d, det = a * d - b * c;
  const cd disc = std::sqrt(tr * tr * 0.25 - det);
  const cd l1 = tr * 0.5 + disc, l2 = tr * 0.5 - disc;
  return std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
}

bool eigenvalues(int n, const double *A, std::vector<cd> &w) {
  w.assign(n, 0.0);
  if (n == 0) return true;
  std::vector<cd> H(n * n);
  double anorm = 0.0;
  for (int i = 0; i < n * n; ++i) {
    H[i] = A[i];
    anorm = std::max(anorm, std::fabs(A[i]));
  }
  hessenberg(n, H);
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0, total = 0;
  std::vector<cd> cs(n), sn(n);
  while (hi >= 0) {
    if (hi == 0) {
      w[0] = H[0];
      break;
    }
    // find lo: the start of the unreduced block ending at hi
    int lo = hi;
    while (lo > 0) {
      const double s = std::abs(H[(lo - 1) * n + lo - 1]) + std::abs(H[lo * n + lo]);
      const double tol = eps * (s > 0 ? s : anorm);
      if (std::abs(H[lo * n + lo - 1]) <= tol) {
        H[lo * n + lo - 1] = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      w[hi] = H[hi * n + hi];
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return false;
    ++iter;
    cd mu;
    if (iter % 11 == 0) {
      mu = H[hi * n + hi] + std::abs(H[hi * n + hi - 1]) * 0.75;  // exceptional shift
    } else {
      mu = wilkinson_shift(H[(hi - 1) * n + hi - 1], H[(hi - 1) * n + hi], H[hi * n + hi - 1],
                           H[hi * n + hi]);
    }
    // QR step on the block [lo, hi] of H - mu I via Givens rotations
    for (int k = lo; k <= hi; ++k) H[k * n + k] -= mu;
    for (int k = lo; k < hi; ++k) {
      const cd a = H[k * n + k], b = H[(k + 1) * n + k];
      const double r = std::sqrt(std::norm(a) + std::norm(b));
      cd c, s;
      if (r == 0.0) {
        c = 1.0;
        s = 0.0;
      } else {
        c = a / r;
        s = b / r;
      }
      cs[k] = c;
      sn[k] = s;
      // rows k, k+1 <- G^H rows ; G = [[c, -conj(s)], [s, conj(c)]]
      for (int j = k; j < n; ++j) {
        const cd x = H[k * n + j], y = H[(k + 1) * n + j];
        H[k * n + j] = std::conj(c) * x + std::conj(s) * y;
        H[(k + 1) * n + j] = -s * x + c * y;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const cd c = cs[k], s = sn[k];
      // columns k, k+1 <- columns * G
      const int imax = std::min(hi, k + 1);
      for (int i = 0; i <= imax; ++i) {
        const cd x = H[i * n + k], y = H[i * n + k + 1];
        H[i * n + k] = x * c + y * s;
        H[i * n + k + 1] = -x * std::conj(s) + y * std::conj(c);
      }
    }
    for (int k = lo; k <= hi; ++k) H[k * n + k] += mu;
  }
  return true;
}

bool eigenvector_real(int n, const double *A, double lambda, std::vector<double> &x) {
  double anorm = 0.0;
  for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::fabs(A[i]));
  const double shift = lambda + 1e-10 * std::max(1.0, anorm);
  std::vector<double> M(n * n);
  for (int i = 0; i < n * n; ++i) M[i] = A[i];
  for (int i = 0; i < n; ++i) M[i * n + i] -= shift;
  x.assign(n, 1.0);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.01 * std::sin(1.0 + i);
  for (int it = 0; it < 3; ++it) {
    std::vector<double> b = x;
    if (!lu_solve(n, M, b)) {
      // exactly singular: perturb further
      for (int i = 0; i < n; ++i) M[i * n + i] -= 1e-8 * std::max(1.0, anorm);
      b = x;
      if (!lu_solve(n, M, b)) return false;
    }
    double nrm = 0.0;
    for (double v : b) nrm += v * v;
    nrm = std::sqrt(nrm);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return false;
    for (int i = 0; i < n; ++i) x[i] = b[i] / nrm;
  }
  return true;
}

bool cholesky(int n, std::vector<double> &A) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / d;
    }
    for (int k = j + 1; k < n; ++k) A[j * n + k] = 0.0;
  }
  return true;
}

void lower_inverse(int n, const std::vector<double> &Lw, std::vector<double> &Li) {
  Li.assign(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[j * n + j] = 1.0 / Lw[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += Lw[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -s / Lw[i * n + i];
    }
  }
}

}  // namespace dense
}  // namespace mlcc
