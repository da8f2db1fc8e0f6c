// Small dense FP64 linear algebra on the host (DIIS, reduced eigenproblems).
#pragma once
#include <complex>
#include <vector>

namespace mlcc {
namespace dense {
// Solve A x = b (A row-major n x n, copied); b <- x.  false if singular.
bool lu_solve(int n, std::vector<double> A, std::vector<double> &b);
// All eigenvalues of a real row-major n x n matrix.
bool eigenvalues(int n, const double *A, std::vector<std::complex<double>> &w);
// Unit-norm right eigenvector for a real eigenvalue lambda.
bool eigenvector_real(int n, const double *A, double lambda, std::vector<double> &x);
// In-place lower Cholesky factor of a symmetric positive definite matrix.
bool cholesky(int n, std::vector<double> &A);
// Inverse of a lower-triangular matrix.
void lower_inverse(int n, const std::vector<double> &L, std::vector<double> &Li);
}  // namespace dense
}  // namespace mlcc
