// Ground-state and Davidson drivers.
#pragma once

#include <functional>
#include <vector>

#include "problem.h"

namespace mlcc {

mlcc_status ground_state(mlcc_problem &P, const mlcc_solver_opts &o, mlcc_info &info);

// problem on a given execution lane (throws Error); descriptor validation
mlcc_problem *problem_new(mlcc_context *ctx, Exec *ex, const mlcc_problem_desc *desc);
void validate_desc(const mlcc_problem_desc *desc);

// out[n][dim] = A in[n][dim]  (device pointers)
typedef std::function<void(int n, const double *in, double *out)> TransformFn;
// out = precond(w) r  (device pointers, one vector)
typedef std::function<void(double w, const double *r, double *out)> PrecondFn;

struct DavidsonResult {
  std::vector<double> omega, residual;
  std::vector<int> complex;
  int iterations = 0, transforms = 0, collapses = 0;
  bool converged = false, stalled = false;
  DBuf X;  // [n_roots][dim] Ritz vectors (unit norm)
};

// Lowest n_roots eigenvalues of a nonsymmetric operator (or the n_roots
// closest to target_w when target_near != 0).  Start vectors: the first
// n_start rows of start (device) followed by unit vectors at guess_idx.
DavidsonResult davidson(Exec &ex, Alloc *al, int64_t dim, int n_roots, int n_guess,
                        int max_space, int max_iter, double tol,
                        const std::vector<int64_t> &guess_idx, const TransformFn &apply,
                        const PrecondFn &precond, const double *start, int n_start,
                        int target_near, double target_w);

}  // namespace mlcc
