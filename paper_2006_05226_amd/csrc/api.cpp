// The extern "C" boundary of libmlcc: argument checking, host/device pointer
// handling, error translation.  See include/mlcc.h for the contract.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "api_util.h"
#include "drivers.h"

using namespace mlcc;

namespace {

// Stage a caller array (host or device) as a device pointer.
struct In {
  DBuf buf;
  const double *p = nullptr;
  In(mlcc_problem &P, const double *src, int64_t n) {
    if (is_device_ptr(src)) {
      p = src;
    } else {
      buf.alloc(P.ex->al, n * sizeof(double));
      MLCC_HIP(hipMemcpyAsync(buf.p, src, n * sizeof(double), hipMemcpyHostToDevice,
                              P.ex->stream));
      p = buf.as<double>();
    }
  }
};
struct Out {
  DBuf buf;
  double *dst;
  double *p = nullptr;
  int64_t n;
  mlcc_problem &P;
  Out(mlcc_problem &Pr, double *d, int64_t nn) : dst(d), n(nn), P(Pr) {
    if (is_device_ptr(d)) {
      p = d;
    } else {
      buf.alloc(P.ex->al, n * sizeof(double));
      p = buf.as<double>();
    }
  }
  void commit() {
    if (p != dst)
      MLCC_HIP(hipMemcpyAsync(dst, p, n * sizeof(double), hipMemcpyDeviceToHost, P.ex->stream));
  }
};

// Contractions whose plain BF16 products keep the energies within 1e-6 Eh and
// the excitation energies within 1e-5 eV of FP64 on the 40/400/1200 MLCC2
// and 60/600/2000 MLCCSD workloads (the study that picked them is
// bench.py --bf16-study), each alone and all together.  Left out: the
// MLCCSD E2 term (with it in plain BF16 the ground state no longer reaches
// 1e-6), and untagged and orbital-selection products.
const std::vector<std::string> kBf16Map = {
    "x1_vv",  "x1_vo",   "fock_exch", "g_aibj", "Z_uL",     "ccs_Xk",    "ccs_coul",  "ccs_W",
    "ccs_vv", "jac_X",   "jac_Y",     "jac_q",  "jac_P",    "jac_r",     "jac_uw",    "dLai",
    "sigma2_LdL", "Zc_uL", "d2s_A1",  "d2s_B1", "cc_g",     "cc_g_vvvv", "cc_ladder", "cc_B2",
    "cc_C2",  "cc_D2",   "cc_Gk",     "cc_Y3",  "cc_Y3c",   "cc_dL",     "cc_dg",     "cc_dF"};

void check_desc(const mlcc_problem_desc *d) {
  MLCC_REQUIRE(d != nullptr, MLCC_E_ARG, "NULL problem descriptor");
  MLCC_REQUIRE((d->L != nullptr || (d->flags & MLCC_SYNTH_L)) && d->eps != nullptr, MLCC_E_ARG,
               "NULL L or eps");
  MLCC_REQUIRE((d->flags & ~(MLCC_SYNTH_L | MLCC_INPUT_ON_DEVICE | MLCC_DETERMINISTIC)) == 0,
               MLCC_E_ARG, "unknown flags");
  if (d->flags & MLCC_INPUT_ON_DEVICE) {
    MLCC_REQUIRE((d->flags & MLCC_SYNTH_L) || is_device_ptr(d->L), MLCC_E_ARG,
                 "MLCC_INPUT_ON_DEVICE: L is not device memory");
    MLCC_REQUIRE(is_device_ptr(d->eps), MLCC_E_ARG, "MLCC_INPUT_ON_DEVICE: eps is not device memory");
    MLCC_REQUIRE(!d->fock || is_device_ptr(d->fock), MLCC_E_ARG,
                 "MLCC_INPUT_ON_DEVICE: fock is not device memory");
  }
  MLCC_REQUIRE(d->n_occ >= 1 && d->n_vir >= 1 && d->n_chol >= 1, MLCC_E_ARG,
               "n_occ, n_vir and n_chol must be >= 1");
  MLCC_REQUIRE(d->model == MLCC_CCS || d->model == MLCC_MLCC2 || d->model == MLCC_MLCCSD ||
                   d->model == MLCC_MLCCSD3,
               MLCC_E_ARG, "unknown model");
  if (d->model == MLCC_MLCCSD3)
    MLCC_REQUIRE(d->n_occ_ccsd >= 0 && d->n_occ_ccsd <= d->n_occ_act && d->n_vir_ccsd >= 0 &&
                     d->n_vir_ccsd <= d->n_vir_act,
                 MLCC_E_ARG, "CCSD space not inside the active space");
  MLCC_REQUIRE(d->precision == MLCC_FP64 || d->precision == MLCC_FP32 ||
                   d->precision == MLCC_BF16X3 || d->precision == MLCC_BF16,
               MLCC_E_ARG, "unknown precision");
  if (d->model != MLCC_CCS) {
    MLCC_REQUIRE(d->n_occ_act >= 0 && d->n_occ_act <= d->n_occ && d->n_vir_act >= 0 &&
                     d->n_vir_act <= d->n_vir,
                 MLCC_E_ARG, "active space larger than the orbital space");
    MLCC_REQUIRE((int64_t)d->n_occ_act * d->n_vir_act <= 46340, MLCC_E_ARG,
                 "active pair count above the supported maximum");
  }
  const int64_t n = (int64_t)d->n_occ + d->n_vir;
  MLCC_REQUIRE(n <= 65535, MLCC_E_ARG, "too many orbitals");
}

}  // namespace

extern "C" {

mlcc_status mlcc_context_create(int device, void *hip_stream, uint64_t hbm_budget,
                                mlcc_context **out) {
  return guarded(nullptr, [&]() -> mlcc_status {
    MLCC_REQUIRE(out != nullptr, MLCC_E_ARG, "NULL output pointer");
    int count = 0;
    MLCC_HIP(hipGetDeviceCount(&count));
    MLCC_REQUIRE(device >= 0 && device < count, MLCC_E_ARG, "no such device");
    MLCC_HIP(hipSetDevice(device));
    auto *c = new mlcc_context();
    c->device = device;
    c->al.device = device;
    c->al.budget = hbm_budget;
    c->ex.al = &c->al;
    c->ex.prof = &c->prof;
    c->bf16_map = kBf16Map;
    c->ex.bf16_map = &c->bf16_map;
    if (hip_stream) {
      c->ex.stream = static_cast<hipStream_t>(hip_stream);
    } else {
      hipError_t e = hipStreamCreateWithFlags(&c->ex.stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete c;
        MLCC_HIP(e);
      }
      c->own_stream = true;
    }
    c->al.stream = c->ex.stream;
    if (hipHostMalloc((void **)&c->ex.pinned, 512 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
      (void)hipGetLastError();
      if (c->own_stream) (void)hipStreamDestroy(c->ex.stream);
      delete c;
      throw Error{MLCC_E_DEVICE, "pinned host allocation failed"};
    }
    // the no-allocation engine's array on this device (its address, once)
    noalloc_scratch_init(device);
    *out = c;
    return MLCC_OK;
  });
}

mlcc_status mlcc_context_destroy(mlcc_context *ctx) {
  if (!ctx) return MLCC_E_ARG;
  context_unref(ctx);
  return MLCC_OK;
}

mlcc_status mlcc_bf16_map(mlcc_context *ctx, const char *tags) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    std::vector<std::string> m;
    if (!tags) {
      m = kBf16Map;
    } else {
      std::string cur;
      for (const char *c = tags;; ++c) {
        if (*c == ',' || *c == '\0') {
          if (!cur.empty()) m.push_back(cur);
          cur.clear();
          if (*c == '\0') break;
        } else if (*c != ' ') {
          cur.push_back(*c);
        }
      }
    }
    ctx->bf16_map.swap(m);
    return MLCC_OK;
  });
}

const char *mlcc_last_error(mlcc_context *ctx) {
  return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

uint64_t mlcc_context_bytes(mlcc_context *ctx) { return ctx ? ctx->al.used : 0; }

}  // extern "C"

namespace mlcc {
void context_unref(mlcc_context *ctx) {
  if (ctx->refs.fetch_sub(1) != 1) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->ex.stream);
  ctx->ex.work.release();
  ctx->ex.red.release();
  ctx->ex.planes.release();
  ctx->al.release_all();
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->ex.stream);
  if (ctx->ex.pinned) (void)hipHostFree(ctx->ex.pinned);
  delete ctx;
}

mlcc_problem *problem_new(mlcc_context *ctx, Exec *ex, const mlcc_problem_desc *desc) {
  check_desc(desc);
  MLCC_HIP(hipSetDevice(ctx->device));
  auto *P = new mlcc_problem();
  P->ctx = ctx;
  P->ex = ex;
  try {
    P->setup(*desc);
  } catch (...) {
    delete P;
    throw;
  }
  return P;
}
void validate_desc(const mlcc_problem_desc *desc) { check_desc(desc); }
}  // namespace mlcc

extern "C" {

mlcc_status mlcc_problem_create(mlcc_context *ctx, const mlcc_problem_desc *desc,
                                mlcc_problem **prob) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(prob != nullptr, MLCC_E_ARG, "NULL output pointer");
    *prob = problem_new(ctx, &ctx->ex, desc);
    ctx->refs.fetch_add(1);
    return MLCC_OK;
  });
}

mlcc_status mlcc_problem_destroy(mlcc_problem *prob) {
  if (!prob) return MLCC_E_ARG;
  mlcc_context *ctx = prob->ctx;
  (void)hipStreamSynchronize(prob->ex->stream);
  delete prob;
  context_unref(ctx);
  return MLCC_OK;
}

mlcc_status mlcc_problem_dims(const mlcc_problem *P, int64_t dims[8]) {
  if (!P || !dims) return MLCC_E_ARG;
  dims[0] = P->d.O;
  dims[1] = P->d.V;
  dims[2] = P->d.J;
  dims[3] = P->d.o;
  dims[4] = P->d.v;
  dims[5] = P->d.M;
  dims[6] = P->d.n1;
  dims[7] = P->dim();
  return MLCC_OK;
}

mlcc_status mlcc_set_amplitudes(mlcc_problem *P, const double *t1, const double *x2) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(t1 != nullptr, MLCC_E_ARG, "NULL t1");
    Exec &ex = *P->ex;
    In a(*P, t1, P->d.n1);
    MLCC_HIP(hipMemcpyAsync(P->t1(), a.p, P->d.n1 * sizeof(double), hipMemcpyDeviceToDevice,
                            ex.stream));
    const int64_t MM = P->d.M * P->d.M;
    if (P->has_doubles()) {
      if (x2) {
        P->ensure_doubles();
        In b(*P, x2, MM);
        MLCC_HIP(hipMemcpyAsync(P->x2(), b.p, MM * sizeof(double), hipMemcpyDeviceToDevice,
                                ex.stream));
        MLCC_HIP(hipStreamSynchronize(ex.stream));
      } else {
        MLCC_REQUIRE(P->model == MLCC_MLCC2, MLCC_E_ARG, "MLCCSD needs t2");
      }
      P->x2_set = x2 != nullptr && P->model == MLCC_MLCC2;
    }
    MLCC_HIP(hipStreamSynchronize(ex.stream));
    P->have_amp = true;
    P->state_valid = false;
    P->jac_ready = false;
    return MLCC_OK;
  });
}

mlcc_status mlcc_residual(mlcc_problem *P, double *omega1, double *omega2, double *x2_out,
                          double *e_corr) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(P->have_amp, MLCC_E_STATE, "no amplitudes set");
    MLCC_REQUIRE(omega1 != nullptr, MLCC_E_ARG, "NULL omega1");
    // MLCC2 keeps its doubles arrays only on request
    P->want_s = x2_out != nullptr && P->has_doubles();
    P->want_om2 = omega2 != nullptr && P->has_doubles();
    if (P->want_s || P->want_om2) P->ensure_doubles();
    try {
      P->compute_state(false);
    } catch (...) {
      P->want_s = P->want_om2 = false;
      throw;
    }
    P->want_s = P->want_om2 = false;
    Exec &ex = *P->ex;
    const int64_t MM = P->d.M * P->d.M;
    Out o1(*P, omega1, P->d.n1);
    MLCC_HIP(hipMemcpyAsync(o1.p, P->om.p, P->d.n1 * sizeof(double), hipMemcpyDeviceToDevice,
                            ex.stream));
    o1.commit();
    if (omega2 && P->has_doubles()) {
      Out o2(*P, omega2, MM);
      MLCC_HIP(hipMemcpyAsync(o2.p, P->om2(), MM * sizeof(double),
                              hipMemcpyDeviceToDevice, ex.stream));
      o2.commit();
      MLCC_HIP(hipStreamSynchronize(ex.stream));
    }
    if (x2_out && P->has_doubles()) {
      Out o3(*P, x2_out, MM);
      MLCC_HIP(hipMemcpyAsync(o3.p, P->x2(), MM * sizeof(double), hipMemcpyDeviceToDevice,
                              ex.stream));
      o3.commit();
      MLCC_HIP(hipStreamSynchronize(ex.stream));
    }
    if (e_corr) *e_corr = P->e_corr;
    MLCC_HIP(hipStreamSynchronize(ex.stream));
    return MLCC_OK;
  });
}

mlcc_status mlcc_ground_state(mlcc_problem *P, const mlcc_solver_opts *opts, double *t1_out,
                              double *e_corr, mlcc_info *info) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(opts != nullptr, MLCC_E_ARG, "NULL options");
    MLCC_REQUIRE(opts->tol > 0, MLCC_E_ARG, "tolerance must be positive");
    if (!P->have_amp) {
      MLCC_HIP(hipMemsetAsync(P->amp.p, 0, P->amp.bytes, P->ex->stream));
    }
    P->x2_set = false;
    mlcc_info inf{};
    const mlcc_status st = ground_state(*P, *opts, inf);
    if (t1_out) {
      Out o(*P, t1_out, P->d.n1);
      MLCC_HIP(hipMemcpyAsync(o.p, P->t1(), P->d.n1 * sizeof(double), hipMemcpyDeviceToDevice,
                              P->ex->stream));
      o.commit();
      MLCC_HIP(hipStreamSynchronize(P->ex->stream));
    }
    if (e_corr) *e_corr = inf.energy;
    if (info) *info = inf;
    return st;
  });
}

mlcc_status mlcc_jacobian_transform(mlcc_problem *P, int32_t n_vec, const double *c,
                                    double *sigma) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(P->have_amp, MLCC_E_STATE, "no amplitudes set");
    MLCC_REQUIRE(n_vec >= 0 && c && sigma, MLCC_E_ARG, "bad vectors");
    if (n_vec == 0) return MLCC_OK;
    if (!P->jac_ready) P->prepare_jacobian();
    const int64_t n = (int64_t)n_vec * P->dim();
    In ci(*P, c, n);
    Out so(*P, sigma, n);
    P->transform(n_vec, ci.p, so.p);
    so.commit();
    MLCC_HIP(hipStreamSynchronize(P->ex->stream));
    return MLCC_OK;
  });
}

mlcc_status mlcc_jacobian_transform_eff(mlcc_problem *P, double omega, int32_t n_vec,
                                        const double *c1, double *s1) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(P->have_amp, MLCC_E_STATE, "no amplitudes set");
    MLCC_REQUIRE(P->model == MLCC_MLCC2, MLCC_E_ARG, "effective transformation is MLCC2 only");
    MLCC_REQUIRE(n_vec >= 0 && c1 && s1 && std::isfinite(omega), MLCC_E_ARG, "bad arguments");
    if (n_vec == 0) return MLCC_OK;
    if (!P->jac_ready) P->prepare_jacobian();
    const int64_t n = (int64_t)n_vec * P->d.n1;
    In ci(*P, c1, n);
    Out so(*P, s1, n);
    if (P->has_doubles()) P->transform_eff(omega, n_vec, ci.p, so.p);
    else P->transform(n_vec, ci.p, so.p);
    so.commit();
    MLCC_HIP(hipStreamSynchronize(P->ex->stream));
    return MLCC_OK;
  });
}

// guesses: unit vectors at the lowest e_A - e_I (ties: lower A, then lower I)
static std::vector<int64_t> singles_guesses(mlcc_problem &P, int n) {
  std::vector<double> d(P.d.n1);
  P.fetch_n(P.eps_vo.as<double>(), d.data(), (int)P.d.n1);
  std::vector<int64_t> idx(P.d.n1);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
  idx.resize(std::min<int64_t>(n, P.d.n1));
  return idx;
}

mlcc_status mlcc_davidson_solve(mlcc_problem *P, int32_t n_roots, const mlcc_solver_opts *opts,
                                double *omega, double *r1, mlcc_info *info) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(P->have_amp, MLCC_E_STATE, "no amplitudes (run the ground state first)");
    MLCC_REQUIRE(opts && omega, MLCC_E_ARG, "NULL argument");
    MLCC_REQUIRE(n_roots >= 1 && n_roots <= P->d.n1, MLCC_E_ARG, "bad number of roots");
    MLCC_REQUIRE(opts->tol > 0, MLCC_E_ARG, "tolerance must be positive");
    if (!P->jac_ready) P->prepare_jacobian();
    Exec &ex = *P->ex;
    const int n_guess = std::min<int64_t>(opts->n_guess > 0 ? opts->n_guess : n_roots + 2, P->d.n1);
    const int max_space = opts->max_subspace > 0 ? opts->max_subspace : 20 * n_roots;
    const int max_iter = opts->max_iter > 0 ? opts->max_iter : 100;
    const auto gidx = singles_guesses(*P, n_guess);
    mlcc_info inf{};
    std::vector<double> w(n_roots, 0.0);
    bool converged = false;
    DBuf X;
    int64_t xdim = 0;
    const double *eps_vo = P->eps_vo.as<double>(), *eps_ai = P->eps_ai.as<double>();
    if (!(opts->effective && P->model == MLCC_MLCC2 && P->has_doubles())) {
      const int64_t dim = P->dim();
      const int64_t M = P->has_doubles() ? P->d.M : 0;
      const int64_t n1 = P->d.n1;
      // The doubles live in the subspace symmetric under (ai) <-> (bj); the
      // transformed vectors and the new directions are projected onto it, so
      // that rounding-level asymmetry cannot pull the iteration towards the
      // (unphysical) antisymmetric part of the operator, whose eigenvalues
      // can lie below the physical roots.
      auto apply = [&](int n, const double *in, double *out) {
        P->transform(n, in, out);
        k::symmetrize(ex, M, out + n1, n, dim);
      };
      auto pre = [&](double wr, const double *r, double *o) {
        k::precond(ex, n1, M, eps_vo, eps_ai, wr, r, o);
        k::symmetrize(ex, M, o + n1, 1, dim);
      };
      DavidsonResult dr = davidson(ex, P->ex->al, dim, n_roots, n_guess, max_space, max_iter,
                                   opts->tol, gidx, apply, pre, nullptr, 0, 0, 0.0);
      w = dr.omega;
      converged = dr.converged;
      inf.iterations = dr.iterations;
      inf.transforms = dr.transforms;
      inf.residual = *std::max_element(dr.residual.begin(), dr.residual.end());
      for (int r = 0; r < n_roots; ++r) inf.complex_roots += dr.complex[r];
      X = std::move(dr.X);
      xdim = dim;
    } else {
      // effective singles: omega-dependent operator A_eff(w); each root is
      // iterated to self-consistency w = eigenvalue of A_eff(w), starting from
      // the roots of A_eff at the lowest singles denominator.
      const int64_t n1 = P->d.n1;
      auto pre = [&](double wr, const double *r, double *o) {
        k::precond(ex, n1, 0, eps_vo, eps_ai, wr, r, o);
      };
      std::vector<double> d0(n1);
      P->fetch_n(eps_vo, d0.data(), (int)n1);
      double w0 = *std::min_element(d0.begin(), d0.end());
      auto apply0 = [&](int n, const double *in, double *out) { P->transform_eff(w0, n, in, out); };
      DavidsonResult d0r = davidson(ex, P->ex->al, n1, n_roots, n_guess, max_space, max_iter,
                                    opts->tol, gidx, apply0, pre, nullptr, 0, 0, 0.0);
      inf.transforms += d0r.transforms;
      inf.iterations += d0r.iterations;
      X.alloc(P->ex->al, (size_t)n_roots * n1 * sizeof(double));
      converged = true;
      double worst = 0.0;
      for (int r = 0; r < n_roots; ++r) {
        double wr = d0r.omega[r];
        const double *start = d0r.X.as<double>() + (int64_t)r * n1;
        DBuf cur;
        cur.alloc(P->ex->al, n1 * sizeof(double));
        MLCC_HIP(hipMemcpyAsync(cur.p, start, n1 * sizeof(double), hipMemcpyDeviceToDevice,
                                ex.stream));
        bool ok = false;
        double resid = 0.0;
        for (int outer = 0; outer < 30; ++outer) {
          auto apply = [&](int n, const double *in, double *out) { P->transform_eff(wr, n, in, out); };
          DavidsonResult dr = davidson(ex, P->ex->al, n1, 1, 0, std::max(8, max_space / n_roots),
                                       max_iter, opts->tol, {}, apply, pre, cur.as<double>(), 1, 1,
                                       wr);
          inf.transforms += dr.transforms;
          inf.iterations += dr.iterations;
          const double wn = dr.omega[0];
          resid = dr.residual[0];
          MLCC_HIP(hipMemcpyAsync(cur.p, dr.X.p, n1 * sizeof(double), hipMemcpyDeviceToDevice,
                                  ex.stream));
          const double dw = std::fabs(wn - wr);
          wr = wn;
          if (dr.converged && dw < opts->tol) {
            ok = true;
            break;
          }
        }
        w[r] = wr;
        worst = std::max(worst, resid);
        converged = converged && ok;
        MLCC_HIP(hipMemcpyAsync(X.as<double>() + (int64_t)r * n1, cur.p, n1 * sizeof(double),
                                hipMemcpyDeviceToDevice, ex.stream));
      }
      inf.residual = worst;
      xdim = n1;
    }
    for (int r = 0; r < n_roots; ++r) omega[r] = w[r];
    if (r1) {
      Out o(*P, r1, (int64_t)n_roots * P->d.n1);
      for (int r = 0; r < n_roots; ++r)
        MLCC_HIP(hipMemcpyAsync(o.p + (int64_t)r * P->d.n1, X.as<double>() + (int64_t)r * xdim,
                                P->d.n1 * sizeof(double), hipMemcpyDeviceToDevice, ex.stream));
      o.commit();
      MLCC_HIP(hipStreamSynchronize(ex.stream));
    }
    inf.converged = converged;
    inf.energy = P->e_corr;
    if (info) *info = inf;
    return converged ? MLCC_OK : MLCC_E_NOCONV;
  });
}

mlcc_status mlcc_gemm(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N, int64_t K, int64_t R,
                      int64_t Z, double alpha, const void *A, const int64_t sA[4], const void *B,
                      const int64_t sB[4], double beta, void *C, const int64_t sC[3]) {
  return mlcc_gemm2(ctx, prec, M, N, K, R, Z, alpha, A, sA, B, sB, beta, C, sC, nullptr);
}

mlcc_status mlcc_gemm2(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N, int64_t K,
                       int64_t R, int64_t Z, double alpha, const void *A, const int64_t sA[4],
                       const void *B, const int64_t sB[4], double beta, void *C,
                       const int64_t sC[3], const int64_t lvl[6]) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    check_engine_args(prec, M, N, K, R, Z, A, sA, B, sB, C, sC, lvl, "mlcc_gemm");
    const GemmArgs a = engine_args(M, N, K, R, Z, alpha, A, sA, B, sB, beta, C, sC, lvl);
    MLCC_HIP(hipSetDevice(ctx->device));
    gemm(ctx->ex, engine_prec(prec), a, prec == MLCC_FP64);
    MLCC_HIP(hipStreamSynchronize(ctx->ex.stream));
    return MLCC_OK;
  });
}

mlcc_status mlcc_cnto(mlcc_problem *P, int32_t n_states, const double *R, const double *omega,
                      int32_t n_occ_act, int32_t n_vir_act, double *m_eig, double *n_eig,
                      double *C, double *eps_out, double *fock_out, double *L_out) {
  if (!P) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    MLCC_REQUIRE(R && omega, MLCC_E_ARG, "NULL argument");
    MLCC_REQUIRE(n_states >= 1 && n_states <= P->d.n1, MLCC_E_ARG, "bad number of states");
    MLCC_REQUIRE(n_occ_act >= 0 && n_occ_act <= P->d.O && n_vir_act >= 0 && n_vir_act <= P->d.V,
                 MLCC_E_ARG, "bad active sizes");
    MLCC_HIP(hipSetDevice(P->ctx->device));
    const int64_t n1 = P->d.n1;
    In Rin(*P, R, n_states * n1);
    std::vector<double> w(n_states);
    if (is_device_ptr(omega)) {
      MLCC_HIP(hipMemcpy(w.data(), omega, n_states * sizeof(double), hipMemcpyDeviceToHost));
    } else {
      std::copy(omega, omega + n_states, w.begin());
    }
    for (double x : w) MLCC_REQUIRE(std::isfinite(x), MLCC_E_NUMERIC, "non-finite omega");
    P->cnto(n_states, Rin.p, w.data(), n_occ_act, n_vir_act, m_eig, n_eig, C, eps_out, fock_out,
            L_out, L_out && is_device_ptr(L_out));
    return MLCC_OK;
  });
}

mlcc_status mlcc_gemm_tile(mlcc_context *ctx, int32_t bm, int32_t bn, int32_t last[2]) {
  if (!ctx || bm < 0 || bn < 0) return MLCC_E_ARG;
  if (last) {
    last[0] = ctx->ex.last_bm;
    last[1] = ctx->ex.last_bn;
  }
  ctx->ex.force_bm = bm;
  ctx->ex.force_bn = bn;
  return MLCC_OK;
}

mlcc_status mlcc_gemm_planes(mlcc_context *ctx, int32_t mode) {
  if (!ctx || mode < -1 || mode > 1) return MLCC_E_ARG;
  ctx->ex.planes_mode = mode;
  return MLCC_OK;
}

mlcc_status mlcc_pair_block_occ(mlcc_context *ctx, int32_t occ) {
  if (!ctx || occ < 0) return MLCC_E_ARG;
  ctx->pair_occ = occ;
  return MLCC_OK;
}

mlcc_status mlcc_profile_enable(mlcc_context *ctx, int32_t on) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    MLCC_HIP(hipStreamSynchronize(ctx->ex.stream));
    ctx->prof.clear();
    ctx->prof.on = on != 0;
    return MLCC_OK;
  });
}

int32_t mlcc_profile_get(mlcc_context *ctx, mlcc_kernel_stat *out, int32_t max) {
  if (!ctx) return MLCC_E_ARG;
  mlcc_status st = guarded(ctx, [&]() -> mlcc_status {
    MLCC_HIP(hipStreamSynchronize(ctx->ex.stream));
    std::vector<mlcc_kernel_stat> agg;
    for (const auto &r : ctx->prof.recs) {
      float ms = 0.f;
      MLCC_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      auto it = std::find_if(agg.begin(), agg.end(),
                             [&](const mlcc_kernel_stat &k) { return std::strcmp(k.name, r.tag) == 0; });
      if (it == agg.end()) {
        mlcc_kernel_stat k{};
        std::strncpy(k.name, r.tag, sizeof(k.name) - 1);
        agg.push_back(k);
        it = agg.end() - 1;
      }
      it->launches += 1;
      it->ms += ms;
      it->flops += r.flops;
    }
    for (int i = 0; i < (int)agg.size() && i < max; ++i) out[i] = agg[i];
    return (mlcc_status)agg.size();
  });
  return st;
}

mlcc_status mlcc_debug_get(mlcc_problem *P, int32_t which, double *out) {
  if (!P || !out) return MLCC_E_ARG;
  return guarded(P->ctx, [&]() -> mlcc_status {
    Exec &ex = *P->ex;
    const int64_t n2 = P->d.n2, J = P->d.J, MM = P->d.M * P->d.M;
    DBuf tmp;
    auto get = [&](const void *src, int64_t n, bool isf32) {
      tmp.alloc(P->ex->al, n * sizeof(double));
      if (isf32) k::convert<double, float>(ex, tmp.as<double>(), (const float *)src, n);
      else MLCC_HIP(hipMemcpyAsync(tmp.p, src, n * 8, hipMemcpyDeviceToDevice, ex.stream));
      MLCC_HIP(hipMemcpyAsync(out, tmp.p, n * 8, hipMemcpyDeviceToHost, ex.stream));
      MLCC_HIP(hipStreamSynchronize(ex.stream));
    };
    const bool f32 = P->prec != MLCC_FP64;
    switch (which) {
      case 0: MLCC_REQUIRE(P->Ft.p, MLCC_E_STATE, "no state"); get(P->Ft.p, n2, false); break;
      case 1: MLCC_REQUIRE(P->Lt.p, MLCC_E_STATE, "no state"); get(P->Lt.p, J * n2, f32); break;
      case 2: MLCC_REQUIRE(P->g.p, MLCC_E_STATE, "g~ is not stored"); get(P->g.p, MM, false); break;
      case 3: get(P->t1(), P->d.n1, false); break;
      case 4: MLCC_REQUIRE(P->x2(), MLCC_E_STATE, "no doubles stored"); get(P->x2(), MM, false); break;
      default: throw Error{MLCC_E_ARG, "unknown debug quantity"};
    }
    return MLCC_OK;
  });
}

}  // extern "C"
