// Helpers of the extern "C" boundary shared by its translation units:
// host/device pointer classification and the translation of exceptions into
// status codes and per-context error messages.
#pragma once

#include <new>
#include <stdexcept>
#include <string>

#include "problem.h"

namespace mlcc {

// Message of the last failed context creation on this host thread.
inline thread_local std::string g_create_error;

inline bool is_device_ptr(const void *p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice;
}

inline void set_error(mlcc_context *ctx, const std::string &m) {
  if (!ctx) {
    g_create_error = m;
    return;
  }
  std::lock_guard<std::mutex> lk(ctx->err_mu);
  ctx->last_error = m;
}

// Run f; no exception crosses the C interface.
template <typename F> mlcc_status guarded(mlcc_context *ctx, F &&f) {
  try {
    return f();
  } catch (const Error &e) {
    set_error(ctx, e.msg);
    return e.code;
  } catch (const std::bad_alloc &) {
    set_error(ctx, "host allocation failed");
    return MLCC_E_OOM;
  } catch (const std::exception &e) {
    set_error(ctx, e.what());
    return MLCC_E_DEVICE;
  } catch (...) {
    set_error(ctx, "unknown error");
    return MLCC_E_DEVICE;
  }
}

// Engine arguments from the strides of the C interface (sA = {m, k, r, z},
// sB = {k, n, r, z}, sC = {m, n, z}, lvl = two-level indices or NULL).
inline GemmArgs engine_args(int64_t M, int64_t N, int64_t K, int64_t R, int64_t Z, double alpha,
                            const void *A, const int64_t sA[4], const void *B,
                            const int64_t sB[4], double beta, void *C, const int64_t sC[3],
                            const int64_t *lvl) {
  GemmArgs a;
  a.M = M; a.N = N; a.K = K; a.R = R; a.Z = Z;
  a.A = A; a.sAm = sA[0]; a.sAk = sA[1]; a.sAr = sA[2]; a.sAz = sA[3];
  a.B = B; a.sBk = sB[0]; a.sBn = sB[1]; a.sBr = sB[2]; a.sBz = sB[3];
  a.C = C; a.Cin = C; a.sCm = sC[0]; a.sCn = sC[1]; a.sCz = sC[2];
  a.alpha = alpha; a.beta = beta;
  if (lvl) {
    a.Mlo = lvl[0]; a.sAm_hi = lvl[1]; a.sCm_hi = lvl[2];
    a.Nlo = lvl[3]; a.sBn_hi = lvl[4]; a.sCn_hi = lvl[5];
  }
  return a;
}

// Argument checks shared by the engine entry points.
inline void check_engine_args(int32_t prec, int64_t M, int64_t N, int64_t K, int64_t R,
                              int64_t Z, const void *A, const int64_t *sA, const void *B,
                              const int64_t *sB, void *C, const int64_t *sC, const int64_t *lvl,
                              const char *who) {
  MLCC_REQUIRE(prec == MLCC_FP64 || prec == MLCC_FP32 || prec == MLCC_BF16X3 || prec == MLCC_BF16,
               MLCC_E_ARG, "bad precision");
  MLCC_REQUIRE(M >= 0 && N >= 0 && K >= 0 && R >= 1 && Z >= 1, MLCC_E_ARG, "bad sizes");
  MLCC_REQUIRE(A && B && C && sA && sB && sC, MLCC_E_ARG, "NULL argument");
  MLCC_REQUIRE(!lvl || (lvl[0] >= 0 && lvl[3] >= 0), MLCC_E_ARG, "bad two-level sizes");
  MLCC_REQUIRE(is_device_ptr(A) && is_device_ptr(B) && is_device_ptr(C), MLCC_E_ARG,
               std::string(who) + " takes device pointers");
}

inline Prec engine_prec(int32_t prec) {
  return prec == MLCC_FP64   ? Prec::F64
         : prec == MLCC_FP32 ? Prec::F32
         : prec == MLCC_BF16 ? Prec::BF16
                             : Prec::BF16X3;
}

// Address of the no-allocation scratch array on the current device (noalloc.hip).
void noalloc_scratch_init(int device);

}  // namespace mlcc
