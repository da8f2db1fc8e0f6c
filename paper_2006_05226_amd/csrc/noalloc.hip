// The contraction engine for callers that cannot allocate (mlcc_gemm_noalloc):
// the partial sums of split reductions go to a fixed device array instead of
// the context's growable workspace.
//
// The array is a file-scope __device__ object, so each GPU the library runs on
// holds its own copy until the process ends.  In host code its name is only a
// stand-in for the symbol: its device address on a given GPU is taken once,
// with that GPU current, by hipGetSymbolAddress (when the first context on the
// GPU is created) and only that address is ever handed to kernels.
#include <mutex>

#include "api_util.h"

namespace mlcc {
namespace {

__device__ __align__(256) unsigned char scratch[MLCC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};        // device address of scratch per GPU
hipError_t g_err[kMaxDevices] = {};   // failure of the address query, if any
bool g_done[kMaxDevices] = {};

}  // namespace

void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  // the caller has made `device` current
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_err[device] = e;
  g_done[device] = true;
}

namespace {
void *scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  MLCC_REQUIRE(device >= 0 && device < kMaxDevices && g_done[device], MLCC_E_STATE,
               "mlcc_gemm_noalloc: no context was created on this device");
  MLCC_REQUIRE(g_ptr[device] != nullptr, MLCC_E_DEVICE,
               std::string("mlcc_gemm_noalloc: address of the scratch array: ") +
                   hipGetErrorString(g_err[device]));
  return g_ptr[device];
}
}  // namespace

}  // namespace mlcc

using namespace mlcc;

extern "C" mlcc_status mlcc_gemm_noalloc(mlcc_context *ctx, int32_t prec, int64_t M, int64_t N,
                                         int64_t K, int64_t R, int64_t Z, double alpha,
                                         const void *A, const int64_t sA[4], const void *B,
                                         const int64_t sB[4], double beta, void *C,
                                         const int64_t sC[3], const int64_t lvl[6]) {
  if (!ctx) return MLCC_E_ARG;
  return guarded(ctx, [&]() -> mlcc_status {
    check_engine_args(prec, M, N, K, R, Z, A, sA, B, sB, C, sC, lvl, "mlcc_gemm_noalloc");
    GemmArgs a = engine_args(M, N, K, R, Z, alpha, A, sA, B, sB, beta, C, sC, lvl);
    MLCC_HIP(hipSetDevice(ctx->device));
    a.work = scratch_of(ctx->device);
    a.work_cap = MLCC_NOALLOC_SCRATCH_BYTES;
    // a lane of its own: the context's stream and tile override, no
    // allocator (operands are the caller's) and no profiler (its events
    // would be created on first use)
    Exec ex;
    ex.stream = ctx->ex.stream;
    ex.force_bm = ctx->ex.force_bm;
    ex.force_bn = ctx->ex.force_bn;
    gemm(ex, engine_prec(prec), a, prec == MLCC_FP64);
    ctx->ex.last_bm = ex.last_bm;
    ctx->ex.last_bn = ex.last_bn;
    return MLCC_OK;
  });
}
