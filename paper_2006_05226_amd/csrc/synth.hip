// Device-side synthetic Cholesky vectors for benchmark and serving workloads
// whose inputs are too large to stage from the host (MLCC_SYNTH_L).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with
// the published multipliers, Weyl key increments between rounds.  Counter
// (p*n + q, J, 0, 0), key (seed lo, seed hi); the first two output words give
// one standard normal by Box-Muller.  One thread per (J, p <= q) writes both
// mirrored entries, so L[J][p][q] == L[J][q][p] exactly.
#include <cmath>

#include "mlcc_internal.h"

namespace mlcc {
namespace k {
namespace {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__global__ void k_synth(double *L, int64_t J, int64_t n, double sigma, uint32_t k0,
                        uint32_t k1) {
  const int64_t per = n * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < J * per;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = t / per, pq = t - K * per;
    const int64_t p = pq / n, q = pq - p * n;
    if (q < p) continue;
    const U4 r = philox4x32_10(U4{(uint32_t)pq, (uint32_t)K, 0u, 0u}, k0, k1);
    const double u1 = ((double)r.x + 0.5) * (1.0 / 4294967296.0);
    const double u2 = ((double)r.y + 0.5) * (1.0 / 4294967296.0);
    const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    const double v = sigma * exp(-(double)K / 10.0) * z;
    L[K * per + p * n + q] = v;
    L[K * per + q * n + p] = v;
  }
}

}  // namespace

void synth_cholesky(Exec &ex, double *L, int64_t J, int64_t n, int O, int V, uint64_t seed) {
  const double sigma = 0.5 / std::sqrt((double)O * (double)V);
  const int64_t total = J * n * n;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(k_synth, dim3(blocks), dim3(256), 0, ex.stream, L, J, n, sigma,
                     (uint32_t)seed, (uint32_t)(seed >> 32));
  MLCC_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace mlcc
