// Entry of the contraction engine (kernel: gemm_kernel.h; one instantiation
// unit per operand type).
#include "gemm_kernel.h"

namespace mlcc {

std::pair<hipEvent_t, hipEvent_t> Profiler::next() {
  if (used == pool.size()) {
    hipEvent_t a, b;
    MLCC_HIP(hipEventCreate(&a));
    MLCC_HIP(hipEventCreate(&b));
    pool.push_back({a, b});
  }
  return pool[used++];
}

void gemm(Exec &ex, Prec prec, const GemmArgs &a, bool out_f64) {
  if (a.M <= 0 || a.N <= 0 || a.Z <= 0) return;
  MLCC_REQUIRE(a.Z <= ((int64_t)1 << 24), MLCC_E_ARG, "gemm: batch count too large");
  GemmArgs b = a;
  b.slack = ex.al && ex.al->owns(a.A) && ex.al->owns(a.B);
  b.bf16x3 = prec == Prec::BF16X3 || prec == Prec::BF16;
  b.bf16_plain = false;
  if (prec == Prec::BF16 && ex.bf16_map)
    for (const std::string &t : *ex.bf16_map)
      if (t == a.tag) b.bf16_plain = true;
  if (prec == Prec::F64) gemm_f64(ex, b);
  else if (out_f64) gemm_f32_out64(ex, b);
  else gemm_f32(ex, b);
}

}  // namespace mlcc
