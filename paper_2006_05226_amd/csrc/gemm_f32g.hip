// Contraction engine instantiation: FP32 operands, FP32 output, general operands (element-wise
// loads where 16-byte groups do not fit).
#include "gemm_kernel.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, float, BMv, BNv, false>, &gk::tile_occupancy<float, float, BMv, BNv, false>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES_GENERAL(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
}  // namespace

void gemm_f32_general(Exec &ex, const GemmArgs &a) {
  if (a.K <= 0 || a.R <= 0) {
    // empty reduction: C = beta * Cin (a strided copy / scale); no A, B reads
    GemmArgs b = a;
    b.K = 0;
    b.R = 1;
    b.alpha = 0.0;
    gk::launch_tile<float, float, 32, 32, false>(ex, b, 1);
    return;
  }
  gk::dispatch_load<float, float>(ex, a, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0])), 16.0);
}

}  // namespace mlcc
