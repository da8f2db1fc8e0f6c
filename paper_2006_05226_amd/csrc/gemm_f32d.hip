// Contraction engine instantiation: FP32 operands, FP64 output.
#include "gemm_kernel.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, double, BMv, BNv>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
}  // namespace

void gemm_f32_out64(Exec &ex, const GemmArgs &a) {
  if (a.K <= 0 || a.R <= 0) {
    // empty reduction: C = beta * Cin (a strided copy / scale); no A, B reads
    GemmArgs b = a;
    b.K = 0;
    b.R = 1;
    b.alpha = 0.0;
    gk::launch_tile<float, double, 32, 32>(ex, b, 1);
    return;
  }
  gk::dispatch<float, double>(ex, a, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0])));
}

}  // namespace mlcc
