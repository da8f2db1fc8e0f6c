// Contraction engine instantiation: FP32 operands, FP32 output, operands that load as
// 16-byte groups throughout.
#include "gemm_kernel.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, float, BMv, BNv, true>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
}  // namespace

void gemm_f32(Exec &ex, const GemmArgs &a) {
  if (a.K > 0 && a.R > 0 && gk::gemm_vonly(a, gk::Tr<float>::VEC))
    gk::dispatch<float, float>(ex, a, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0])));
  else
    gemm_f32_general(ex, a);
}

}  // namespace mlcc
