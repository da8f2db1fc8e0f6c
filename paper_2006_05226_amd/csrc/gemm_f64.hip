// Contraction engine instantiation: FP64 operands, FP64 output, operands that load as
// 16-byte groups throughout.
#include "gemm_kernel.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<double, double, BMv, BNv, true>, &gk::tile_occupancy<double, double, BMv, BNv, true>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
}  // namespace

void gemm_f64(Exec &ex, const GemmArgs &a) {
  if (a.K > 0 && a.R > 0 && gk::gemm_vonly(a, gk::Tr<double>::VEC))
    gk::dispatch<double, double>(ex, a, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0])));
  else
    gemm_f64_general(ex, a);
}

}  // namespace mlcc
