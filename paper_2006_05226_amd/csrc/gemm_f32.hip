// Contraction engine instantiation: FP32 operands, FP32 output, operands that load as
// 16-byte groups throughout (FP32 MFMA, or split or plain products on the
// BF16 matrix cores).
#include "gemm_kernel.h"
#include "gemm_split.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, float, BMv, BNv, true>, &gk::tile_occupancy<float, float, BMv, BNv, true>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, float, BMv, BNv, true, 1>, &gk::tile_occupancy<float, float, BMv, BNv, true, 1>},
const gk::Tile kSplitTiles[] = {MLCC_GEMM_TILES_SPLIT(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, float, BMv, BNv, true, 2>, &gk::tile_occupancy<float, float, BMv, BNv, true, 2>},
const gk::Tile kPlainTiles[] = {MLCC_GEMM_TILES_PLAIN(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
}  // namespace

void gemm_f32(Exec &ex, const GemmArgs &a) {
  if (a.K > 0 && a.R > 0 && gk::gemm_split_ok(a) && a.bf16_plain)
    gk::dispatch_load<float, float>(ex, a, kPlainTiles, (int)(sizeof(kPlainTiles) / sizeof(kPlainTiles[0])),
                                 48.0);
  else if (a.K > 0 && a.R > 0 && gk::gemm_split_ok(a))
    gk::dispatch_load<float, float>(ex, a, kSplitTiles, (int)(sizeof(kSplitTiles) / sizeof(kSplitTiles[0])),
                                 48.0);
  else if (a.K > 0 && a.R > 0 && gk::gemm_vonly(a, gk::Tr<float>::VEC))
    gk::dispatch_load<float, float>(ex, a, kTiles, (int)(sizeof(kTiles) / sizeof(kTiles[0])), 16.0);
  else
    gemm_f32_general(ex, a);
}

}  // namespace mlcc
