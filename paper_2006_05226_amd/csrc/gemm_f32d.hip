// Contraction engine instantiation: FP32 operands, FP64 output, operands that load as
// 16-byte groups throughout (FP32 MFMA, or split or plain products on the
// BF16 matrix cores, from packed planes for the large ones).
#include "gemm_kernel.h"
#include "gemm_planes.h"

namespace mlcc {
namespace {
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, double, BMv, BNv, true>, &gk::tile_occupancy<float, double, BMv, BNv, true>},
const gk::Tile kTiles[] = {MLCC_GEMM_TILES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, double, BMv, BNv, true, 1>, &gk::tile_occupancy<float, double, BMv, BNv, true, 1>},
const gk::Tile kSplitTiles[] = {MLCC_GEMM_TILES_SPLIT(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv) {BMv, BNv, &gk::launch_tile<float, double, BMv, BNv, true, 2>, &gk::tile_occupancy<float, double, BMv, BNv, true, 2>},
const gk::Tile kPlainTiles[] = {MLCC_GEMM_TILES_PLAIN(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv, WMv, WNv, KSv, NSv) {BMv, BNv, WMv * WNv, KSv, &gk::launch_planes<double, BMv, BNv, WMv, WNv, false, KSv, NSv>, &gk::planes_occupancy<double, BMv, BNv, WMv, WNv, false, KSv, NSv>},
const gk::PlaneTile kSplitPlanes[] = {MLCC_GEMM_TILES_PLANES(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv, WMv, WNv, KSv, NSv) {BMv, BNv, WMv * WNv, KSv, &gk::launch_planes<double, BMv, BNv, WMv, WNv, true, KSv, NSv>, &gk::planes_occupancy<double, BMv, BNv, WMv, WNv, true, KSv, NSv>},
const gk::PlaneTile kPlainPlanes[] = {MLCC_GEMM_TILES_PLANES_PLAIN(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
#define MLCC_TILE_ENTRY(BMv, BNv, WMv, WNv, KSv, NSv) {BMv, BNv, WMv * WNv, KSv, &gk::launch_planes<double, BMv, BNv, WMv, WNv, true, KSv, NSv, true>, &gk::planes_occupancy<double, BMv, BNv, WMv, WNv, true, KSv, NSv, true>},
const gk::PlaneTile kF32Planes[] = {MLCC_GEMM_TILES_PLANES_F32(MLCC_TILE_ENTRY)};
#undef MLCC_TILE_ENTRY
template <typename T, int N> constexpr int count(const T (&)[N]) { return N; }
}  // namespace

void gemm_f32_out64(Exec &ex, const GemmArgs &a) {
  if (a.K > 0 && a.R > 0 && gk::gemm_split_ok(a)) {
    const bool plain = a.bf16_plain;
    if (gk::use_planes(ex, a, plain)) {
      if (plain) gk::gemm_planes<double>(ex, a, true, kPlainPlanes, count(kPlainPlanes));
      else gk::gemm_planes<double>(ex, a, false, kSplitPlanes, count(kSplitPlanes));
    } else if (plain) {
      gk::dispatch_load<float, double>(ex, a, kPlainTiles, count(kPlainTiles), 48.0);
    } else {
      gk::dispatch_load<float, double>(ex, a, kSplitTiles, count(kSplitTiles), 48.0);
    }
  } else if (gk::planes_any_layout(ex, a)) {
    gk::gemm_planes<double>(ex, a, false, kSplitPlanes, count(kSplitPlanes));
  } else if (!a.bf16x3 && gk::use_planes_f32(ex, a)) {
    gk::gemm_planes_f32<double>(ex, a, kF32Planes, count(kF32Planes));
  } else if (a.K > 0 && a.R > 0 && gk::gemm_vonly(a, gk::Tr<float>::VEC)) {
    gk::dispatch_load<float, double>(ex, a, kTiles, count(kTiles), 16.0);
  } else {
    gemm_f32_out64_general(ex, a);
  }
}

}  // namespace mlcc
