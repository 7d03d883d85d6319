// route_r8_z8.hip — routing kernels for 8-byte records, Z = 256.
#include "route_launch.h"

namespace bos {
hipError_t launch_route_r8_z8(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s) {
  return launch_route_m<8, 8>(a, mode, nitems, grid, s);
}
hipError_t launch_route_b_r8_z8(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks,
                               uint32_t threads, uint32_t lds, int mode, hipStream_t s) {
  return launch_route_bm<8, 8>(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
}
hipError_t launch_orp_finish_r8_z8(const FinishArgs& a, uint32_t grid, hipStream_t s) {
  return launch_orp_finish_t<8, 8>(a, grid, s);
}
}  // namespace bos
