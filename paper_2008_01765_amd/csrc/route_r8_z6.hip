// route_r8_z6.hip — routing kernels for 8-byte records, Z = 64.
#include "route_launch.h"

namespace bos {
hipError_t launch_route_r8_z6(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s) {
  return launch_route_m<8, 6>(a, mode, nitems, grid, s);
}
hipError_t launch_orp_finish_r8_z6(const FinishArgs& a, uint32_t grid, hipStream_t s) {
  return launch_orp_finish_t<8, 6>(a, grid, s);
}
}  // namespace bos
