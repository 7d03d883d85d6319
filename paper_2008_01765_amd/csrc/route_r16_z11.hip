// route_r16_z11.hip — routing kernels for 16-byte records, Z = 2048.
#include "route_launch.h"

namespace bos {
hipError_t launch_route_r16_z11(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s) {
  return launch_route_m<16, 11>(a, mode, nitems, grid, s);
}
hipError_t launch_orp_finish_r16_z11(const FinishArgs& a, uint32_t grid, hipStream_t s) {
  return launch_orp_finish_t<16, 11>(a, grid, s);
}
}  // namespace bos
