// route_r8_z5.hip — routing kernels for 8-byte records, Z = 32.
#include "route_launch.h"

namespace bos {
hipError_t launch_route_r8_z5(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s) {
  return launch_route_m<8, 5>(a, mode, nitems, grid, s);
}
}  // namespace bos
