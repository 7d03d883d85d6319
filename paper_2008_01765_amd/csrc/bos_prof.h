// bos_prof.h — optional per-launch timing with HIP events (measurement hook).
// When enabled through bos_profile_enable(), every kernel launch of the method
// is bracketed by two events on its own stream; bos_profile_read() returns the
// elapsed time and the algorithmic HBM bytes of each launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bos {
void prof_begin(uint32_t kind, uint32_t index, uint64_t bytes, hipStream_t s);
void prof_end(hipStream_t s);
}  // namespace bos
