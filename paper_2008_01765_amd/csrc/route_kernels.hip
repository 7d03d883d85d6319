// route_kernels.hip — dispatch of the register-resident routing kernels
// (route_impl.h) over record size and Z; the instantiations live in
// route_r*_z*.hip so that they compile in parallel.
#include "bos_common.h"

namespace bos {
hipError_t launch_route_r8_z4(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z5(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z6(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z7(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z8(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z9(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z10(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r8_z11(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z4(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z5(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z6(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z7(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z8(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z9(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z10(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);
hipError_t launch_route_r16_z11(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s);

// Routing pass with the register-resident kernel (Z in [16, 2048], klev >= 1);
// split: the split form of a last pass that is not also the first (sorting
// finish only).
hipError_t launch_route(int rec, const PassArgs& a, bool first, bool last, uint32_t nitems, uint32_t grid,
                        hipStream_t s, bool split) {
  if (split && (first || !last)) return hipErrorInvalidValue;
  const int mode = (first ? 1 : 0) | (last ? 2 : 0) | (split ? 4 : 0);
  if (rec == 8) {
    switch (a.lz) {
    case 4: return launch_route_r8_z4(a, mode, nitems, grid, s);
    case 5: return launch_route_r8_z5(a, mode, nitems, grid, s);
    case 6: return launch_route_r8_z6(a, mode, nitems, grid, s);
    case 7: return launch_route_r8_z7(a, mode, nitems, grid, s);
    case 8: return launch_route_r8_z8(a, mode, nitems, grid, s);
    case 9: return launch_route_r8_z9(a, mode, nitems, grid, s);
    case 10: return launch_route_r8_z10(a, mode, nitems, grid, s);
    default: return launch_route_r8_z11(a, mode, nitems, grid, s);
    }
  }
  switch (a.lz) {
    case 4: return launch_route_r16_z4(a, mode, nitems, grid, s);
    case 5: return launch_route_r16_z5(a, mode, nitems, grid, s);
    case 6: return launch_route_r16_z6(a, mode, nitems, grid, s);
    case 7: return launch_route_r16_z7(a, mode, nitems, grid, s);
    case 8: return launch_route_r16_z8(a, mode, nitems, grid, s);
    case 9: return launch_route_r16_z9(a, mode, nitems, grid, s);
    case 10: return launch_route_r16_z10(a, mode, nitems, grid, s);
    default: return launch_route_r16_z11(a, mode, nitems, grid, s);
  }
}

hipError_t launch_route_b_r8_z5(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r8_z8(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r8_z9(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r8_z10(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r16_z5(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r16_z8(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r16_z9(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);
hipError_t launch_route_b_r16_z10(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads, uint32_t lds, int mode, hipStream_t s);

// Batched routing pass (all segments share record size, Z and mode); batches
// are built for Z in {256, 512, 1024} and, for tests of the overflow path, 32.
// split: the split form of a last pass that is not also the first.
hipError_t launch_route_batched(int rec, uint32_t lz, bool first, bool last, const PassArgs* segs,
                                const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads,
                                uint32_t lds, hipStream_t s, bool split) {
  if (split && (first || !last)) return hipErrorInvalidValue;
  const int mode = (first ? 1 : 0) | (last ? 2 : 0) | (split ? 4 : 0);
  if (rec == 8) {
    switch (lz) {
      case 5: return launch_route_b_r8_z5(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
      case 8: return launch_route_b_r8_z8(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
      case 9: return launch_route_b_r8_z9(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
      case 10: return launch_route_b_r8_z10(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
      default: return hipErrorNotSupported;
    }
  }
  switch (lz) {
    case 5: return launch_route_b_r16_z5(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
    case 8: return launch_route_b_r16_z8(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
    case 9: return launch_route_b_r16_z9(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
    case 10: return launch_route_b_r16_z10(segs, blk_start, nsegs, blocks, threads, lds, mode, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t launch_orp_finish_r8_z4(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z5(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z6(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z7(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z8(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z9(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z10(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r8_z11(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z4(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z5(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z6(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z7(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z8(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z9(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z10(const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_orp_finish_r16_z11(const FinishArgs& a, uint32_t grid, hipStream_t s);

// Per-bin finish of bos_orp after a split last pass (Z in [16, 2048]).
hipError_t launch_orp_finish(int rec, uint32_t lz, const FinishArgs& a, uint32_t grid, hipStream_t s) {
  if (rec == 8) {
    switch (lz) {
      case 4: return launch_orp_finish_r8_z4(a, grid, s);
      case 5: return launch_orp_finish_r8_z5(a, grid, s);
      case 6: return launch_orp_finish_r8_z6(a, grid, s);
      case 7: return launch_orp_finish_r8_z7(a, grid, s);
      case 8: return launch_orp_finish_r8_z8(a, grid, s);
      case 9: return launch_orp_finish_r8_z9(a, grid, s);
      case 10: return launch_orp_finish_r8_z10(a, grid, s);
      case 11: return launch_orp_finish_r8_z11(a, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (lz) {
    case 4: return launch_orp_finish_r16_z4(a, grid, s);
    case 5: return launch_orp_finish_r16_z5(a, grid, s);
    case 6: return launch_orp_finish_r16_z6(a, grid, s);
    case 7: return launch_orp_finish_r16_z7(a, grid, s);
    case 8: return launch_orp_finish_r16_z8(a, grid, s);
    case 9: return launch_orp_finish_r16_z9(a, grid, s);
    case 10: return launch_orp_finish_r16_z10(a, grid, s);
    case 11: return launch_orp_finish_r16_z11(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bos
