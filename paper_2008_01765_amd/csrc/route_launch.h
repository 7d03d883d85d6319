// route_launch.h — launch helpers of the register-resident routing kernel.
#pragma once
#include "route_impl.h"
#include "finish_impl.h"

namespace bos {

// The kernel a routing launch runs (route_kernel, or its three-waves form).
template <int R, int LZ, int MODE>
const void* route_fn() {
  if constexpr (kW3<R, LZ, MODE>)
    return reinterpret_cast<const void*>(&route_kernel_w3<R, LZ, MODE>);
  else
    return reinterpret_cast<const void*>(&route_kernel<R, LZ, MODE>);
}
template <int R, int LZ, int MODE>
const void* route_b_fn() {
  if constexpr (kW3<R, LZ, MODE>)
    return reinterpret_cast<const void*>(&route_kernel_b_w3<R, LZ, MODE>);
  else
    return reinterpret_cast<const void*>(&route_kernel_b<R, LZ, MODE>);
}

template <int R, int LZ, int MODE>
hipError_t launch_route_t(const PassArgs& a, uint32_t nitems, uint32_t grid, hipStream_t s) {
  BOS_TRACE_BIND();
  const uint32_t m = (1u << LZ) << a.klev;
  uint32_t threads = m >> 4;
  if (threads < 64) threads = 64;
  const uint32_t lds = pass_lds_bytes(R, 1u << LZ, a.klev, (MODE & 2) && a.fin == 0, (MODE & 2) && !(MODE & 4));
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(route_fn<R, LZ, MODE>(), hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  static uint32_t occ_lds = 0, occ_blocks = 0;
  if (occ_lds != lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, route_fn<R, LZ, MODE>(), int(threads), lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    occ_lds = lds;
    occ_blocks = uint32_t(nb);
  }
  const uint32_t persistent = grid * occ_blocks;
  // the fused last pass runs one workgroup per block (ticket order); every
  // other pass is a persistent walk over the blocks
  const bool ticketed = (MODE & 2) && !(MODE & 4);
  const uint32_t g = ticketed ? nitems : (persistent < nitems ? persistent : nitems);
  if constexpr (kW3<R, LZ, MODE>)
    hipLaunchKernelGGL((route_kernel_w3<R, LZ, MODE>), dim3(g), dim3(threads), lds, s, a, nitems);
  else
    hipLaunchKernelGGL((route_kernel<R, LZ, MODE>), dim3(g), dim3(threads), lds, s, a, nitems);
  return hipGetLastError();
}

// Batched launch: nsegs segments (device tables segs / blk_start), total
// `blocks` workgroups of `threads` lanes and `lds` bytes of LDS each.
template <int R, int LZ, int MODE>
hipError_t launch_route_bt(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks,
                           uint32_t threads, uint32_t lds, hipStream_t s) {
  BOS_TRACE_BIND();
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(route_b_fn<R, LZ, MODE>(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if constexpr (kW3<R, LZ, MODE>)
    hipLaunchKernelGGL((route_kernel_b_w3<R, LZ, MODE>), dim3(blocks), dim3(threads), lds, s, segs, blk_start,
                       nsegs);
  else
    hipLaunchKernelGGL((route_kernel_b<R, LZ, MODE>), dim3(blocks), dim3(threads), lds, s, segs, blk_start, nsegs);
  return hipGetLastError();
}

template <int R, int LZ>
hipError_t launch_route_bm(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks,
                           uint32_t threads, uint32_t lds, int mode, hipStream_t s) {
  switch (mode) {
    case 0: return launch_route_bt<R, LZ, 0>(segs, blk_start, nsegs, blocks, threads, lds, s);
    case 1: return launch_route_bt<R, LZ, 1>(segs, blk_start, nsegs, blocks, threads, lds, s);
    case 2: return launch_route_bt<R, LZ, 2>(segs, blk_start, nsegs, blocks, threads, lds, s);
    case 6: return launch_route_bt<R, LZ, 6>(segs, blk_start, nsegs, blocks, threads, lds, s);
    default: return launch_route_bt<R, LZ, 3>(segs, blk_start, nsegs, blocks, threads, lds, s);
  }
}

template <int R, int LZ>
hipError_t launch_route_m(const PassArgs& a, int mode, uint32_t nitems, uint32_t grid, hipStream_t s) {
  // blocks of at least 1024 slots fill whole waves: the unguarded kernels
  const bool full = ((uint32_t(1u << LZ) << a.klev) >> 4) >= 64u;
  // a first pass (not also the last) whose groups all start on a multiple of
  // 8 elements runs the build without the staged loads
  const bool aligned = mode == 1 && full && (a.n & ((8ull << a.levels) - 1ull)) == 0;
  switch (mode | (full ? 16 : 0) | (aligned ? 32 : 0)) {
    case 0: return launch_route_t<R, LZ, 0>(a, nitems, grid, s);
    case 1: return launch_route_t<R, LZ, 1>(a, nitems, grid, s);
    case 2: return launch_route_t<R, LZ, 2>(a, nitems, grid, s);
    case 3: return launch_route_t<R, LZ, 3>(a, nitems, grid, s);
    case 6: return launch_route_t<R, LZ, 6>(a, nitems, grid, s);
    case 16: return launch_route_t<R, LZ, 16>(a, nitems, grid, s);
    case 17: return launch_route_t<R, LZ, 17>(a, nitems, grid, s);
    case 18: return launch_route_t<R, LZ, 18>(a, nitems, grid, s);
    case 19: return launch_route_t<R, LZ, 19>(a, nitems, grid, s);
    case 22: return launch_route_t<R, LZ, 22>(a, nitems, grid, s);
    case 49: return launch_route_t<R, LZ, 49>(a, nitems, grid, s);
    default: return hipErrorInvalidValue;
  }
}

// Per-bin finish of bos_orp (finish_impl.h): a persistent walk over groups of
// bins, as many workgroups as fit on `grid` compute units at once; the fast
// kernel, then the exact one (which returns at once unless a key tie was
// flagged).  *a.tie must be zero on entry.
template <int R, int LZ, bool EXACT>
hipError_t launch_orp_finish_e(const FinishArgs& a, uint32_t grid, hipStream_t s) {
  BOS_TRACE_BIND();
  constexpr uint32_t HL = (1u << LZ) >> 4, BPW = kFinishThreads / HL;
  const uint32_t lds = finish_lds_bytes(R, LZ, EXACT);
  static bool attr_set = false;
  static uint32_t occ = 0;
  const void* fn = reinterpret_cast<const void*>(&orp_finish_kernel<R, LZ, EXACT>);
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, int(kFinishThreads), lds) != hipSuccess || nb < 1)
      nb = 1;
    occ = uint32_t(nb);
    attr_set = true;
  }
  const uint64_t nb = a.gb_hi ? a.gb_hi - a.gb_lo : a.nbins;  // a staged launch finishes bins [gb_lo, gb_hi)
  const uint64_t groups = (nb + BPW - 1) / BPW;
  const uint64_t cap = uint64_t(grid) * occ;
  const uint32_t g = uint32_t(groups < cap ? groups : cap);
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL((orp_finish_kernel<R, LZ, EXACT>), dim3(g), dim3(kFinishThreads), lds, s, a);
  return hipGetLastError();
}

template <int R, int LZ>
hipError_t launch_orp_finish_t(const FinishArgs& a, uint32_t grid, hipStream_t s) {
  hipError_t e = launch_orp_finish_e<R, LZ, false>(a, grid, s);
  if (e == hipSuccess && LZ <= 10) e = launch_orp_finish_e<R, LZ, true>(a, grid, s);
  return e;
}

}  // namespace bos
