// strip_kernels.hip — strip of the dummies after the split form of the last
// routing pass (Section 3.2: the bins' reals, concatenated in bin order, are
// the permuted array).
//
// The last pass leaves bin gb's reals in slots gb*Z .. gb*Z + loads[gb] - 1 of
// the binned array and every routing block's real count in bsum[blk].  One
// workgroup scans the block counts into output offsets; the strip kernel then
// copies each block's bins to their offsets.  Every address is a function of
// the loads, which the method reveals (they are what a simulator of the
// access pattern gets, Lemma 3.3).
#include "bos_common.h"

namespace bos {

constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kStripThreads = 256, kStripItems = 8;

// In-place exclusive scan of v[0..count) by one workgroup: each thread sums a
// contiguous chunk, the chunk sums are scanned in LDS, then each thread
// rewrites its chunk.
__device__ __forceinline__ void scan_blocks(unsigned long long* v, uint32_t count) {
  __shared__ unsigned long long part[kScanThreads];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (count + kScanThreads - 1) / kScanThreads;
  const uint32_t b = t * per < count ? t * per : count, e = b + per < count ? b + per : count;
  unsigned long long sum = 0;
  for (uint32_t i = b; i < e; ++i) sum += v[i];
  part[t] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
    const unsigned long long x = t >= off ? part[t - off] : 0ull;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  unsigned long long run = part[t] - sum;
  for (uint32_t i = b; i < e; ++i) {
    const unsigned long long x = v[i];
    v[i] = run;
    run += x;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(unsigned long long* v, uint32_t count) {
  scan_blocks(v, count);
}

// One routing block's bins (NB = 2^klev of them) to out[boff[blk] ..).
template <int R>
__device__ __forceinline__ void strip_block(const void* binned_, const uint32_t* loads,
                                            const unsigned long long* boff, void* out_, uint64_t n, uint32_t klev,
                                            uint32_t lz, uint64_t blk) {
  using T = typename RecOf<R>::T;
  __shared__ uint32_t pre[513];  // NB <= 512: a block has at most 8192 slots, Z >= 16
  const T* binned = static_cast<const T*>(binned_);
  T* out = static_cast<T*>(out_);
  const uint32_t tid = threadIdx.x, NB = 1u << klev;
  const uint64_t bin0 = blk << klev;
  for (uint32_t j = tid; j < NB; j += kStripThreads) pre[j + 1] = loads[bin0 + j];
  __syncthreads();
  if (tid == 0) {
    pre[0] = 0;
    for (uint32_t j = 1; j <= NB; ++j) pre[j] += pre[j - 1];
  }
  __syncthreads();
  const uint32_t total = pre[NB];
  const uint64_t base = boff[blk];
  using V = typename NativeOf<T>::V;  // native vectors stay in registers
  const V* bv = reinterpret_cast<const V*>(binned);
  V* ov = reinterpret_cast<V*>(out);
  for (uint32_t q0 = 0; q0 < total; q0 += kStripThreads * kStripItems) {
    V v[kStripItems];
    uint64_t dst[kStripItems];
#pragma unroll
    for (uint32_t k = 0; k < kStripItems; ++k) {
      const uint32_t q = q0 + k * kStripThreads + tid;
      // bin j: the last with pre[j] <= q (lanes past the end read bin 0's
      // first slot and store nothing)
      const uint32_t qq = q < total ? q : 0u;
      uint32_t lo = 0, hi = NB;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= qq)
          lo = mid;
        else
          hi = mid;
      }
      v[k] = bv[((bin0 + lo) << lz) + (qq - pre[lo])];
      dst[k] = q < total ? base + q : ~0ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < kStripItems; ++k)
      if (dst[k] < n) ov[dst[k]] = v[k];
  }
}

template <int R>
__global__ __launch_bounds__(kStripThreads) void strip_kernel(const void* binned, const uint32_t* loads,
                                                              const unsigned long long* boff, void* out, uint64_t n,
                                                              uint32_t klev, uint32_t lz) {
  strip_block<R>(binned, loads, boff, out, n, klev, lz, blockIdx.x);
}

// Batched forms: one scan workgroup per instance; the strip workgroups of
// instance s are blockIdx.x in [segs[s].first, segs[s].first + nblocks).
__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel_b(const StripSeg* segs) {
  const StripSeg sg = segs[blockIdx.x];
  scan_blocks(sg.bsum, sg.nblocks);
}

template <int R>
__global__ __launch_bounds__(kStripThreads) void strip_kernel_b(const StripSeg* segs, uint32_t nsegs) {
  uint32_t lo = 0, hi = nsegs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].first <= blockIdx.x)
      lo = mid;
    else
      hi = mid;
  }
  const StripSeg sg = segs[lo];
  strip_block<R>(sg.binned, sg.loads, sg.bsum, sg.out, sg.n, sg.klev, sg.lz, blockIdx.x - sg.first);
}

// Batched scan + strip over nsegs instances (device table segs, `blocks` strip
// workgroups in all).
hipError_t launch_strip_batched(int rec, const StripSeg* segs, uint32_t nsegs, uint32_t blocks, hipStream_t s) {
  if (nsegs == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_blocks_kernel_b, dim3(nsegs), dim3(kScanThreads), 0, s, segs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || blocks == 0) return e;
  if (rec == 8)
    hipLaunchKernelGGL(strip_kernel_b<8>, dim3(blocks), dim3(kStripThreads), 0, s, segs, nsegs);
  else
    hipLaunchKernelGGL(strip_kernel_b<16>, dim3(blocks), dim3(kStripThreads), 0, s, segs, nsegs);
  return hipGetLastError();
}

hipError_t launch_strip(int rec, const void* binned, const uint32_t* loads, unsigned long long* bsum, void* out,
                        uint64_t n, uint32_t nblocks, uint32_t klev, uint32_t lz, hipStream_t s) {
  if (klev > 9 || nblocks == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, bsum, nblocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (rec == 8)
    hipLaunchKernelGGL(strip_kernel<8>, dim3(nblocks), dim3(kStripThreads), 0, s, binned, loads, bsum, out, n, klev,
                       lz);
  else
    hipLaunchKernelGGL(strip_kernel<16>, dim3(nblocks), dim3(kStripThreads), 0, s, binned, loads, bsum, out, n, klev,
                       lz);
  return hipGetLastError();
}

}  // namespace bos
