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
//
// The bins arrive compacted but unsorted (reals in the order the last level
// left them).  The comparison sort that follows (Section 3.3) starts with an
// oblivious sort of fixed tiles of `tile` records: a bin inside one tile is
// put in order with its tile, so its inner order never shows.  A bin that
// straddles a tile boundary would hand the tiles a split that depends on the
// input order, so the strip sorts such a bin (an oblivious network in LDS)
// before writing it: its lower records go to the first tile.  Which bins
// straddle depends on the loads only.
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
  for (uint32_t i = b; i < e; ++i) {
    BOS_TR(0, 30, i);
    sum += v[i];
  }
  BOS_TR(0, 31, t);
  part[t] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
    if (t >= off) BOS_TR(0, 31, t - off);
    const unsigned long long x = t >= off ? part[t - off] : 0ull;
    __syncthreads();
    BOS_TR(0, 31, t);
    part[t] += x;
    __syncthreads();
  }
  BOS_TR(0, 31, t);
  unsigned long long run = part[t] - sum;
  for (uint32_t i = b; i < e; ++i) {
    BOS_TR(0, 30, i);
    const unsigned long long x = v[i];
    v[i] = run;
    run += x;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_blocks_kernel(unsigned long long* v, uint32_t count) {
  scan_blocks(v, count);
}

// First level of the block-count scan: workgroup c turns v[c*1024 ..
// c*1024 + 1023] into its exclusive scan in place (coalesced, one count per
// thread) and writes the chunk's total to tot[c]; a second, one-workgroup
// scan of tot gives every chunk's offset.
__global__ __launch_bounds__(kScanThreads) void scan_chunks_kernel(unsigned long long* v, uint32_t count,
                                                                   unsigned long long* tot) {
  __shared__ unsigned long long wsum[kScanThreads / 64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
  const uint64_t idx = uint64_t(blockIdx.x) * kScanThreads + tid;
  if (idx < count) BOS_TR(0, 30, idx);
  const unsigned long long x = idx < count ? v[idx] : 0ull;
  unsigned long long incl = x;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const unsigned long long y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) {
    BOS_TR(0, 31, wv);
    wsum[wv] = incl;
  }
  __syncthreads();
  unsigned long long before = 0, total = 0;
#pragma unroll
  for (uint32_t w = 0; w < kScanThreads / 64; ++w) {
    BOS_TR(0, 31, w);
    const unsigned long long t = wsum[w];
    before += w < wv ? t : 0ull;
    total += t;
  }
  if (idx < count) {
    BOS_TR(0, 30, idx);
    v[idx] = before + incl - x;
  }
  if (tid == 0) {
    BOS_TR(0, 32, blockIdx.x);
    tot[blockIdx.x] = total;
  }
}

// Bitonic sort of sb[0..P2) by (key, payload) (P2 a power of two), by the
// whole workgroup.
template <typename T>
__device__ __forceinline__ void lds_bitonic(T* sb, uint32_t P2) {
  for (uint32_t size = 2; size <= P2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < P2 / 2; t += kStripThreads) {
        const uint32_t i = ((t & ~(stride - 1u)) << 1) | (t & (stride - 1u)), k = i + stride;
        const bool asc = (i & size) == 0;
        BOS_TR(0, 33, i);
        BOS_TR(0, 33, k);
        const T x = sb[i], y = sb[k];
        const bool swap = asc ? rec_less(y, x) : rec_less(x, y);
        sb[i] = sel(swap, y, x);
        sb[k] = sel(swap, x, y);
      }
      __syncthreads();
    }
  }
}

// One routing block's bins (NB = 2^klev of them) to out[boff[blk] + coff[blk /
// 1024] ..) (coff null: boff alone); bins that straddle a multiple of `tile`
// are sorted first (tile = 0: none).
// Staged (out-of-core) launches read a copy of the blocks' slots (binned
// index minus bin_slot0) and write a copy of their output range (out index
// minus out0); both are 0 otherwise.
template <int R>
__device__ __forceinline__ void strip_block(const void* binned_, const uint32_t* loads,
                                            const unsigned long long* boff, const unsigned long long* coff,
                                            void* out_, uint64_t n, uint32_t klev, uint32_t lz, uint64_t blk,
                                            uint32_t tile, uint64_t bin_slot0 = 0, uint64_t out0 = 0) {
  using T = typename RecOf<R>::T;
  __shared__ uint32_t pre[513];  // NB <= 512: a block has at most 8192 slots, Z >= 16
  __shared__ uint16_t strad[512];
  __shared__ uint32_t nstrad;
  __shared__ __align__(16) unsigned char sbin_raw[2048 * R];  // one bin of at most Z <= 2048 reals
  const T* binned = static_cast<const T*>(binned_);
  T* out = static_cast<T*>(out_);
  const uint32_t tid = threadIdx.x, NB = 1u << klev;
  const uint64_t bin0 = blk << klev;
  for (uint32_t j = tid; j < NB; j += kStripThreads) {
    BOS_TR(0, 34, bin0 + j);
    BOS_TR(0, 35, j + 1);
    pre[j + 1] = loads[bin0 + j];
  }
  __syncthreads();
  if (tid == 0) {
    pre[0] = 0;
    for (uint32_t j = 1; j <= NB; ++j) BOS_TR(0, 35, j);
    for (uint32_t j = 1; j <= NB; ++j) pre[j] += pre[j - 1];
    nstrad = 0;
  }
  __syncthreads();
  BOS_TR(0, 35, NB);
  const uint32_t total = pre[NB];
  BOS_TR(0, 36, blk);
  const uint64_t base = boff[blk] + (coff ? coff[blk / kScanThreads] : 0ull);
  if (tile) {
    // the straddling bins, in bin order (tile is a power of two)
    if (tid == 0) {
      const uint32_t tl = uint32_t(__builtin_ctz(tile));
      uint32_t c = 0;
      for (uint32_t j = 0; j < NB; ++j) {
        const uint64_t b0 = base + pre[j], b1 = base + pre[j + 1];
        if (b1 - b0 >= 2 && (b0 >> tl) != ((b1 - 1) >> tl)) {
          BOS_TR(0, 37, c);
          strad[c++] = uint16_t(j);
        }
      }
      nstrad = c;
    }
    __syncthreads();
    T* sb = reinterpret_cast<T*>(sbin_raw);
    const uint32_t ns = nstrad;
    for (uint32_t k = 0; k < ns; ++k) {
      const uint32_t j = strad[k], ld = pre[j + 1] - pre[j];
      uint32_t P2 = 2;
      while (P2 < ld) P2 <<= 1;
      const T* src = binned + ((bin0 + j) << lz) - bin_slot0;
      for (uint32_t i = tid; i < P2; i += kStripThreads) {
        if (i < ld) BOS_TR(0, 38, ((bin0 + j) << lz) + i);
        BOS_TR(0, 33, i);
        sb[i] = i < ld ? src[i] : max_rec<T>();
      }
      __syncthreads();
      lds_bitonic(sb, P2);
      const uint64_t o = base + pre[j];
      for (uint32_t i = tid; i < ld; i += kStripThreads)
        if (o + i < n) {
          BOS_TR(0, 33, i);
          BOS_TR(0, 39, o + i);
          out[o + i - out0] = sb[i];
        }
      __syncthreads();
    }
  }
  const uint32_t ns = tile ? nstrad : 0u;
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
        BOS_TR(0, 35, mid);
        if (pre[mid] <= qq)
          lo = mid;
        else
          hi = mid;
      }
      // a straddling bin was written sorted above
      bool done = false;
      for (uint32_t m = 0; m < ns; ++m) {
        BOS_TR(0, 37, m);
        done |= strad[m] == lo;
      }
      BOS_TR(0, 35, lo);
      BOS_TR(0, 38, ((bin0 + lo) << lz) + (qq - pre[lo]));
      v[k] = bv[((bin0 + lo) << lz) + (qq - pre[lo]) - bin_slot0];
      dst[k] = q < total && !done ? base + q : ~0ull;
    }
#pragma unroll
    for (uint32_t k = 0; k < kStripItems; ++k)
      if (dst[k] < n) {
        BOS_TR(0, 39, dst[k]);
        ov[dst[k] - out0] = v[k];
      }
  }
}

template <int R>
__global__ __launch_bounds__(kStripThreads) void strip_kernel(const void* binned, const uint32_t* loads,
                                                              const unsigned long long* boff,
                                                              const unsigned long long* coff, void* out, uint64_t n,
                                                              uint32_t klev, uint32_t lz, uint32_t tile) {
  strip_block<R>(binned, loads, boff, coff, out, n, klev, lz, blockIdx.x, tile);
}

// Strip of blocks blk0 .. blk0 + gridDim.x - 1 from staged copies (out-of-core).
template <int R>
__global__ __launch_bounds__(kStripThreads) void strip_kernel_staged(const void* binned, const uint32_t* loads,
                                                                     const unsigned long long* boff,
                                                                     const unsigned long long* coff, void* out,
                                                                     uint64_t n, uint32_t klev, uint32_t lz,
                                                                     uint32_t tile, uint64_t blk0, uint64_t bin_slot0,
                                                                     uint64_t out0) {
  strip_block<R>(binned, loads, boff, coff, out, n, klev, lz, blk0 + blockIdx.x, tile, bin_slot0, out0);
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
  strip_block<R>(sg.binned, sg.loads, sg.bsum, nullptr, sg.out, sg.n, sg.klev, sg.lz, blockIdx.x - sg.first,
                 sg.tile);
}

// Batched scan + strip over nsegs instances (device table segs, `blocks` strip
// workgroups in all).
hipError_t launch_strip_batched(int rec, const StripSeg* segs, uint32_t nsegs, uint32_t blocks, hipStream_t s) {
  BOS_TRACE_BIND();
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

// The two-level scan of the block counts alone (bos_orp's finish reads the
// offsets): bsum scanned in place within chunks of 1024, coff the chunk offsets.
hipError_t launch_block_scan(unsigned long long* bsum, unsigned long long* coff, uint32_t nblocks, hipStream_t s) {
  BOS_TRACE_BIND();
  if (nblocks == 0 || !coff) return hipErrorInvalidValue;
  const uint32_t nchunks = (nblocks + kScanThreads - 1) / kScanThreads;
  hipLaunchKernelGGL(scan_chunks_kernel, dim3(nchunks), dim3(kScanThreads), 0, s, bsum, nblocks, coff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, coff, nchunks);
  return hipGetLastError();
}

// tile: records per tile of the comparison sort's first phase (bins that
// straddle a tile boundary are sorted); lz <= 11.  coff: device,
// nblocks / 1024 + 1 words (the chunk offsets of the two-level scan).
hipError_t launch_strip(int rec, const void* binned, const uint32_t* loads, unsigned long long* bsum,
                        unsigned long long* coff, void* out, uint64_t n, uint32_t nblocks, uint32_t klev, uint32_t lz,
                        uint32_t tile, hipStream_t s) {
  BOS_TRACE_BIND();
  if (klev > 9 || lz > 11 || nblocks == 0 || (tile & (tile - 1u)) || !coff) return hipErrorInvalidValue;
  const uint32_t nchunks = (nblocks + kScanThreads - 1) / kScanThreads;
  hipLaunchKernelGGL(scan_chunks_kernel, dim3(nchunks), dim3(kScanThreads), 0, s, bsum, nblocks, coff);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanThreads), 0, s, coff, nchunks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (rec == 8)
    hipLaunchKernelGGL(strip_kernel<8>, dim3(nblocks), dim3(kStripThreads), 0, s, binned, loads, bsum, coff, out, n,
                       klev, lz, tile);
  else
    hipLaunchKernelGGL(strip_kernel<16>, dim3(nblocks), dim3(kStripThreads), 0, s, binned, loads, bsum, coff, out, n,
                       klev, lz, tile);
  return hipGetLastError();
}

}  // namespace bos

namespace bos {

// Strip of routing blocks [blk0, blk0 + nblk) of an out-of-core sort: their
// bins' slots staged at `binned` (global slot index minus bin_slot0), their
// output range staged at `out` (global record index minus out0); bsum and coff
// already scanned (launch_block_scan).
hipError_t launch_strip_staged(int rec, const void* binned, const uint32_t* loads, const unsigned long long* bsum,
                               const unsigned long long* coff, void* out, uint64_t n, uint32_t klev, uint32_t lz,
                               uint32_t tile, uint64_t blk0, uint32_t nblk, uint64_t bin_slot0, uint64_t out0,
                               hipStream_t s) {
  BOS_TRACE_BIND();
  if (klev > 9 || lz > 11 || (tile & (tile - 1u)) || !coff) return hipErrorInvalidValue;
  if (nblk == 0) return hipSuccess;
  if (rec == 8)
    hipLaunchKernelGGL(strip_kernel_staged<8>, dim3(nblk), dim3(kStripThreads), 0, s, binned, loads, bsum, coff, out,
                       n, klev, lz, tile, blk0, bin_slot0, out0);
  else
    hipLaunchKernelGGL(strip_kernel_staged<16>, dim3(nblk), dim3(kStripThreads), 0, s, binned, loads, bsum, coff,
                       out, n, klev, lz, tile, blk0, bin_slot0, out0);
  return hipGetLastError();
}

}  // namespace bos
