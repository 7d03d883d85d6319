// sort_kernels.hip — gfx950 kernels of the comparison sorts.
//
// 1. The non-oblivious comparison sort that finishes bucket oblivious sort
//    (Section 3.3): tiles sorted in LDS, then merge-path merge passes.  Its
//    memory accesses depend on the relative order of the (randomly permuted)
//    records only, which is what the paper's composition argument needs.
// 2. An oblivious bitonic sort (Batcher), the baseline of the paper's Table 1,
//    on the same records: tiles sorted in LDS, global strides fused four or
//    five at a time in registers, the remaining strides of every merge in LDS.
#include "bos.h"
#include "bos_common.h"
#include "bos_prof.h"

namespace bos {

constexpr uint32_t kTileThreads = 512;

__device__ __forceinline__ uint32_t lpad(uint32_t s) { return s + (s >> 5); }

// In-LDS bitonic network over `cnt` (power of two) records.  Ascending when
// dir_bit == 0, else the direction of element i is taken from bit dir_bit of
// its global index g0 + i (standard bitonic direction rule).
template <typename T>
__device__ __forceinline__ void lds_bitonic(T* s, uint32_t cnt, uint32_t k2_first, uint32_t k2_last,
                                            uint32_t j2_first, uint64_t g0) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  for (uint32_t k2 = k2_first; k2 <= k2_last; k2 <<= 1) {
    for (uint32_t j2 = (k2 == k2_first ? j2_first : (k2 >> 1)); j2 > 0; j2 >>= 1) {
      for (uint32_t p = tid; p < (cnt >> 1); p += nthr) {
        const uint32_t lo = ((p & ~(j2 - 1u)) << 1) | (p & (j2 - 1u));
        const uint32_t hi = lo + j2;
        const bool up = ((g0 + lo) & k2) == 0;
        const T a = s[lpad(lo)], b = s[lpad(hi)];
        const bool sw = up ? rec_less(b, a) : rec_less(a, b);
        s[lpad(lo)] = sel(sw, b, a);
        s[lpad(hi)] = sel(sw, a, b);
      }
      __syncthreads();
    }
  }
}

// Sort tiles of `ts` records of buf (in place) ascending; the tail tile is
// padded with maximal records in LDS.
template <int R>
__global__ __launch_bounds__(kTileThreads) void tile_sort_kernel(void* buf, uint64_t n, uint32_t ts) {
  using T = typename RecOf<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  T* B = static_cast<T*>(buf);
  const uint64_t base = uint64_t(blockIdx.x) * ts;
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x)
    s[lpad(t)] = (base + t < n) ? B[base + t] : max_rec<T>();
  __syncthreads();
  // all tiles ascending: direction taken from a bit above the tile
  lds_bitonic(s, ts, 2, ts, 1, 0);
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x)
    if (base + t < n) B[base + t] = s[lpad(t)];
}

// Number of elements of A among the first d outputs of the stable merge of
// A[0..la) and B[0..lb) (A wins ties).
template <typename T>
__device__ __forceinline__ uint64_t merge_path(const T* A, uint64_t la, const T* Bv, uint64_t lb, uint64_t d) {
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (!rec_less(Bv[d - mid - 1], A[mid]))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

constexpr uint32_t kMergeThreads = 256, kMergeItems = 8, kMergeTile = kMergeThreads * kMergeItems;

// One merge pass: runs of width w (a multiple of kMergeTile) are merged in
// pairs from src into dst.  One block produces kMergeTile outputs.
template <int R>
__global__ __launch_bounds__(kMergeThreads) void merge_pass_kernel(const void* src_, void* dst_, uint64_t n,
                                                                    uint64_t w) {
  using T = typename RecOf<R>::T;
  __shared__ T s[kMergeTile + 1];
  __shared__ uint64_t sp[4];
  const T* src = static_cast<const T*>(src_);
  T* dst = static_cast<T*>(dst_);
  const uint64_t o0 = uint64_t(blockIdx.x) * kMergeTile;
  if (o0 >= n) return;
  const uint64_t lo = (o0 / (2 * w)) * (2 * w);
  const uint64_t mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
  const T* A = src + lo;
  const T* Bv = src + mid;
  const uint64_t la = mid - lo, lb = hi - mid;
  const uint64_t d0 = o0 - lo, d1 = (o0 + kMergeTile < hi ? o0 + kMergeTile : hi) - lo;
  if (threadIdx.x == 0) sp[0] = merge_path(A, la, Bv, lb, d0);
  if (threadIdx.x == 32) sp[1] = merge_path(A, la, Bv, lb, d1);
  __syncthreads();
  const uint64_t a0 = sp[0], a1 = sp[1], b0 = d0 - a0, b1 = d1 - a1;
  const uint32_t na = uint32_t(a1 - a0), nb = uint32_t(b1 - b0), cnt = na + nb;
  for (uint32_t t = threadIdx.x; t < cnt; t += blockDim.x) s[t] = t < na ? A[a0 + t] : Bv[b0 + t - na];
  __syncthreads();
  // each thread merges kMergeItems outputs of the tile
  const uint32_t dd = threadIdx.x * kMergeItems;
  if (dd >= cnt) return;
  uint32_t l = dd > nb ? dd - nb : 0, h = dd < na ? dd : na;
  const T* SA = s;
  const T* SB = s + na;
  while (l < h) {
    const uint32_t md = (l + h) >> 1;
    if (!rec_less(SB[dd - md - 1], SA[md]))
      l = md + 1;
    else
      h = md;
  }
  uint32_t ia = l, ib = dd - l;
  const uint32_t end = dd + kMergeItems < cnt ? dd + kMergeItems : cnt;
  for (uint32_t k = dd; k < end; ++k) {
    const bool take_a = ia < na && (ib >= nb || !rec_less(SB[ib], SA[ia]));
    dst[o0 + k] = take_a ? SA[ia++] : SB[ib++];
  }
}

// ---- bitonic baseline ------------------------------------------------------

// Local phases: sort tiles of ts records with the global direction rule (the
// tile's direction alternates with bit ts of its index).
template <int R>
__global__ __launch_bounds__(kTileThreads) void bitonic_tile_kernel(void* buf, uint32_t ts) {
  using T = typename RecOf<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  T* B = static_cast<T*>(buf);
  const uint64_t base = uint64_t(blockIdx.x) * ts;
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x) s[lpad(t)] = B[base + t];
  __syncthreads();
  lds_bitonic(s, ts, 2, ts, 1, base);
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x) B[base + t] = s[lpad(t)];
}

// Strides j2 < ts of merge phase k2, in LDS.
template <int R>
__global__ __launch_bounds__(kTileThreads) void bitonic_tail_kernel(void* buf, uint32_t ts, uint64_t k2) {
  using T = typename RecOf<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  T* B = static_cast<T*>(buf);
  const uint64_t base = uint64_t(blockIdx.x) * ts;
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x) s[lpad(t)] = B[base + t];
  __syncthreads();
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const bool up = (base & k2) == 0;  // constant over the tile since k2 > ts
  for (uint32_t j2 = ts >> 1; j2 > 0; j2 >>= 1) {
    for (uint32_t p = tid; p < (ts >> 1); p += nthr) {
      const uint32_t lo = ((p & ~(j2 - 1u)) << 1) | (p & (j2 - 1u)), hi = lo + j2;
      const T a = s[lpad(lo)], b = s[lpad(hi)];
      const bool sw = up ? rec_less(b, a) : rec_less(a, b);
      s[lpad(lo)] = sel(sw, b, a);
      s[lpad(hi)] = sel(sw, a, b);
    }
    __syncthreads();
  }
  for (uint32_t t = threadIdx.x; t < ts; t += blockDim.x) B[base + t] = s[lpad(t)];
}

// RS consecutive global strides j2 = jtop, jtop/2, ..., jtop/2^(RS-1) of merge
// phase k2, fused in registers: every thread owns the 2^RS records that these
// strides connect.
template <int R, int RS>
__global__ __launch_bounds__(256) void bitonic_global_kernel(void* buf, uint64_t N, uint64_t k2, uint64_t jtop) {
  using T = typename RecOf<R>::T;
  T* B = static_cast<T*>(buf);
  const uint64_t jlow = jtop >> (RS - 1);
  const uint64_t groups = N >> RS;
  for (uint64_t gidx = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; gidx < groups;
       gidx += uint64_t(gridDim.x) * blockDim.x) {
    // base index: insert RS zero bits at positions log2(jlow) .. log2(jtop)
    const uint64_t lowpart = gidx & (jlow - 1);
    const uint64_t highpart = (gidx / jlow) << RS;
    const uint64_t base = highpart * jlow + lowpart;
    const bool up = (base & k2) == 0;
    T v[1 << RS];
#pragma unroll
    for (int e = 0; e < (1 << RS); ++e) v[e] = B[base + uint64_t(e) * jlow];
#pragma unroll
    for (int st = RS - 1; st >= 0; --st) {
#pragma unroll
      for (int e = 0; e < (1 << RS); ++e) {
        if (e & (1 << st)) continue;
        const int e2 = e | (1 << st);
        const T a = v[e], b = v[e2];
        const bool sw = up ? rec_less(b, a) : rec_less(a, b);
        v[e] = sel(sw, b, a);
        v[e2] = sel(sw, a, b);
      }
    }
#pragma unroll
    for (int e = 0; e < (1 << RS); ++e) B[base + uint64_t(e) * jlow] = v[e];
  }
}

template <int R>
__global__ void pad_copy_kernel(const void* in_, void* out_, uint64_t n, uint64_t N) {
  using T = typename RecOf<R>::T;
  const T* in = static_cast<const T*>(in_);
  T* out = static_cast<T*>(out_);
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += uint64_t(gridDim.x) * blockDim.x)
    out[i] = i < n ? in[i] : max_rec<T>();
}

// ---- launchers -------------------------------------------------------------

static uint32_t grid_for(uint64_t work, uint32_t threads, uint32_t cap) {
  uint64_t b = (work + threads - 1) / threads;
  if (b > cap) b = cap;
  if (b == 0) b = 1;
  return uint32_t(b);
}

template <typename K>
static hipError_t allow_lds(K kernel) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

uint32_t tile_lds_bytes(int rec, uint32_t ts) { return (ts + (ts >> 5)) * uint32_t(rec); }

template <int R>
static hipError_t comparison_sort_t(void* buf0, void* buf1, uint64_t n, uint32_t ts, hipStream_t s, void** result) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = allow_lds(tile_sort_kernel<R>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  *result = buf0;
  if (n <= 1) return hipSuccess;
  const uint64_t tiles = (n + ts - 1) / ts;
  prof_begin(BOS_K_SORT_TILE, 0, 2 * n * R, s);
  hipLaunchKernelGGL(tile_sort_kernel<R>, dim3(uint32_t(tiles)), dim3(kTileThreads), tile_lds_bytes(R, ts), s,
                     buf0, n, ts);
  prof_end(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* src = buf0;
  void* dst = buf1;
  uint32_t pass = 0;
  for (uint64_t w = ts; w < n; w *= 2) {
    const uint64_t blocks = (n + kMergeTile - 1) / kMergeTile;
    prof_begin(BOS_K_SORT_MERGE, pass++, 2 * n * R, s);
    hipLaunchKernelGGL(merge_pass_kernel<R>, dim3(uint32_t(blocks)), dim3(kMergeThreads), 0, s, src, dst, n, w);
    prof_end(s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    void* t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return hipSuccess;
}

// Number of merge passes the comparison sort runs for n records and tile ts.
uint32_t comparison_sort_passes(uint64_t n, uint32_t ts) {
  uint32_t c = 0;
  if (n <= 1) return 0;
  for (uint64_t w = ts; w < n; w *= 2) ++c;
  return c;
}

hipError_t launch_comparison_sort(int rec, void* buf0, void* buf1, uint64_t n, uint32_t ts, hipStream_t s,
                                  void** result) {
  return rec == 8 ? comparison_sort_t<8>(buf0, buf1, n, ts, s, result)
                  : comparison_sort_t<16>(buf0, buf1, n, ts, s, result);
}

template <int R>
static hipError_t bitonic_t(const void* in, void* out, uint64_t n, void* ws, uint64_t N, uint32_t ts,
                            hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = allow_lds(bitonic_tile_kernel<R>);
    if (e == hipSuccess) e = allow_lds(bitonic_tail_kernel<R>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(pad_copy_kernel<R>, dim3(grid_for(N, 256, 8192)), dim3(256), 0, s, in, ws, n, N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t lds = tile_lds_bytes(R, ts);
  uint32_t gpass = 0, tpass = 0;
  prof_begin(BOS_K_BITONIC_TILE, 0, 2 * N * R, s);
  hipLaunchKernelGGL(bitonic_tile_kernel<R>, dim3(uint32_t(N / ts)), dim3(kTileThreads), lds, s, ws, ts);
  prof_end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (uint64_t k2 = uint64_t(ts) * 2; k2 <= N; k2 <<= 1) {
    uint64_t j2 = k2 >> 1;
    while (j2 >= ts) {
      // strides j2 .. max(ts, j2 / 16): fuse up to 5 of them
      int rs = 1;
      while (rs < 5 && (j2 >> rs) >= ts) ++rs;
      const uint64_t groups = N >> rs;
      const dim3 g(grid_for(groups, 256, 65535)), b(256);
      prof_begin(BOS_K_BITONIC_GLOBAL, gpass++, 2 * N * R, s);
      switch (rs) {
        case 1: hipLaunchKernelGGL((bitonic_global_kernel<R, 1>), g, b, 0, s, ws, N, k2, j2); break;
        case 2: hipLaunchKernelGGL((bitonic_global_kernel<R, 2>), g, b, 0, s, ws, N, k2, j2); break;
        case 3: hipLaunchKernelGGL((bitonic_global_kernel<R, 3>), g, b, 0, s, ws, N, k2, j2); break;
        case 4: hipLaunchKernelGGL((bitonic_global_kernel<R, 4>), g, b, 0, s, ws, N, k2, j2); break;
        default: hipLaunchKernelGGL((bitonic_global_kernel<R, 5>), g, b, 0, s, ws, N, k2, j2); break;
      }
      prof_end(s);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      j2 >>= rs;
    }
    prof_begin(BOS_K_BITONIC_TAIL, tpass++, 2 * N * R, s);
    hipLaunchKernelGGL(bitonic_tail_kernel<R>, dim3(uint32_t(N / ts)), dim3(kTileThreads), lds, s, ws, ts, k2);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipMemcpyAsync(out, ws, n * R, hipMemcpyDeviceToDevice, s);
}

hipError_t launch_bitonic(int rec, const void* in, void* out, uint64_t n, void* ws, uint64_t N, uint32_t ts,
                          hipStream_t s) {
  return rec == 8 ? bitonic_t<8>(in, out, n, ws, N, ts, s) : bitonic_t<16>(in, out, n, ws, N, ts, s);
}

}  // namespace bos
