// sort_kernels.hip — gfx950 kernels of the comparison sorts.
//
// 1. The non-oblivious comparison sort that finishes bucket oblivious sort
//    (Section 3.3): tiles of 4096 records sorted by a register bitonic network,
//    then merge passes (merge-path splits per 4096-record output tile).  Its
//    memory accesses depend on the relative order of the (randomly permuted)
//    records only, which is what the paper's composition argument needs.
// 2. An oblivious bitonic sort (Batcher), the baseline of the paper's Table 1,
//    on the same records: tiles of 8192 (8-byte records) or 4096 records
//    sorted by the same register network, global strides fused up to five at
//    a time in registers, the strides of every merge below the tile in one
//    register tile pass.
#include "bos.h"
#include "bos_common.h"
#include "bos_prof.h"
#include "route_impl.h"

#include <cstring>
#include <utility>

namespace bos {


// Every G-th record of a four-way merge pass's input is a sample (G = 2^kSmpLog).
template <int R>
constexpr uint32_t kSmpLog = R == 8 ? 6u : 5u;

// A sorted tile's share of the samples: the records at multiples of G.  A
// lane holds 16 consecutive records from a multiple of 16 (G >= 16), so only
// its first record can be one.
template <int R, typename T>
__device__ __forceinline__ void write_sample(void* smp, uint64_t base, uint64_t n, T first) {
  if (smp && (base & ((1ull << kSmpLog<R>) - 1)) == 0 && base < n) {
    BOS_TR(1, 41, base >> kSmpLog<R>);
    static_cast<T*>(smp)[base >> kSmpLog<R>] = first;
  }
}

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

// Number of elements of A among the first d outputs of the stable merge of
// A[0..la) and B[0..lb) (A wins ties).
template <typename T>
__device__ __forceinline__ uint64_t merge_path(const T* A, uint64_t la, const T* Bv, uint64_t lb, uint64_t d) {
  uint64_t lo = d > lb ? d - lb : 0, hi = d < la ? d : la;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    BOS_TR(1, 42, d - mid - 1);
    BOS_TR(1, 43, mid);
    if (!rec_less(Bv[d - mid - 1], A[mid]))
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// ---- register-resident tile sort and partitioned merge passes -------------

// Tiles of 2^TLOG records (TLOG = 10, 11 or 12), 16 records per thread.
template <uint32_t TLOG>
constexpr uint32_t tile_threads() { return (1u << TLOG) / 16u; }

// Tiles of 4096 records: every compare-exchange of the bitonic network pairs
// two registers of one lane.  Three layouts of the tile over 256 lanes x 16
// registers put one 4-bit group of the slot index in the register index:
// P = bits 0-3 (lane = bits 4-11), R = bits 4-7 (lane = bits 0-3 and 8-11),
// Q = bits 8-11 (lane = bits 0-7).  A phase whose stages reach a higher group
// moves the tile through LDS (padded slot s + s/16) into that group's layout
// and back, so no stage exchanges records between lanes (a lane exchange costs
// a move per record word on top of the compare-exchange).  Every LDS address
// is a function of (lane, register) only.
template <int G>
__device__ __forceinline__ uint32_t tslot(uint32_t l, uint32_t e) {
  if constexpr (G == 0) return (l << 4) | e;
  else if constexpr (G == 1) return ((l >> 4) << 8) | (e << 4) | (l & 15u);
  else return (e << 8) | l;
}

// Stages of phase KK (merges of 2^KK slots) on register bits JB .. 0 of
// layout G (slot bits 4G + JB .. 4G); a pair sorts ascending when bit KK of
// its slots is 0, and every pair does in the last phase.
template <int KK, int G, int JB, typename E>
__device__ __forceinline__ void tile_reg_stages(E (&v)[16], uint32_t l) {
  if constexpr (JB >= 0) {
    constexpr uint32_t hb = 1u << JB;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (e & hb) continue;
      const bool asc = KK == 12 || ((tslot<G>(l, e) >> KK) & 1u) == 0u;
      cx_reg(v[e], v[e | hb], asc);
    }
    tile_reg_stages<KK, G, JB - 1>(v, l);
  }
}

// Padded LDS slot tslot + tslot/16 of register e, as a lane base plus e times
// a constant: P 17 l + e, R 272 (l/16) + l mod 16 + 17 e, Q l + l/16 + 272 e.
template <int G>
__device__ __forceinline__ uint32_t tpad_base(uint32_t l) {
  if constexpr (G == 0) return 17u * l;
  else if constexpr (G == 1) return 272u * (l >> 4) + (l & 15u);
  else return l + (l >> 4);
}
template <int G>
constexpr uint32_t tpad_step() { return G == 0 ? 1u : G == 1 ? 17u : 272u; }

template <int G, typename E, typename T>
__device__ __forceinline__ void tile_to_lds(const E (&v)[16], const LdsR<T>& lds, uint32_t l) {
  const uint32_t b = tpad_base<G>(l);
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) lds.st(b + e * tpad_step<G>(), v[e]);
}
template <int G, typename E, typename T>
__device__ __forceinline__ void tile_from_lds(E (&v)[16], const LdsR<T>& lds, uint32_t l) {
  const uint32_t b = tpad_base<G>(l);
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) v[e] = lds.ld(b + e * tpad_step<G>());
}

// Phases KK .. 12 of the bitonic sort of a 4096-record tile; v holds layout P
// on entry and exit.  A lane writes back exactly the slots it read in the same
// layout, so only a change of layout needs a barrier.
template <int KK, typename E, typename T>
__device__ __forceinline__ void tile_phase(E (&v)[16], const LdsR<T>& lds, uint32_t l) {
  if constexpr (KK <= 12) {
    if constexpr (KK >= 5) {
      tile_to_lds<0>(v, lds, l);
      __syncthreads();
      if constexpr (KK >= 9) {
        tile_from_lds<2>(v, lds, l);
        tile_reg_stages<KK, 2, KK - 9>(v, l);  // slot bits KK-1 .. 8
        tile_to_lds<2>(v, lds, l);
        __syncthreads();
      }
      tile_from_lds<1>(v, lds, l);
      tile_reg_stages<KK, 1, (KK >= 9 ? 3 : KK - 5)>(v, l);  // slot bits min(KK-1, 7) .. 4
      tile_to_lds<1>(v, lds, l);
      __syncthreads();
      tile_from_lds<0>(v, lds, l);
    }
    tile_reg_stages<KK, 0, (KK >= 4 ? 3 : KK - 1)>(v, l);  // slot bits min(KK-1, 3) .. 0
    tile_phase<KK + 1>(v, lds, l);
  }
}

// Sort one tile of 2^TLOG records of buf in place (record order; slots past n
// sort last as the maximal record): 4096-record tiles with the three-layout
// network above, smaller ones with the register network of the per-bin
// finish.
template <int R, uint32_t TLOG>
__device__ __forceinline__ void tile_sort_one(void* buf, uint64_t n, uint64_t tile, void* smp) {
  using T = typename RecOf<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* srec = reinterpret_cast<T*>(smem);
  T* B = static_cast<T*>(buf);
  const uint32_t lq = threadIdx.x;
  ElemR<T> v[16];
  LdsR<T> lds{srec};
  lds.tw = 1;
  if constexpr (TLOG == 12) {
    // Loads and stores in layout Q (register e of lane l is slot 256 e + l:
    // a wave reads and writes 64 consecutive records per instruction), turned
    // into layout P through LDS before the network and back after it.
    const uint64_t t0 = tile << 12;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint64_t gi = t0 + (e << 8) + lq;
      if (gi < n) BOS_TR(1, 40, gi);
      v[e] = ElemR<T>{gi < n ? B[gi] : max_rec<T>()};
    }
    tile_to_lds<2>(v, lds, lq);
    __syncthreads();
    tile_from_lds<0>(v, lds, lq);
    tile_phase<1>(v, lds, lq);
    tile_to_lds<0>(v, lds, lq);
    __syncthreads();
    tile_from_lds<2>(v, lds, lq);
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint64_t gi = t0 + (e << 8) + lq;
      if (gi < n) {
        BOS_TR(1, 40, gi);
        B[gi] = v[e].r;
        if (smp && (gi & ((1ull << kSmpLog<R>) - 1)) == 0) {
          BOS_TR(1, 41, gi >> kSmpLog<R>);
          static_cast<T*>(smp)[gi >> kSmpLog<R>] = v[e].r;
        }
      }
    }
    return;
  }
  const uint64_t base = (tile << TLOG) + 16u * lq;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    if (base + e < n) BOS_TR(1, 40, base + e);
    v[e] = ElemR<T>{base + e < n ? B[base + e] : max_rec<T>()};
  }
  bin_bitonic<TLOG>(v, lds, 0u, lq, true);
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e)
    if (base + e < n) {
      BOS_TR(1, 40, base + e);
      B[base + e] = v[e].r;
    }
  write_sample<R>(smp, base, n, v[0].r);
}

template <int R, uint32_t TLOG>
__global__ __launch_bounds__(tile_threads<TLOG>()) void tile_sort_reg_kernel(void* buf, uint64_t n, void* smp) {
  tile_sort_one<R, TLOG>(buf, n, blockIdx.x, smp);
}

// Segment holding launch index x (largest s with segs[s].first <= x).
__device__ __forceinline__ uint32_t find_seg(const SortSeg* segs, uint32_t nsegs, uint32_t x) {
  uint32_t lo = 0, hi = nsegs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].first <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <int R, uint32_t TLOG>
__global__ __launch_bounds__(tile_threads<TLOG>()) void tile_sort_reg_kernel_b(const SortSeg* segs,
                                                                              uint32_t nsegs) {
  const SortSeg sg = segs[find_seg(segs, nsegs, blockIdx.x)];
  tile_sort_one<R, TLOG>(sg.src, sg.n, blockIdx.x - sg.first, sg.dst);
}

// Merge tiles: kMTile outputs per workgroup of 256 threads, kMItems per thread
// (16 records of 8 bytes or 8 of 16, so that a thread's loads and outputs stay
// in registers).
template <int R>
constexpr uint32_t kMTile = merge_tile_records(R);
template <int R>
constexpr uint32_t kMItems = R == 8 ? 16u : 8u;
template <int R>
constexpr uint32_t kMThreads = kMTile<R> / kMItems<R>;

// Merge-path split of output tile boundary b of one merge pass (runs of width
// w merged in pairs): absolute start of the tile's part of the left and the
// right run.
template <int R>
__device__ __forceinline__ void merge_partition_one(const void* src_, uint64_t n, uint64_t w, uint64_t* split,
                                                    uint64_t b) {
  using T = typename RecOf<R>::T;
  const T* src = static_cast<const T*>(src_);
  const uint64_t o = b * kMTile<R>;
  const uint64_t lo = o & ~(2 * w - 1);  // run widths are powers of two
  const uint64_t mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
  const uint64_t a = merge_path(src + lo, mid - lo, src + mid, hi - mid, o - lo);
  BOS_TR(1, 44, 2 * b);
  split[2 * b] = lo + a;
  split[2 * b + 1] = mid + (o - lo - a);
}

template <int R>
__global__ void merge_partition_kernel(const void* src, uint64_t n, uint64_t w, uint64_t* split, uint64_t ntiles) {
  const uint64_t b = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < ntiles) merge_partition_one<R>(src, n, w, split, b);
}

template <int R>
__global__ void merge_partition_kernel_b(const SortSeg* segs, uint32_t nsegs, uint32_t total) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total) return;
  const SortSeg sg = segs[find_seg(segs, nsegs, x)];
  merge_partition_one<R>(sg.src, sg.n, sg.w, sg.split, x - sg.first);
}

// Merge ITEMS outputs of the stable merge of SA[0..na) and SB[0..nb) (A wins
// ties), starting at output dd, by a merge-path search and a serial merge.
template <typename T, uint32_t ITEMS>
__device__ __forceinline__ void merge_items(const T* SA, uint32_t na, const T* SB, uint32_t nb, uint32_t dd,
                                            T (&out)[ITEMS]) {
  uint32_t l = dd > nb ? dd - nb : 0, h = dd < na ? dd : na;
  while (l < h) {
    const uint32_t md = (l + h) >> 1;
    BOS_TR(1, 45, dd - md - 1);
    BOS_TR(1, 46, md);
    if (!rec_less(SB[dd - md - 1], SA[md]))
      l = md + 1;
    else
      h = md;
  }
  uint32_t ia = l, ib = dd - l;
#pragma unroll
  for (uint32_t k = 0; k < ITEMS; ++k) {
    BOS_TR(1, 45, ib);
    BOS_TR(1, 46, ia);
    const bool take_a = ia < na && (ib >= nb || !rec_less(SB[ib], SA[ia]));
    const T va = SA[ia < na ? ia : 0], vb = SB[ib < nb ? ib : 0];
    out[k] = sel(take_a, va, vb);  // per word: a select of whole records goes through scratch
    ia += take_a ? 1u : 0u;
    ib += take_a ? 0u : 1u;
  }
}

// One output tile of a merge pass: load the tile's inputs into LDS, every
// thread merges kMItems outputs, outputs are staged in LDS and written
// coalesced.  When run pairs (2w records) are at least a tile long, the tile
// takes the two parts of one pair that the partition kernel found; shorter
// pairs (first passes after a tile sort of fewer than kMTile records) lie
// whole inside the tile, which then merges each of them.
template <int R>
__device__ __forceinline__ void merge_tile_one(const void* src_, void* dst_, uint64_t n, uint64_t w,
                                               const uint64_t* split, uint64_t b) {
  using T = typename RecOf<R>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  const T* src = static_cast<const T*>(src_);
  T* dst = static_cast<T*>(dst_);
  const uint64_t o0 = b * kMTile<R>;
  const bool whole_pairs = 2 * w < kMTile<R>;
  uint64_t a0 = o0, b0 = o0;
  uint32_t na = 0, nb = 0, cnt = 0;
  if (whole_pairs) {
    cnt = uint32_t((o0 + kMTile<R> < n ? o0 + kMTile<R> : n) - o0);
    na = cnt;  // the tile is read as one contiguous range
  } else {
    const uint64_t lo = o0 & ~(2 * w - 1);  // run widths are powers of two
    const uint64_t mid = lo + w < n ? lo + w : n, hi = lo + 2 * w < n ? lo + 2 * w : n;
    const uint64_t o1 = o0 + kMTile<R> < hi ? o0 + kMTile<R> : hi;
    BOS_TR(1, 44, 2 * b);
    a0 = split[2 * b];
    b0 = split[2 * b + 1];
    if (o1 != hi) BOS_TR(1, 44, 2 * b + 2);
    const uint64_t a1 = o1 == hi ? mid : split[2 * b + 2], b1 = o1 == hi ? hi : split[2 * b + 3];
    na = uint32_t(a1 - a0);
    nb = uint32_t(b1 - b0);
    cnt = na + nb;
  }
  {
    // issue every load of this thread before the first LDS store (native
    // vectors, so the array stays in registers; lanes past the tile reload a
    // valid record)
    using V = typename NativeOf<T>::V;
    const V* srcv = reinterpret_cast<const V*>(src);
    V* sv = reinterpret_cast<V*>(s);
    V in[kMItems<R>];
#pragma unroll
    for (uint32_t k = 0; k < kMItems<R>; ++k) {
      const uint32_t t = threadIdx.x + k * kMThreads<R>;
      const uint64_t gi = t < na ? a0 + t : b0 + t - na;
      BOS_TR(1, 48, t < cnt ? gi : a0);
      in[k] = srcv[t < cnt ? gi : a0];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the stores
#pragma unroll
    for (uint32_t k = 0; k < kMItems<R>; ++k) {
      const uint32_t t = threadIdx.x + k * kMThreads<R>;
      if (t < cnt) sv[t] = in[k];
    }
  }
  __syncthreads();
  const uint32_t dd = threadIdx.x * kMItems<R>;
  T out[kMItems<R>];
  if (dd < cnt) {
    // the two runs this thread merges from, and its first output among theirs
    uint32_t pb = 0, pa = na, pbn = nb;
    if (whole_pairs) {
      // this thread's outputs lie in one pair (2w is a multiple of kMItems<R>)
      const uint32_t w32 = uint32_t(w);
      pb = dd & ~(2 * w32 - 1);
      pa = cnt - pb < w32 ? cnt - pb : w32;
      pbn = cnt - pb - pa < w32 ? cnt - pb - pa : w32;
    }
    merge_items(s + pb, pa, s + pb + pa, pbn, dd - pb, out);
  }
  __syncthreads();
  if (dd < cnt) {
#pragma unroll
    for (uint32_t k = 0; k < kMItems<R>; ++k) s[dd + k + (dd >> 4)] = out[k];  // one pad slot per 16
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < kMItems<R>; ++k) {
    const uint32_t t = threadIdx.x + k * kMThreads<R>;
    if (t < cnt) {
      BOS_TR(1, 49, o0 + t);
      dst[o0 + t] = s[t + (t >> 4)];
    }
  }
}

// Compare-exchange of a lane's 16 records (register sub-tile `sub` of 4096
// records, lane lq) with those of sub-tile psub: lane 255 - lq, registers in
// reverse order when `mirror` (the first stage of a merge of two ascending
// runs), else the same lane and registers.  The lower sub-tile keeps the
// minima.  Sub-tiles exchange through their padded LDS regions (SP slots each).
template <typename T, uint32_t SP>
__device__ __forceinline__ void subtile_cross(ElemR<T> (&v)[16], T* s, uint32_t sub, uint32_t lq, uint32_t psub,
                                              bool mirror) {
  __syncthreads();  // the LDS regions are free (the last network stage read them)
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) s[sub * SP + 17u * lq + e] = v[e].r;
  __syncthreads();
  const uint32_t plq = mirror ? 255u - lq : lq;
  const bool keep_min = sub < psub;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    const ElemR<T> p{s[psub * SP + 17u * plq + (mirror ? 15u - e : e)]};
    const bool take = e_less(p, v[e]) == keep_min;
    v[e] = e_sel(take, p, v[e]);
  }
  __syncthreads();
}

// Tiles of 2^TLOG records for TLOG = 13 or 14: 2^(TLOG - 12) register tiles of
// 4096 records (256 lanes and one padded LDS region each) are sorted side by
// side, then merged with the bitonic merge network: a compare-exchange across
// two sorted runs, first element against last (which leaves two bitonic halves,
// every element of the first at most every element of the second), then the
// ascending half-cleaner stages inside each half.  It saves TLOG - 12 merge
// passes over HBM.
template <int R, uint32_t TLOG>
__device__ __forceinline__ void tile_sort_big_one(void* buf, uint64_t n, uint64_t tile, void* smp) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t kSub = 4096, kSubPad = kSub + kSub / 16;
  static_assert(TLOG == 13 || TLOG == 14, "two or four register tiles");
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  T* B = static_cast<T*>(buf);
  const uint32_t tid = threadIdx.x, sub = tid / 256u, lq = tid % 256u;
  const uint64_t base = (tile << TLOG) + uint64_t(sub) * kSub + 16u * lq;
  const LdsR<T> lds{s};
  ElemR<T> v[16];
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) v[e] = ElemR<T>{base + e < n ? B[base + e] : max_rec<T>()};
  bin_bitonic<12>(v, lds, sub * kSubPad, lq, true);
  auto cross = [&](uint32_t psub, bool mirror) { subtile_cross<T, kSubPad>(v, s, sub, lq, psub, mirror); };
  // runs of 4096 -> 8192: sub-tiles 2j, 2j+1
  cross(sub ^ 1u, true);
  bin_bitonic_merge<12>(v, lds, sub * kSubPad, lq, true);
  if constexpr (TLOG == 14) {
    // runs of 8192 -> 16384: mirror across the two runs, then the stage of
    // distance 4096 inside each run, then the stages inside every sub-tile
    cross(3u - sub, true);
    cross(sub ^ 1u, false);
    bin_bitonic_merge<12>(v, lds, sub * kSubPad, lq, true);
  }
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e)
    if (base + e < n) B[base + e] = v[e].r;
  write_sample<R>(smp, base, n, v[0].r);
}

template <int R, uint32_t TLOG>
__global__ __launch_bounds__(tile_threads<TLOG>()) void tile_sort_big_kernel(void* buf, uint64_t n, void* smp) {
  tile_sort_big_one<R, TLOG>(buf, n, blockIdx.x, smp);
}

template <int R, uint32_t TLOG>
__global__ __launch_bounds__(tile_threads<TLOG>()) void tile_sort_big_kernel_b(const SortSeg* segs,
                                                                              uint32_t nsegs) {
  const SortSeg sg = segs[find_seg(segs, nsegs, blockIdx.x)];
  tile_sort_big_one<R, TLOG>(sg.src, sg.n, blockIdx.x - sg.first, sg.dst);
}

template <int R>
__global__ __launch_bounds__(kMThreads<R>) void merge_tile_kernel(const void* src, void* dst, uint64_t n, uint64_t w,
                                                               const uint64_t* split) {
  merge_tile_one<R>(src, dst, n, w, split, blockIdx.x);
}

template <int R>
__global__ __launch_bounds__(kMThreads<R>) void merge_tile_kernel_b(const SortSeg* segs, uint32_t nsegs) {
  const SortSeg sg = segs[find_seg(segs, nsegs, blockIdx.x)];
  merge_tile_one<R>(sg.src, sg.dst, sg.n, sg.w, sg.split, blockIdx.x - sg.first);
}

// ---- four-way merge passes --------------------------------------------------
//
// A pass merges runs of width w = 2^lw in groups of four, so the comparison
// sort crosses HBM half as often.  Tiles are cut by value: every G-th record
// of the input is a sample (G = kMTile/64), and every kSplM-th record of a
// group's four sample runs merged, in the order (record, run, position), opens
// a tile.  Between two such splitters each run holds at most its splitter
// samples' G-blocks plus, for the three runs that do not own the opening
// splitter, one partial block, so a tile holds at most kSplM*G + 3(G-1)
// records (4029 of 4096 for 8-byte records, 2013 of 2048 for 16-byte ones;
// aligning the second merge result adds at most ITEMS-1 slots).

// A four-way tile is merged by 256 threads with as many records each as a
// two-way pass's thread: fewer, longer merges per thread halve the merge-path
// searches per record (8 records per thread over 512 threads, or 32 over 128,
// were slower).
template <int R>
constexpr uint32_t kM4Items = kMItems<R>;
template <int R>
constexpr uint32_t kM4Threads = kMTile<R> / kM4Items<R>;
constexpr uint32_t kSplM = 60;                  // samples per tile
// the tile bound above, with the alignment slots, fits a merge tile
static_assert(kSplM * (1u << kSmpLog<8>) + 3u * ((1u << kSmpLog<8>) - 1u) + kM4Items<8> - 1u <= kMTile<8>,
              "four-way tile bound, 8-byte records");
static_assert(kSplM * (1u << kSmpLog<16>) + 3u * ((1u << kSmpLog<16>) - 1u) + kM4Items<16> - 1u <= kMTile<16>,
              "four-way tile bound, 16-byte records");

// Does record x of run kx come before record e of run ke (x != e's slot)?
template <typename T>
__device__ __forceinline__ bool precedes(T x, uint32_t kx, T e, uint32_t ke) {
  return kx < ke ? !rec_less(e, x) : rec_less(x, e);
}

// Samples of a four-way pass's input, smp[i] = src[i*G], when a two-way pass
// produced it (the tile sort and the four-way tile kernel write their own).
template <int R>
__device__ __forceinline__ void sample_gather_one(const void* src_, void* smp_, uint64_t n, uint64_t blk) {
  using T = typename RecOf<R>::T;
  const uint64_t i = blk * blockDim.x + threadIdx.x;
  if (i < ((n + (1ull << kSmpLog<R>) - 1) >> kSmpLog<R>)) {
    BOS_TR(1, 41, i);
    static_cast<T*>(smp_)[i] = static_cast<const T*>(src_)[i << kSmpLog<R>];
  }
}
template <int R>
__global__ void sample_gather_kernel(const void* src_, void* smp_, uint64_t n) {
  sample_gather_one<R>(src_, smp_, n, blockIdx.x);
}

// Ranks of the samples in their group, kSplS<R> samples per thread with all
// their searches advancing together (one round of loads per halving).  A
// sample whose rank is a multiple of kSplM opens tile rank/kSplM of its group;
// for it, spl[4*tile + k] receives the count of run k's samples before it
// (k != its run j) and spl[4*tile + j] = kSplOwn | its sample index.
template <int R>
constexpr uint32_t kSplS = R == 8 ? 4u : 2u;  // (more would spill registers)
constexpr uint64_t kSplOwn = 1ull << 63;
template <int R>
__device__ __forceinline__ void merge4_rank_one(const void* smp_, uint64_t n, uint32_t lw, uint64_t ntf,
                                                uint64_t* spl, uint64_t blk) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t LG = kSmpLog<R>;
  constexpr uint64_t G = 1ull << LG;
  const T* smp = static_cast<const T*>(smp_);
  const uint64_t ns = (n + G - 1) >> LG, w = 1ull << lw;
  const uint64_t i0 = (blk * blockDim.x + threadIdx.x) * kSplS<R>;
  if (i0 >= ns) return;
  T e[kSplS<R>];
  uint32_t j[kSplS<R>], own[kSplS<R>], c[kSplS<R>][4], cl[kSplS<R>][4], rb[kSplS<R>][4];
  uint32_t maxl = 0;
#pragma unroll
  for (uint32_t q = 0; q < kSplS<R>; ++q) {
    const uint64_t i = i0 + q < ns ? i0 + q : i0;  // past the end: repeat the first (not stored)
    const uint64_t p = i << LG, gs = (p >> (lw + 2)) << (lw + 2);
    j[q] = uint32_t(p >> lw) & 3u;
    BOS_TR(1, 41, i);
    e[q] = smp[i];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint64_t st = gs + k * w < n ? gs + k * w : n, len = n - st < w ? n - st : w;
      rb[q][k] = uint32_t(st >> LG);
      own[q] = k == j[q] ? rb[q][k] : (k == 0 ? 0u : own[q]);
      c[q][k] = 0;
      cl[q][k] = k == j[q] ? 0u : uint32_t((len + G - 1) >> LG);
      maxl = cl[q][k] > maxl ? cl[q][k] : maxl;
    }
  }
  while (maxl > 0) {
    maxl = 0;
#pragma unroll
    for (uint32_t q = 0; q < kSplS<R>; ++q) {
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        if (cl[q][k] == 0) continue;
        const uint32_t half = cl[q][k] >> 1;
        BOS_TR(1, 41, uint64_t(rb[q][k]) + c[q][k] + half);
        if (precedes(smp[uint64_t(rb[q][k]) + c[q][k] + half], k, e[q], j[q])) {
          c[q][k] += half + 1;
          cl[q][k] -= half + 1;
        } else {
          cl[q][k] = half;
        }
        maxl = cl[q][k] > maxl ? cl[q][k] : maxl;
      }
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < kSplS<R>; ++q) {
    const uint64_t i = i0 + q;
    if (i >= ns) continue;
    const uint64_t p = i << LG, g = p >> (lw + 2);
    const uint32_t r = uint32_t(i - own[q]) + c[q][0] + c[q][1] + c[q][2] + c[q][3];
    if (r % kSplM != 0) continue;
    uint64_t* out = spl + 4 * (g * ntf + r / kSplM);
    BOS_TR(1, 50, 4 * (g * ntf + r / kSplM));
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) out[k] = k == j[q] ? (kSplOwn | i) : uint64_t(c[q][k]);
  }
}

template <int R>
__global__ void merge4_rank_kernel(const void* smp_, uint64_t n, uint32_t lw, uint64_t ntf, uint64_t* spl) {
  merge4_rank_one<R>(smp_, n, lw, ntf, spl, blockIdx.x);
}

// The same ranks when a workgroup's kSplW<R> samples lie in one run (the
// sample runs hold at least kSplW<R> samples).  One wave finds, for each other
// run k, how many of its samples precede the workgroup's first and last sample
// (64-ary searches: a round of 64 probes and a ballot narrows the range 64-fold);
// the samples between those two counts are copied to LDS, where each thread
// searches for its own samples (in global memory if the window exceeds kSplCap).
template <int R>
constexpr uint32_t kSplW = 256u * kSplS<R>;
template <int R>
constexpr uint32_t kSplCap = R == 8 ? 2048u : 1024u;
template <int R>
__device__ __forceinline__ void merge4_rank_wide_one(const void* smp_, uint64_t n, uint32_t lw, uint64_t ntf,
                                                     uint64_t* spl, uint64_t blk) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t LG = kSmpLog<R>, CAP = kSplCap<R>;
  constexpr uint64_t G = 1ull << LG;
  __shared__ T win[3 * CAP];
  __shared__ uint32_t wlo[4], wlen[4];
  const T* smp = static_cast<const T*>(smp_);
  const uint64_t ns = (n + G - 1) >> LG, w = 1ull << lw;
  const uint64_t base = blk * kSplW<R>;
  const uint64_t last = (base + kSplW<R> < ns ? base + kSplW<R> : ns) - 1;
  const uint64_t p0 = base << LG, g = p0 >> (lw + 2), gs = g << (lw + 2);
  const uint32_t j = uint32_t(p0 >> lw) & 3u;
  uint64_t rb[4];
  uint32_t sc[4];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint64_t st = gs + k * w < n ? gs + k * w : n, len = n - st < w ? n - st : w;
    rb[k] = st >> LG;
    sc[k] = uint32_t((len + G - 1) >> LG);
  }
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    BOS_TR(1, 41, base);
    BOS_TR(1, 41, last);
    const T ef = smp[base], el = smp[last];
    uint32_t lo[4][2], hi[4][2];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
      for (uint32_t b = 0; b < 2; ++b) {
        lo[k][b] = 0;
        hi[k][b] = k == j ? 0u : sc[k];
      }
    bool more = true;
    while (more) {
      more = false;
      // every open search's probe first (one round of loads), then the ballots
      T x[4][2];
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
        for (uint32_t b = 0; b < 2; ++b) {
          const uint32_t l = lo[k][b], h = hi[k][b], st = (h - l + 63) / 64, q = l + lane * st;
          BOS_TR(1, 41, l < h ? rb[k] + (q < h ? q : l) : base);
          x[k][b] = smp[l < h ? rb[k] + (q < h ? q : l) : base];  // a closed search rereads a valid sample
        }
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k)
#pragma unroll
        for (uint32_t b = 0; b < 2; ++b) {
          if (lo[k][b] >= hi[k][b]) continue;  // uniform over the wave
          const uint32_t l = lo[k][b], h = hi[k][b], st = (h - l + 63) / 64, q = l + lane * st;
          const bool pr = q < h && precedes(x[k][b], k, sel(b != 0, el, ef), j);
          const uint32_t f = uint32_t(__popcll(__ballot(pr)));
          if (f == 0) {
            hi[k][b] = l;
          } else {
            lo[k][b] = l + (f - 1) * st + 1;
            hi[k][b] = l + f * st < h ? l + f * st : h;
          }
          more = more || lo[k][b] < hi[k][b];
        }
    }
    if (lane == 0)
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        wlo[k] = lo[k][0];
        wlen[k] = lo[k][1] - lo[k][0];
      }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    if (k == j || wlen[k] > CAP) continue;
    const uint32_t slot = k < j ? k : k - 1;
    for (uint32_t t = threadIdx.x; t < wlen[k]; t += 256) {
      BOS_TR(1, 41, rb[k] + wlo[k] + t);
      BOS_TR(1, 51, slot * CAP + t);
      win[slot * CAP + t] = smp[rb[k] + wlo[k] + t];
    }
  }
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kSplS<R>; ++q) {
    const uint64_t i = base + q * 256u + threadIdx.x;
    if (i > last) continue;
    BOS_TR(1, 41, i);
    const T e = smp[i];
    uint32_t c[4];
    uint32_t r = uint32_t(i - rb[j]);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      c[k] = 0;
      if (k == j) continue;
      const uint32_t slot = k < j ? k : k - 1;
      const bool inl = wlen[k] <= CAP;
      uint32_t l = 0, len = wlen[k];
      while (len > 0) {
        const uint32_t half = len >> 1;
        if (inl) BOS_TR(1, 51, slot * CAP + l + half);
        else BOS_TR(1, 41, rb[k] + wlo[k] + l + half);
        const T x = inl ? win[slot * CAP + l + half] : smp[rb[k] + wlo[k] + l + half];
        if (precedes(x, k, e, j)) {
          l += half + 1;
          len -= half + 1;
        } else {
          len = half;
        }
      }
      c[k] = wlo[k] + l;
      r += c[k];
    }
    if (r % kSplM != 0) continue;
    uint64_t* out = spl + 4 * (g * ntf + r / kSplM);
    BOS_TR(1, 50, 4 * (g * ntf + r / kSplM));
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) out[k] = k == j ? (kSplOwn | i) : uint64_t(c[k]);
  }
}

template <int R>
__global__ __launch_bounds__(256) void merge4_rank_wide_kernel(const void* smp_, uint64_t n, uint32_t lw,
                                                               uint64_t ntf, uint64_t* spl) {
  merge4_rank_wide_one<R>(smp_, n, lw, ntf, spl, blockIdx.x);
}

// One thread per tile: the tile's exact start in each run.  Samples c-1 and
// c of run k bracket the opening sample e, so the search covers the records
// between them; the three searches advance together.
template <int R>
__device__ __forceinline__ void merge4_bound_one(const void* src_, const void* smp_, uint64_t n, uint32_t lw,
                                                 uint64_t total, uint64_t* spl, uint64_t blk) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t LG = kSmpLog<R>;
  constexpr uint64_t G = 1ull << LG;
  const T* src = static_cast<const T*>(src_);
  const uint64_t t = blk * blockDim.x + threadIdx.x;
  if (t >= total) return;
  uint64_t wd[4];
  uint32_t j = 0, owners = 0;
  BOS_TR(1, 50, 4 * t);
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    wd[k] = spl[4 * t + k];
    j = (wd[k] & kSplOwn) ? k : j;
    owners += (wd[k] & kSplOwn) ? 1u : 0u;
  }
  const uint64_t i = wd[j] & ~kSplOwn, p = i << LG, w = 1ull << lw, gs = (p >> (lw + 2)) << (lw + 2);
  // entries not of the form the rank kernel writes: mark the tile invalid
  // (the merge kernel skips it) rather than search out of bounds
  bool ok = owners == 1 && i < ((n + G - 1) >> LG);
  uint64_t st[4], lb[4], cl[4], maxl = 0;
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    st[k] = gs + k * w < n ? gs + k * w : n;
    const uint64_t len = n - st[k] < w ? n - st[k] : w;
    ok = ok && (k == j || wd[k] <= (len + G - 1) >> LG);
  }
  if (!ok) {
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) spl[4 * t + k] = ~0ull;
    return;
  }
  BOS_TR(1, 41, i);
  const T e = static_cast<const T*>(smp_)[i];
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint64_t len = n - st[k] < w ? n - st[k] : w, ck = wd[k];
    lb[k] = k == j ? p - st[k] : ck > 0 ? (ck - 1) * G + 1 : 0;
    const uint64_t hi = ck * G < len ? ck * G : len;
    cl[k] = k == j || ck == 0 ? 0 : hi - lb[k];
    maxl = cl[k] > maxl ? cl[k] : maxl;
  }
  while (maxl > 0) {
    maxl = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      if (cl[k] == 0) continue;
      const uint64_t half = cl[k] >> 1;
      BOS_TR(1, 48, st[k] + lb[k] + half);
      if (precedes(src[st[k] + lb[k] + half], k, e, j)) {
        lb[k] += half + 1;
        cl[k] -= half + 1;
      } else {
        cl[k] = half;
      }
      maxl = cl[k] > maxl ? cl[k] : maxl;
    }
  }
  BOS_TR(1, 50, 4 * t);
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) spl[4 * t + k] = st[k] + lb[k];
}

template <int R>
__global__ void merge4_bound_kernel(const void* src_, const void* smp_, uint64_t n, uint32_t lw, uint64_t total,
                                    uint64_t* spl) {
  merge4_bound_one<R>(src_, smp_, n, lw, total, spl, blockIdx.x);
}

// ITEMS outputs, from output dd on, of the merge of A (na records at slot
// xa) and B (nb records at slot xb) in LDS; PAD: slot q lives at q + q/16
// (the padded staging layout).  The current head of each side stays in
// registers, so a step reads one record.
template <bool PAD, typename T, uint32_t ITEMS>
__device__ __forceinline__ void merge_items_lds(const T* s, uint32_t xa, uint32_t na, uint32_t xb, uint32_t nb,
                                                uint32_t dd, T (&out)[ITEMS]) {
  auto at = [&](uint32_t q) {
    BOS_TR(1, 47, q);
    return PAD ? s[q + (q >> 4)] : s[q];
  };
  uint32_t l = dd > nb ? dd - nb : 0, h = dd < na ? dd : na;
  while (l < h) {
    const uint32_t md = (l + h) >> 1;
    if (!rec_less(at(xb + dd - md - 1), at(xa + md)))
      l = md + 1;
    else
      h = md;
  }
  uint32_t ia = l, ib = dd - l;
  T va = at(xa + (ia < na ? ia : 0)), vb = at(xb + (ib < nb ? ib : 0));
  // every step without branches: the conditions combine as bits and both
  // candidate slots are formed before one of them is read
#pragma unroll
  for (uint32_t k = 0; k < ITEMS; ++k) {
    const bool take_a = (ia < na) & ((ib >= nb) | !rec_less(vb, va));
    out[k] = sel(take_a, va, vb);
    ia += uint32_t(take_a);
    ib += uint32_t(!take_a);
    if (k + 1 < ITEMS) {
      const uint32_t qa = xa + (ia < na ? ia : 0u), qb = xb + (ib < nb ? ib : 0u);
      const T nv = at(take_a ? qa : qb);
      va = sel(take_a, nv, va);
      vb = sel(take_a, vb, nv);
    }
  }
}

// One tile of a four-way pass: load the tile's four run segments, merge runs
// 0+1 and 2+3 (the second result starts at an ITEMS-aligned slot so that no
// thread's outputs straddle the two), merge the two results, write the tile
// coalesced and, when smp is set, the next pass's samples.  A tile whose
// bounds are not what the splitters guarantee is skipped (no access outside
// its runs or the LDS tile).
template <int R>
__device__ __forceinline__ void merge4_tile_one(const void* src_, void* dst_, uint64_t n, uint32_t lw,
                                                const uint64_t* spl, uint64_t ntf, uint64_t ng, uint64_t ntl,
                                                void* smp_, uint64_t tile, unsigned long long* err) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t IT = kM4Items<R>, NT = kM4Threads<R>, TT = kMTile<R>, LG = kSmpLog<R>;
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  const T* src = static_cast<const T*>(src_);
  T* dst = static_cast<T*>(dst_);
  T* smp = static_cast<T*>(smp_);
  const uint64_t w = 1ull << lw, g = tile / ntf, b = tile - g * ntf, gs = g << (lw + 2);
  const uint64_t ntg = g + 1 < ng ? ntf : ntl;
  uint64_t a[4], e[4], o0 = gs;
  bool ok = b < ntg;
  BOS_TR(1, 50, 4 * tile);
  if (b + 1 < ntg) BOS_TR(1, 50, 4 * tile + 4);
#pragma unroll
  for (uint32_t k = 0; k < 4; ++k) {
    const uint64_t st = gs + k * w < n ? gs + k * w : n, en = n - st < w ? st + (n - st) : st + w;
    a[k] = spl[4 * tile + k];
    e[k] = b + 1 < ntg ? spl[4 * tile + 4 + k] : en;
    ok = ok && st <= a[k] && a[k] <= e[k] && e[k] <= en;
    o0 += a[k] - st;
  }
  // A tile whose bounds break what the splitters guarantee is skipped (no
  // access out of bounds) and reported in the error word, which the host
  // turns into a non-OK status.
  if (!ok) {
    if (threadIdx.x == 0) atomicOr(err, 1ull);
    return;
  }
  const uint32_t n0 = uint32_t(e[0] - a[0]), n1 = uint32_t(e[1] - a[1]), n2 = uint32_t(e[2] - a[2]),
                 n3 = uint32_t(e[3] - a[3]);
  const uint32_t nx = n0 + n1, ny = n2 + n3, cnt = nx + ny, nxa = (nx + IT - 1) & ~(IT - 1);
  if (nxa + ny > TT) {
    if (threadIdx.x == 0) atomicOr(err, 1ull);
    return;
  }
  if (cnt == 0) return;
  {
    using V = typename NativeOf<T>::V;
    const V* srcv = reinterpret_cast<const V*>(src);
    V* sv = reinterpret_cast<V*>(s);
    const uint64_t fb = n0 ? a[0] : n1 ? a[1] : n2 ? a[2] : a[3];  // a record of the tile
    V in[IT];
#pragma unroll
    for (uint32_t k = 0; k < IT; ++k) {
      const uint32_t t = threadIdx.x + k * NT;
      const uint64_t gi = t < n0 ? a[0] + t : t < nx ? a[1] + (t - n0) : t < nx + n2 ? a[2] + (t - nx)
                                                                                      : a[3] + (t - nx - n2);
      BOS_TR(1, 48, t < cnt ? gi : fb);
      in[k] = srcv[t < cnt ? gi : fb];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (uint32_t k = 0; k < IT; ++k) {
      const uint32_t t = threadIdx.x + k * NT;
      if (t < cnt) sv[t] = in[k];
    }
  }
  __syncthreads();
  const uint32_t dd = threadIdx.x * IT;
  T out[IT];
  uint32_t lim = 0;
  if (dd < nx) {
    merge_items_lds<false>(s, 0u, n0, n0, n1, dd, out);
    lim = nx;
  } else if (dd >= nxa && dd - nxa < ny) {
    merge_items_lds<false>(s, nx, n2, nx + n2, n3, dd - nxa, out);
    lim = nxa + ny;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < IT; ++k)
    if (dd + k < lim) s[dd + k + ((dd + k) >> 4)] = out[k];
  __syncthreads();
  if (dd < cnt) merge_items_lds<true>(s, 0u, nx, nxa, ny, dd, out);
  __syncthreads();
  if (dd < cnt) {
#pragma unroll
    for (uint32_t k = 0; k < IT; ++k) s[dd + k + ((dd + k) >> 4)] = out[k];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t k = 0; k < IT; ++k) {
    const uint32_t t = threadIdx.x + k * NT;
    if (t < cnt) {
      const T v = s[t + (t >> 4)];
      const uint64_t o = o0 + t;
      BOS_TR(1, 49, o);
      dst[o] = v;
      if (smp && (o & ((1ull << LG) - 1)) == 0) {
        BOS_TR(1, 41, o >> LG);
        smp[o >> LG] = v;
      }
    }
  }
}

template <int R>
__global__ __launch_bounds__(kM4Threads<R>) void merge4_tile_kernel(const void* src, void* dst, uint64_t n, uint32_t lw,
                                                                const uint64_t* spl, uint64_t ntf, uint64_t ng,
                                                                uint64_t ntl, void* smp, unsigned long long* err) {
  merge4_tile_one<R>(src, dst, n, lw, spl, ntf, ng, ntl, smp, blockIdx.x, err);
}

// Batched four-way passes: one table entry (M4Seg) per instance; launch k
// (0 gather, 1 per-sample ranks, 2 workgroup-wide ranks, 3 tile starts,
// 4 tiles) gives the instance blocks first[k] .. first[k] + count[k] - 1.
__device__ __forceinline__ uint32_t m4_find(const M4Seg* segs, uint32_t nsegs, uint32_t x, uint32_t k) {
  uint32_t lo = 0, hi = nsegs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].first[k] <= x)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <int R>
__global__ void sample_gather_kernel_b(const M4Seg* segs, uint32_t nsegs) {
  const M4Seg& sg = segs[m4_find(segs, nsegs, blockIdx.x, 0)];
  sample_gather_one<R>(sg.src, sg.smp, sg.n, blockIdx.x - sg.first[0]);
}
template <int R>
__global__ void merge4_rank_kernel_b(const M4Seg* segs, uint32_t nsegs) {
  const M4Seg& sg = segs[m4_find(segs, nsegs, blockIdx.x, 1)];
  merge4_rank_one<R>(sg.smp, sg.n, sg.lw, sg.ntf, sg.spl, blockIdx.x - sg.first[1]);
}
template <int R>
__global__ __launch_bounds__(256) void merge4_rank_wide_kernel_b(const M4Seg* segs, uint32_t nsegs) {
  const M4Seg& sg = segs[m4_find(segs, nsegs, blockIdx.x, 2)];
  merge4_rank_wide_one<R>(sg.smp, sg.n, sg.lw, sg.ntf, sg.spl, blockIdx.x - sg.first[2]);
}
template <int R>
__global__ void merge4_bound_kernel_b(const M4Seg* segs, uint32_t nsegs) {
  const M4Seg& sg = segs[m4_find(segs, nsegs, blockIdx.x, 3)];
  merge4_bound_one<R>(sg.src, sg.smp, sg.n, sg.lw, sg.total, sg.spl, blockIdx.x - sg.first[3]);
}
template <int R>
__global__ __launch_bounds__(kM4Threads<R>) void merge4_tile_kernel_b(const M4Seg* segs, uint32_t nsegs) {
  const M4Seg& sg = segs[m4_find(segs, nsegs, blockIdx.x, 4)];
  merge4_tile_one<R>(sg.src, sg.dst, sg.n, sg.lw, sg.spl, sg.ntf, sg.ng, sg.ntl, sg.next_smp,
                     blockIdx.x - sg.first[4], sg.err);
}

// Tiles of a four-way pass over runs of width 2^lw: per full group (ntf), in
// the last group (ntl), the group count (ng) and the total.
struct Merge4Tiles {
  uint64_t ntf, ntl, ng, total;
};
static Merge4Tiles merge4_tiles(int rec, uint64_t n, uint32_t lw) {
  const uint32_t lg = rec == 8 ? kSmpLog<8> : kSmpLog<16>;
  const uint64_t w = 1ull << lw, gw = w << 2, G = 1ull << lg;
  Merge4Tiles t;
  t.ng = (n + gw - 1) / gw;
  t.ntf = ((gw >> lg) + kSplM - 1) / kSplM;
  const uint64_t gl = (t.ng - 1) * gw;
  uint64_t sl = 0;
  for (uint32_t k = 0; k < 4; ++k) {
    const uint64_t st = gl + k * w < n ? gl + k * w : n, len = n - st < w ? n - st : w;
    sl += (len + G - 1) >> lg;
  }
  t.ntl = (sl + kSplM - 1) / kSplM;
  t.total = (t.ng - 1) * t.ntf + t.ntl;
  return t;
}

// Batched status words: segment s gets p[0] = no overflow, p[1..count) = 0.
__global__ void fill_status_kernel_b(const FillSeg* segs, uint32_t nsegs) {
  if (blockIdx.x >= nsegs) return;
  const FillSeg sg = segs[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < sg.count; i += blockDim.x)
    sg.p[i] = i == 0 && !sg.zero_first ? kNoOverflow : 0ull;
}

__global__ void or_u64_kernel(unsigned long long* dst, const unsigned long long* src) {
  if (threadIdx.x == 0) *dst |= *src;
}

// Per-instance outcome of a batch: BOS_ERR_OVERFLOW (2) when its status word
// shows an overflow, else BOS_ERR_INTERNAL (7) when its comparison-sort error
// word is set, else BOS_OK (0); a null pointer skips that check.
__global__ void batch_status_kernel(unsigned long long* const* status, unsigned long long* const* err, uint32_t* out,
                                    uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const bool ovf = status[i] != nullptr && *status[i] != kNoOverflow;
  const bool bad = err != nullptr && err[i] != nullptr && *err[i] != 0ull;
  out[i] = ovf ? 2u : bad ? 7u : 0u;
}

// ---- bitonic baseline ------------------------------------------------------
//
// Batcher's bitonic sort over N = 2^m slots: the n records, then maximal
// records up to N.  Merge phase k2 (blocks of k2 slots, ascending where bit k2
// of the slot index is 0) runs its strides >= ts in register-fused global
// passes and its strides < ts in one tile pass; the phases up to ts run in the
// first tile pass.  A tile pass holds ts = 2^TLOG records in registers, 16 per
// lane in register sub-tiles of 4096 records (the network of the comparison
// sort's tile sort), and sorts or merges them ascending; a tile whose direction
// is descending is stored in reverse.  That is the descending network's output,
// since records are totally ordered and equal records are byte-identical.

// Tile `tile` of src (slots >= n_src read as the maximal record): MERGE = false
// sorts it (the phases up to ts), MERGE = true runs the strides ts/2 .. 1 of
// phase k2 on the bitonic sequence it holds.  Slots below n_dst are stored to
// dst (in place when dst == src: a workgroup reads its whole tile first).
template <int R, uint32_t TLOG, bool MERGE>
__device__ __forceinline__ void bitonic_tile_one(const void* src_, void* dst_, uint64_t n_src, uint64_t n_dst,
                                                 uint64_t k2, uint64_t tile) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t kSub = 4096, kSubPad = kSub + kSub / 16, ts = 1u << TLOG;
  static_assert(TLOG >= 12 && TLOG <= 14, "one, two or four register sub-tiles");
  extern __shared__ __align__(16) unsigned char smem[];
  T* s = reinterpret_cast<T*>(smem);
  const T* S = static_cast<const T*>(src_);
  T* D = static_cast<T*>(dst_);
  const uint32_t tid = threadIdx.x, sub = tid / 256u, lq = tid % 256u;
  const uint64_t tbase = tile << TLOG;
  const uint32_t q0 = sub * kSub;  // the sub-tile's first slot
  LdsR<T> lsub{s + sub * kSubPad};
  ElemR<T> v[16];
  // loads and stores in layout Q of the sub-tile (register e of lane l is its
  // slot 256 e + l: a wave reads and writes 64 consecutive records per
  // instruction); the networks are those of the comparison sort's tile sort
  // (register pairs only, layouts switched through the sub-tile's LDS region)
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    const uint64_t g = tbase + q0 + (e << 8) + lq;
    v[e] = ElemR<T>{MERGE || g < n_src ? S[g] : max_rec<T>()};
  }
  if constexpr (!MERGE) {
    tile_to_lds<2>(v, lsub, lq);
    __syncthreads();
    tile_from_lds<0>(v, lsub, lq);
    tile_phase<1>(v, lsub, lq);
    if constexpr (TLOG >= 13) {
      subtile_cross<T, kSubPad>(v, s, sub, lq, sub ^ 1u, true);
      tile_phase<12>(v, lsub, lq);
    }
    if constexpr (TLOG == 14) {
      subtile_cross<T, kSubPad>(v, s, sub, lq, 3u - sub, true);
      subtile_cross<T, kSubPad>(v, s, sub, lq, sub ^ 1u, false);
      tile_phase<12>(v, lsub, lq);
    }
    __syncthreads();  // every lane's last reads of layout P are done
    tile_to_lds<0>(v, lsub, lq);
    __syncthreads();
    tile_from_lds<2>(v, lsub, lq);
  } else {
    // the cross-sub-tile strides pair the same (lane, register) of two
    // sub-tiles, in any layout; then phase 12 from layout Q: slot bits 11-8
    // in Q, 7-4 in R, 3-0 in P, and back to Q
    if constexpr (TLOG == 14) subtile_cross<T, kSubPad>(v, s, sub, lq, sub ^ 2u, false);
    if constexpr (TLOG >= 13) subtile_cross<T, kSubPad>(v, s, sub, lq, sub ^ 1u, false);
    tile_reg_stages<12, 2, 3>(v, lq);
    tile_to_lds<2>(v, lsub, lq);
    __syncthreads();
    tile_from_lds<1>(v, lsub, lq);
    tile_reg_stages<12, 1, 3>(v, lq);
    tile_to_lds<1>(v, lsub, lq);
    __syncthreads();
    tile_from_lds<0>(v, lsub, lq);
    tile_reg_stages<12, 0, 3>(v, lq);
    __syncthreads();  // every lane's reads of layout R are done
    tile_to_lds<0>(v, lsub, lq);
    __syncthreads();
    tile_from_lds<2>(v, lsub, lq);
  }
  const bool desc = (tbase & k2) != 0;  // descending: slot p goes to ts - 1 - p
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    const uint32_t p = q0 + (e << 8) + lq;
    const uint64_t o = tbase + (desc ? ts - 1u - p : p);
    if (o < n_dst) D[o] = v[e].r;
  }
}

template <int R, uint32_t TLOG, bool MERGE>
__global__ __launch_bounds__(tile_threads<TLOG>()) void bitonic_tile_kernel(const void* src, void* dst,
                                                                           uint64_t n_src, uint64_t n_dst,
                                                                           uint64_t k2) {
  bitonic_tile_one<R, TLOG, MERGE>(src, dst, n_src, n_dst, k2, blockIdx.x);
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

// LDS of the tile sort of 2^TLOG records (padded slots).
template <int R, uint32_t TLOG>
constexpr uint32_t tile_sort_lds() { return ((1u << TLOG) + (1u << TLOG) / 16u) * uint32_t(R); }

// Tile sizes the comparison sort offers for records of `rec` bytes (the LDS
// of a workgroup holds at most 8192 + 512 slots of 16 bytes).
bool sort_tile_ok(int rec, uint32_t t) {
  return t == 1024 || t == 2048 || t == 4096 || t == 8192 || (t == 16384 && rec == 8);
}

template <int R, uint32_t TLOG>
static hipError_t launch_tile_sort_t(void* buf, uint64_t n, hipStream_t s, void* smp) {
  constexpr bool BIG = TLOG > 12;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = BIG ? allow_lds(tile_sort_big_kernel<R, BIG ? TLOG : 13>)
                             : allow_lds(tile_sort_reg_kernel<R, BIG ? 12 : TLOG>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const uint64_t tiles = (n + (1ull << TLOG) - 1) >> TLOG;
  const uint32_t threads = tile_threads<TLOG>(), lds = tile_sort_lds<R, TLOG>();
  if constexpr (BIG)
    hipLaunchKernelGGL((tile_sort_big_kernel<R, TLOG>), dim3(uint32_t(tiles)), dim3(threads), lds, s, buf, n, smp);
  else
    hipLaunchKernelGGL((tile_sort_reg_kernel<R, TLOG>), dim3(uint32_t(tiles)), dim3(threads), lds, s, buf, n, smp);
  return hipGetLastError();
}

// The split region of the comparison sort: two-way merge-path splits, then
// the sample of a four-way pass's input, then its tile starts.
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
static size_t split2_bytes(uint64_t n) {
  constexpr uint64_t t = merge_tile_records(16);  // the smaller merge tile
  return size_t((n + t - 1) / t + 2) * 16;
}
static size_t sample_bytes(int rec, uint64_t n) {
  const uint32_t lg = rec == 8 ? kSmpLog<8> : kSmpLog<16>;
  return size_t((n >> lg) + 2) * uint32_t(rec);
}
static size_t spl4_bytes(int rec, uint64_t n) {
  // tiles of any four-way pass: at most (samples / kSplM) + groups + 1, with
  // groups of at least 4 * kMTile records
  const uint32_t lg = rec == 8 ? kSmpLog<8> : kSmpLog<16>;
  const uint64_t tiles = ((n >> lg) + 1) / kSplM + n / (4ull * merge_tile_records(rec)) + 3;
  return size_t(tiles + 1) * 32;
}

// Four-way passes take every two remaining merge levels once runs are at
// least a merge tile long; the two-way pass takes the rest (runs shorter than
// a tile, and one level when the count left is odd).
static uint32_t levels_left(uint64_t n, uint64_t w) {
  uint32_t c = 0;
  for (; w < n; w <<= 1) ++c;
  return c;
}
static bool four_way_next(int rec, uint64_t n, uint64_t w) {
  const uint32_t l = levels_left(n, w);
  return w >= merge_tile_records(rec) && l >= 2 && l % 2 == 0;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s);
unsigned long long* comparison_sort_err_word(uint64_t* split, uint64_t n, int rec);

template <int R>
static hipError_t comparison_sort_t(void* buf0, void* buf1, uint64_t n, uint32_t ts, uint64_t* split,
                                    hipStream_t s, void** result, bool multiway) {
  BOS_TRACE_BIND();
  static bool attr = false;
  if (!attr) {
    hipError_t e = allow_lds(merge_tile_kernel<R>);
    if (e == hipSuccess) e = allow_lds(merge4_tile_kernel<R>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (!sort_tile_ok(R, ts)) return hipErrorInvalidValue;
  *result = buf0;
  // the error word is cleared on every call, before anything can return
  unsigned long long* err = comparison_sort_err_word(split, n, R);
  {
    const hipError_t e0 = launch_fill_u64(err, 1, 0ull, s);
    if (e0 != hipSuccess) return e0;
  }
  if (n <= 1) return hipSuccess;
  char* region = reinterpret_cast<char*>(split);
  void* smp = region + align256(split2_bytes(n));
  uint64_t* spl = reinterpret_cast<uint64_t*>(region + align256(split2_bytes(n)) + align256(sample_bytes(R, n)));
  // the tile sort writes the first merge pass's samples when that pass is four-way
  bool have_sample = multiway && ts < n && four_way_next(R, n, ts);
  void* tsmp = have_sample ? smp : nullptr;
  prof_begin(BOS_K_SORT_TILE, 0, 2 * n * R, s);
  hipError_t e = hipErrorInvalidValue;
  switch (ts) {
    case 1024: e = launch_tile_sort_t<R, 10>(buf0, n, s, tsmp); break;
    case 2048: e = launch_tile_sort_t<R, 11>(buf0, n, s, tsmp); break;
    case 4096: e = launch_tile_sort_t<R, 12>(buf0, n, s, tsmp); break;
    case 8192: e = launch_tile_sort_t<R, 13>(buf0, n, s, tsmp); break;
    default:
      if constexpr (R == 8) e = launch_tile_sort_t<R, 14>(buf0, n, s, tsmp);
      break;
  }
  prof_end(s);
  if (e != hipSuccess) return e;
  void* src = buf0;
  void* dst = buf1;
  uint32_t pass = 0;
  const uint64_t mtiles = (n + kMTile<R> - 1) / kMTile<R>;
  const uint32_t merge_lds = (kMTile<R> + (kMTile<R> >> 4)) * uint32_t(R);
  for (uint64_t w = ts; w < n;) {
    if (multiway && four_way_next(R, n, w)) {
      uint32_t lw = 0;
      while ((1ull << lw) < w) ++lw;
      const Merge4Tiles t = merge4_tiles(R, n, lw);
      const uint64_t nsmp = (n + (1ull << kSmpLog<R>) - 1) >> kSmpLog<R>;
      const bool next4 = four_way_next(R, n, w << 2);
      prof_begin(BOS_K_SORT_MERGE, pass++, 2 * n * R, s);
      if (!have_sample)
        hipLaunchKernelGGL(sample_gather_kernel<R>, dim3(uint32_t((nsmp + 255) / 256)), dim3(256), 0, s, src, smp, n);
      if ((w >> kSmpLog<R>) >= kSplW<R>) {
        hipLaunchKernelGGL(merge4_rank_wide_kernel<R>, dim3(uint32_t((nsmp + kSplW<R> - 1) / kSplW<R>)), dim3(256), 0,
                           s, smp, n, lw, t.ntf, spl);
      } else {
        const uint64_t rthreads = (nsmp + kSplS<R> - 1) / kSplS<R>;
        hipLaunchKernelGGL(merge4_rank_kernel<R>, dim3(uint32_t((rthreads + 255) / 256)), dim3(256), 0, s, smp, n, lw,
                           t.ntf, spl);
      }
      hipLaunchKernelGGL(merge4_bound_kernel<R>, dim3(uint32_t((t.total + 255) / 256)), dim3(256), 0, s, src, smp, n,
                         lw, t.total, spl);
      hipLaunchKernelGGL(merge4_tile_kernel<R>, dim3(uint32_t(t.total)), dim3(kM4Threads<R>), merge_lds, s, src, dst, n,
                         lw, spl, t.ntf, t.ng, t.ntl, next4 ? smp : nullptr, err);
      prof_end(s);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      have_sample = next4;
      std::swap(src, dst);
      w <<= 2;
      continue;
    }
    have_sample = false;
    prof_begin(BOS_K_SORT_MERGE, pass++, 2 * n * R, s);
    // boundaries 0..mtiles-1 (the end of the last tile is the end of its run pair)
    hipLaunchKernelGGL(merge_partition_kernel<R>, dim3(uint32_t((mtiles + 255) / 256)), dim3(256), 0, s, src, n, w,
                       split, mtiles);
    hipLaunchKernelGGL(merge_tile_kernel<R>, dim3(uint32_t(mtiles)), dim3(kMThreads<R>), merge_lds, s, src, dst, n, w,
                       split);
    prof_end(s);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::swap(src, dst);
    w <<= 1;
  }
  *result = src;
  return hipSuccess;
}

// HBM passes of the comparison sort with four-way passes (multiway) or
// two-way passes only.
uint32_t comparison_sort_hbm_passes(int rec, uint64_t n, uint32_t ts, bool multiway) {
  uint32_t c = 0;
  if (n <= 1) return 0;
  for (uint64_t w = ts; w < n; ++c) w <<= (multiway && four_way_next(rec, n, w)) ? 2 : 1;
  return c;
}

// Bytes of the split region the merge passes need.
size_t comparison_sort_split_bytes(uint64_t n, int rec) {
  return align256(split2_bytes(n)) + align256(sample_bytes(rec, n)) + align256(spl4_bytes(rec, n)) + 256;
}

// The four-way passes' error word: nonzero once a tile failed its bound
// checks (cleared at the start of every comparison sort with four-way passes).
unsigned long long* comparison_sort_err_word(uint64_t* split, uint64_t n, int rec) {
  char* region = reinterpret_cast<char*>(split);
  return reinterpret_cast<unsigned long long*>(region + align256(split2_bytes(n)) + align256(sample_bytes(rec, n)) +
                                               align256(spl4_bytes(rec, n)));
}

// Merge pass p (0-based) of the comparison sort of n records after tiles of
// ts (with four-way passes where they apply): its input run width, whether it
// is four-way, and whether the pass after it is.  False when p is past the
// last pass.
bool merge_pass_at(int rec, uint64_t n, uint32_t ts, uint32_t p, uint64_t* w_out, bool* four, bool* next_four) {
  if (n <= 1) return false;
  uint64_t w = ts;
  for (uint32_t c = 0; w < n; ++c) {
    const bool f = four_way_next(rec, n, w);
    if (c == p) {
      *w_out = w;
      *four = f;
      *next_four = f && four_way_next(rec, n, w << 2);
      return true;
    }
    w <<= f ? 2 : 1;
  }
  return false;
}

// Samples of the first merge pass, when it is four-way (the tile sort writes
// them), else null.
void* first_pass_samples(int rec, uint64_t n, uint32_t ts, uint64_t* split) {
  if (n <= 1 || ts >= n || !four_way_next(rec, n, ts)) return nullptr;
  return reinterpret_cast<char*>(split) + align256(split2_bytes(n));
}

// Table entry of one instance in a batched four-way pass over runs of width w
// whose samples are already written (gather = false: by the tile sort or the
// previous four-way pass) or not; counts[k] = its blocks in launch k.
void merge4_seg(int rec, const void* src, void* dst, uint64_t n, uint64_t* split, uint64_t w, bool gather,
                bool next_four, M4Seg* sg, uint32_t counts[5]) {
  char* region = reinterpret_cast<char*>(split);
  uint32_t lw = 0;
  while ((1ull << lw) < w) ++lw;
  const Merge4Tiles t = merge4_tiles(rec, n, lw);
  const uint32_t lg = rec == 8 ? kSmpLog<8> : kSmpLog<16>;
  const uint64_t nsmp = (n + (1ull << lg) - 1) >> lg;
  const uint32_t sw = rec == 8 ? kSplW<8> : kSplW<16>, ss = rec == 8 ? kSplS<8> : kSplS<16>;
  std::memset(sg, 0, sizeof(*sg));
  sg->src = src;
  sg->dst = dst;
  sg->smp = region + align256(split2_bytes(n));
  sg->next_smp = next_four ? sg->smp : nullptr;
  sg->spl = reinterpret_cast<uint64_t*>(region + align256(split2_bytes(n)) + align256(sample_bytes(rec, n)));
  sg->err = comparison_sort_err_word(split, n, rec);
  sg->n = n;
  sg->ntf = t.ntf;
  sg->ng = t.ng;
  sg->ntl = t.ntl;
  sg->total = t.total;
  sg->lw = lw;
  const bool wide = (w >> lg) >= sw;
  counts[0] = gather ? uint32_t((nsmp + 255) / 256) : 0u;
  counts[1] = wide ? 0u : uint32_t(((nsmp + ss - 1) / ss + 255) / 256);
  counts[2] = wide ? uint32_t((nsmp + sw - 1) / sw) : 0u;
  counts[3] = uint32_t((t.total + 255) / 256);
  counts[4] = uint32_t(t.total);
}

template <int R>
static hipError_t merge4_batched_t(const M4Seg* segs, uint32_t nsegs, const uint32_t totals[5], hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    const hipError_t e = allow_lds(merge4_tile_kernel_b<R>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (nsegs == 0) return hipSuccess;
  if (totals[0]) hipLaunchKernelGGL(sample_gather_kernel_b<R>, dim3(totals[0]), dim3(256), 0, s, segs, nsegs);
  if (totals[1]) hipLaunchKernelGGL(merge4_rank_kernel_b<R>, dim3(totals[1]), dim3(256), 0, s, segs, nsegs);
  if (totals[2]) hipLaunchKernelGGL(merge4_rank_wide_kernel_b<R>, dim3(totals[2]), dim3(256), 0, s, segs, nsegs);
  if (totals[3]) hipLaunchKernelGGL(merge4_bound_kernel_b<R>, dim3(totals[3]), dim3(256), 0, s, segs, nsegs);
  const uint32_t lds = (kMTile<R> + (kMTile<R> >> 4)) * uint32_t(R);
  if (totals[4])
    hipLaunchKernelGGL(merge4_tile_kernel_b<R>, dim3(totals[4]), dim3(kM4Threads<R>), lds, s, segs, nsegs);
  return hipGetLastError();
}

// One batched four-way pass over the instances of segs (totals[k]: blocks of
// launch k summed over them).
hipError_t launch_merge4_batched(int rec, const M4Seg* segs, uint32_t nsegs, const uint32_t totals[5],
                                 hipStream_t s) {
  BOS_TRACE_BIND();
  return rec == 8 ? merge4_batched_t<8>(segs, nsegs, totals, s) : merge4_batched_t<16>(segs, nsegs, totals, s);
}

// multiway: four-way passes where they apply (split must then hold
// comparison_sort_split_bytes(n, rec)); else two-way passes only.
hipError_t launch_comparison_sort(int rec, void* buf0, void* buf1, uint64_t n, uint32_t ts, uint64_t* split,
                                  hipStream_t s, void** result, bool multiway) {
  return rec == 8 ? comparison_sort_t<8>(buf0, buf1, n, ts, split, s, result, multiway)
                  : comparison_sort_t<16>(buf0, buf1, n, ts, split, s, result, multiway);
}

// Tile of the bitonic baseline: 8192 records of 8 bytes or 4096 of 16, 70 KB
// of padded LDS per workgroup (at n = 2^28 x 8 B the sort took 52.6 ms with
// 8192-record tiles, 53.3 with 4096 and 55.9 with 16384).
uint32_t bitonic_tile(int rec) { return rec == 8 ? 8192u : 4096u; }

template <int R>
static hipError_t bitonic_t(const void* in, void* out, uint64_t n, void* ws, uint64_t N, hipStream_t s) {
  constexpr uint32_t TL = R == 8 ? 13u : 12u, ts = 1u << TL;
  static bool attr = false;
  if (!attr) {
    hipError_t e = allow_lds(bitonic_tile_kernel<R, TL, false>);
    if (e == hipSuccess) e = allow_lds(bitonic_tile_kernel<R, TL, true>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (N < ts || (N & (N - 1)) != 0) return hipErrorInvalidValue;
  const uint32_t lds = tile_sort_lds<R, TL>(), threads = tile_threads<TL>(), tiles = uint32_t(N / ts);
  hipError_t e;
  uint32_t gpass = 0, tpass = 0;
  // phases up to ts; a single tile is the whole sort
  prof_begin(BOS_K_BITONIC_TILE, 0, uint64_t(n) * 2 * R, s);
  hipLaunchKernelGGL((bitonic_tile_kernel<R, TL, false>), dim3(tiles), dim3(threads), lds, s, in,
                     N == ts ? out : ws, n, N == ts ? n : N, uint64_t(ts));
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
    // strides below ts; the last phase writes the n smallest slots to out
    const bool last = k2 == N;
    prof_begin(BOS_K_BITONIC_TAIL, tpass++, 2 * N * R, s);
    hipLaunchKernelGGL((bitonic_tile_kernel<R, TL, true>), dim3(tiles), dim3(threads), lds, s, ws,
                       last ? out : ws, N, last ? n : N, k2);
    prof_end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int R, uint32_t TLOG>
static hipError_t batched_tile_sort_t(const SortSeg* segs, uint32_t nsegs, uint32_t total, hipStream_t s) {
  constexpr bool BIG = TLOG > 12;
  static bool attr = false;
  if (!attr) {
    const hipError_t e = BIG ? allow_lds(tile_sort_big_kernel_b<R, BIG ? TLOG : 13>)
                             : allow_lds(tile_sort_reg_kernel_b<R, BIG ? 12 : TLOG>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const uint32_t threads = tile_threads<TLOG>(), lds = tile_sort_lds<R, TLOG>();
  if constexpr (BIG)
    hipLaunchKernelGGL((tile_sort_big_kernel_b<R, TLOG>), dim3(total), dim3(threads), lds, s, segs, nsegs);
  else
    hipLaunchKernelGGL((tile_sort_reg_kernel_b<R, TLOG>), dim3(total), dim3(threads), lds, s, segs, nsegs);
  return hipGetLastError();
}

template <int R>
static hipError_t batched_sort_launch_t(int kind, uint32_t tile, const SortSeg* segs, uint32_t nsegs,
                                        uint32_t total, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    const hipError_t e = allow_lds(merge_tile_kernel_b<R>);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (total == 0) return hipSuccess;
  if (kind == 0) {
    if (!sort_tile_ok(R, tile)) return hipErrorInvalidValue;
    if (tile == 4096) return batched_tile_sort_t<R, 12>(segs, nsegs, total, s);
    if (tile == 2048) return batched_tile_sort_t<R, 11>(segs, nsegs, total, s);
    if (tile == 1024) return batched_tile_sort_t<R, 10>(segs, nsegs, total, s);
    if (tile == 8192) return batched_tile_sort_t<R, 13>(segs, nsegs, total, s);
    if constexpr (R == 8) return batched_tile_sort_t<R, 14>(segs, nsegs, total, s);
    return hipErrorInvalidValue;
  } else if (kind == 1) {
    hipLaunchKernelGGL(merge_partition_kernel_b<R>, dim3((total + 255) / 256), dim3(256), 0, s, segs, nsegs, total);
  } else {
    const uint32_t lds = (kMTile<R> + (kMTile<R> >> 4)) * uint32_t(R);
    hipLaunchKernelGGL(merge_tile_kernel_b<R>, dim3(total), dim3(kMThreads<R>), lds, s, segs, nsegs);
  }
  return hipGetLastError();
}

// Batched comparison-sort launch: kind 0 = tile sort (tiles of `tile`
// records), 1 = merge partition, 2 = merge tiles; `total` = tiles summed over
// the segments.
hipError_t launch_sort_batched(int rec, int kind, uint32_t tile, const SortSeg* segs, uint32_t nsegs,
                               uint32_t total, hipStream_t s) {
  BOS_TRACE_BIND();
  return rec == 8 ? batched_sort_launch_t<8>(kind, tile, segs, nsegs, total, s)
                  : batched_sort_launch_t<16>(kind, tile, segs, nsegs, total, s);
}

hipError_t launch_fill_status_batched(const FillSeg* segs, uint32_t nsegs, hipStream_t s) {
  if (nsegs == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_status_kernel_b, dim3(nsegs), dim3(256), 0, s, segs, nsegs);
  return hipGetLastError();
}

// *dst |= *src, stream-ordered (one thread).
hipError_t launch_or_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s) {
  hipLaunchKernelGGL(or_u64_kernel, dim3(1), dim3(64), 0, s, dst, src);
  return hipGetLastError();
}

hipError_t launch_batch_status(unsigned long long* const* status, unsigned long long* const* err, uint32_t* out,
                               uint32_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_status_kernel, dim3((count + 255) / 256), dim3(256), 0, s, status, err, out, count);
  return hipGetLastError();
}

hipError_t launch_bitonic(int rec, const void* in, void* out, uint64_t n, void* ws, uint64_t N,
                          hipStream_t s) {
  return rec == 8 ? bitonic_t<8>(in, out, n, ws, N, s) : bitonic_t<16>(in, out, n, ws, N, s);
}

}  // namespace bos
