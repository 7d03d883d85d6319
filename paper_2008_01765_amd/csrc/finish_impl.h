// finish_impl.h — per-bin finish of the bucket ORP (Section 3.2) after the
// split form of the last routing pass: each final bin's reals are put in a
// uniformly random order and written, dummies stripped, to the bin's place in
// the output.
//
// The split last pass leaves bin gb's reals compacted in slots gb*Z ..
// gb*Z + loads[gb] - 1 of the binned array (in the order the network left
// them) and every routing block's real count, which a two-level scan turns
// into block offsets.  This kernel then, per bin:
//   1. sorts the bin's Z slots in record order (key, payload), dummies last,
//      so that the permutation below does not depend on the order in which
//      the butterfly delivered the reals, and leaves the sorted bin in LDS;
//   2. gives the p-th real the 64-bit key r(gb*Z + p): word (g mod 4) of the
//      Philox4x64-10 block g/4 under key (seed, 1) and counter (g/4, attempt);
//   3. orders the bin by (r, p), dummies last (a uniformly random order of
//      the reals: random labels followed by a sort, the construction of
//      Section 4.1).  The network sorts one 64-bit word per slot, the top
//      64 - log2 Z bits of r with p below them, which is the (r, p) order
//      while no two reals share their top key bits; the keys depend on
//      (seed, attempt, bin, p) only, and when two of a bin's reals (or its
//      last real and first dummy) do share them, a flag that depends on no
//      data sends the whole finish through a second launch that sorts
//      (r, record) pairs, the (r, p) order since p follows the records;
//   4. writes output slot j of the bin, j < load, from the LDS copy of the
//      record of rank p(j) to out[offset of the bin + j].
// Both sorts are bitonic networks over all Z slots and the ranks p(j) are a
// function of the keys, so every address but the final writes (which depend
// on the loads, revealed by the method) is a function of (Z, seed, attempt,
// bin) only.
//
// Layout: lane lq of the bin's Z/16 lanes holds slots 16 lq + e (e = 0..15) in
// registers, each record as the 64-bit word(s) that order it (key in the high
// half for 8-byte records).  Stages on slot bits 0..3 pair registers; stages on higher bits
// pair lanes lq ^ X through DPP (X = 1, 2), ds_swizzle (X = 4, 8, 16) or a
// lane permute (X = 32).  Up to Z = 1024 a bin's lanes are one wave's and the
// only LDS is the bin's record copy of step 4 (the routing kernel's padded
// bin layout); Z = 2048 (two waves per bin) sorts through LDS with that
// layout.
#pragma once
#include "route_impl.h"

namespace bos {

constexpr uint32_t kFinishThreads = 256;

namespace finish_detail {

template <uint32_t X>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  if constexpr (X == 1) return dpp<kDppXor1>(v);
  else if constexpr (X == 2) return dpp<kDppXor2>(v);
  else if constexpr (X < 32) return swz_xor<X>(v);
  else return uint32_t(__shfl_xor(int(v), int(X), 64));
}
template <uint32_t X>
__device__ __forceinline__ uint2 lane_xor(uint2 v) {
  return make_uint2(lane_xor<X>(v.x), lane_xor<X>(v.y));
}
template <uint32_t X>
__device__ __forceinline__ uint4 lane_xor(uint4 v) {
  return make_uint4(lane_xor<X>(v.x), lane_xor<X>(v.y), lane_xor<X>(v.z), lane_xor<X>(v.w));
}
template <uint32_t X, typename T>
__device__ __forceinline__ ElemR<T> e_xor(const ElemR<T>& a) {
  return ElemR<T>{lane_xor<X>(a.r)};
}
template <uint32_t X, typename T>
__device__ __forceinline__ ElemRK<T> e_xor(const ElemRK<T>& a) {
  return ElemRK<T>{lane_xor<X>(a.r), lane_xor<X>(a.klo), lane_xor<X>(a.khi), lane_xor<X>(a.aux)};
}

// Comparators of the networks below: CMP 0 = e_less of the element type
// (record order, or the packed key words of the fast launch), 2 = (random
// key, record).
template <int CMP, typename E>
__device__ __forceinline__ bool lt(const E& a, const E& b) {
  if constexpr (CMP == 0) return e_less(a, b);
  else return (a.key < b.key) | ((a.key == b.key) & f_less(a.r, b.r));
}

// Compare-exchange of two registers (x gets the smaller when ascending) and
// with the element of lane lq ^ X (the lower lane keeps the smaller when
// ascending).  Elements equal under the comparator are byte-identical.
template <int CMP, typename E>
__device__ __forceinline__ void cx_r(E& x, E& y, bool asc) {
  const bool sw = lt<CMP>(y, x) == asc;
  const E nx = e_sel(sw, y, x), ny = e_sel(sw, x, y);
  x = nx;
  y = ny;
}
template <int CMP, uint32_t X, typename E>
__device__ __forceinline__ void cx_xor(E& x, bool is_lo, bool asc) {
  const E p = e_xor<X>(x);
  const bool take = lt<CMP>(p, x) == (is_lo == asc);
  x = e_sel(take, p, x);
}

// Phase KK (merges of 2^KK slots), stages JJ = KK-1 .. 0, on layout P held
// entirely in registers and lane exchanges (LZ <= 10).
template <int LZ, int KK, int JJ, int CMP, typename E>
__device__ __forceinline__ void reg_stages(E (&v)[16], uint32_t lq) {
  if constexpr (JJ >= 0) {
    if constexpr (JJ < 4) {
      constexpr uint32_t hb = 1u << JJ;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        if (e & hb) continue;
        bool asc;
        if constexpr (KK == LZ) asc = true;
        else if constexpr (KK < 4) asc = ((e >> KK) & 1u) == 0u;
        else asc = ((lq >> (KK - 4)) & 1u) == 0u;
        cx_r<CMP>(v[e], v[e | hb], asc);
      }
    } else {
      constexpr uint32_t X = 1u << (JJ - 4);
      const bool is_lo = (lq & X) == 0u;
      bool asc;
      if constexpr (KK == LZ) asc = true;
      else asc = ((lq >> (KK - 4)) & 1u) == 0u;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) cx_xor<CMP, X>(v[e], is_lo, asc);
    }
    reg_stages<LZ, KK, JJ - 1, CMP>(v, lq);
  }
}
template <int LZ, int KK, int CMP, typename E>
__device__ __forceinline__ void reg_phases(E (&v)[16], uint32_t lq) {
  if constexpr (KK <= LZ) {
    reg_stages<LZ, KK, KK - 1, CMP>(v, lq);
    reg_phases<LZ, KK + 1, CMP>(v, lq);
  }
}

}  // namespace finish_detail

// Dynamic LDS bytes of the finish kernel: up to Z = 1024 the fast launch
// stages each bin's records (in record order) for the final gather and the
// exact launch uses none; Z = 2048 sorts through LDS.
__host__ __device__ inline uint32_t finish_lds_bytes(int rec, uint32_t lz, bool exact) {
  const uint32_t z = 1u << lz, zp = z + (z >> 4), bpw = kFinishThreads / (z >> 4);
  if (lz < 11) return exact ? 0u : bpw * zp * uint32_t(rec);
  return (bpw * zp * (uint32_t(rec) + 10u) + 15u) & ~15u;
}

namespace finish_detail {

// A record as the words that order it: one 64-bit word (key << 32 | payload)
// for 8-byte records, (key, payload) for 16-byte ones.
template <int R> struct FRec;
template <> struct FRec<8> {
  uint64_t k;
};
template <> struct FRec<16> {
  uint64_t k, p;
};
__device__ __forceinline__ bool f_less(const FRec<8>& a, const FRec<8>& b) { return a.k < b.k; }
__device__ __forceinline__ bool f_less(const FRec<16>& a, const FRec<16>& b) {
  return (a.k < b.k) | ((a.k == b.k) & (a.p < b.p));
}
__device__ __forceinline__ bool f_eq(const FRec<8>& a, const FRec<8>& b) { return a.k == b.k; }
__device__ __forceinline__ bool f_eq(const FRec<16>& a, const FRec<16>& b) { return (a.k == b.k) & (a.p == b.p); }
__device__ __forceinline__ FRec<8> f_sel(bool c, const FRec<8>& a, const FRec<8>& b) { return {c ? a.k : b.k}; }
__device__ __forceinline__ FRec<16> f_sel(bool c, const FRec<16>& a, const FRec<16>& b) {
  return {c ? a.k : b.k, c ? a.p : b.p};
}
template <uint32_t X>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v) {
  return uint64_t(lane_xor<X>(uint32_t(v))) | (uint64_t(lane_xor<X>(uint32_t(v >> 32))) << 32);
}
template <uint32_t X>
__device__ __forceinline__ FRec<8> f_xor(const FRec<8>& a) { return {lane_xor64<X>(a.k)}; }
template <uint32_t X>
__device__ __forceinline__ FRec<16> f_xor(const FRec<16>& a) { return {lane_xor64<X>(a.k), lane_xor64<X>(a.p)}; }
__device__ __forceinline__ FRec<8> f_load(const uint2& r) { return {(uint64_t(r.x) << 32) | r.y}; }
__device__ __forceinline__ FRec<16> f_load(const uint4& r) {
  return {uint64_t(r.x) | (uint64_t(r.y) << 32), uint64_t(r.z) | (uint64_t(r.w) << 32)};
}
__device__ __forceinline__ uint2 f_store(const FRec<8>& f) { return make_uint2(uint32_t(f.k >> 32), uint32_t(f.k)); }
__device__ __forceinline__ uint4 f_store(const FRec<16>& f) {
  return make_uint4(uint32_t(f.k), uint32_t(f.k >> 32), uint32_t(f.p), uint32_t(f.p >> 32));
}
template <int R> __device__ __forceinline__ FRec<R> f_max();
template <> __device__ __forceinline__ FRec<8> f_max<8>() { return {~0ull}; }
template <> __device__ __forceinline__ FRec<16> f_max<16>() { return {~0ull, ~0ull}; }

// Sort elements of the two per-bin sorts.
template <int R>
struct FE1 {  // record order
  FRec<R> r;
};
template <int R>
struct FE2 {  // random-key order: key r (then the record, for ties)
  uint64_t key;
  FRec<R> r;
};
template <int R>
__device__ __forceinline__ bool e_less(const FE1<R>& a, const FE1<R>& b) { return f_less(a.r, b.r); }
template <int R>
__device__ __forceinline__ FE1<R> e_sel(bool c, const FE1<R>& a, const FE1<R>& b) { return {f_sel(c, a.r, b.r)}; }
template <int R>
__device__ __forceinline__ FE2<R> e_sel(bool c, const FE2<R>& a, const FE2<R>& b) {
  return {c ? a.key : b.key, f_sel(c, a.r, b.r)};
}
template <uint32_t X, int R>
__device__ __forceinline__ FE1<R> e_xor(const FE1<R>& a) { return {f_xor<X>(a.r)}; }
template <uint32_t X, int R>
__device__ __forceinline__ FE2<R> e_xor(const FE2<R>& a) { return {lane_xor64<X>(a.key), f_xor<X>(a.r)}; }

// Key-order element of the fast launch: the top 64 - LZ bits of the key with
// the record rank p in the low LZ bits (dummies all ones).  While no two of a
// bin's reals share their top key bits this orders the reals as (key, p).
struct FE3 {
  uint64_t w;
};
__device__ __forceinline__ bool e_less(const FE3& a, const FE3& b) { return a.w < b.w; }
__device__ __forceinline__ FE3 e_sel(bool c, const FE3& a, const FE3& b) { return {c ? a.w : b.w}; }
template <uint32_t X>
__device__ __forceinline__ FE3 e_xor(const FE3& a) { return {lane_xor64<X>(a.w)}; }

// True when this lane holds two adjacent slots p, p+1 <= load (reals and the
// first dummy) whose words agree in their key bits; the pair across the lane
// boundary is checked by the lower lane.
template <int LZ, uint32_t HL>
__device__ __forceinline__ bool word_tie(const FE3 (&w)[16], uint32_t lq, uint32_t load) {
  bool tie = false;
#pragma unroll
  for (uint32_t e = 0; e + 1 < 16; ++e) {
    const uint32_t p = 16u * lq + e;
    tie |= (p < load) & ((w[e].w >> LZ) == (w[e + 1].w >> LZ));
  }
  if constexpr (HL > 1) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t src = (lane + 1u) & 63u;
    const uint32_t lo = uint32_t(__shfl(int(uint32_t(w[0].w)), int(src), 64));
    const uint32_t hi = uint32_t(__shfl(int(uint32_t(w[0].w >> 32)), int(src), 64));
    const uint64_t nw = (uint64_t(hi) << 32) | lo;
    const uint32_t p = 16u * lq + 15u;
    tie |= (lq + 1u < HL) & (p < load) & ((w[15].w >> LZ) == (nw >> LZ));
  }
  return tie;
}

// Record sort of a bin of 2^LZ slots (LZ = 8..10, the bin's 2^(LZ-4) lanes in
// one wave) with every compare-exchange on two registers of one lane: three
// layouts put one group of slot-index bits in the register index, P = bits
// 0-3 (lane = bits 4 .. LZ-1), R = bits 4-7 (lane = bits 0-3 and 8 .. LZ-1)
// and Q = bits LZ-4 .. LZ-1 (lane = bits 0 .. LZ-5); a phase whose stages
// reach bits above 3 moves the bin through its LDS slots (padded s + s/16)
// into those layouts and back, in place of lane exchanges.  Addresses depend
// on (lane, register) only.
template <int LZ, int G>
__device__ __forceinline__ uint32_t bslot(uint32_t l, uint32_t e) {
  if constexpr (G == 0) return (l << 4) | e;
  else if constexpr (G == 1) return ((l >> 4) << 8) | (e << 4) | (l & 15u);
  else return (e << (LZ - 4)) | l;
}
template <int LZ, int KK, int G, int JB, typename E>
__device__ __forceinline__ void lay_stages(E (&v)[16], uint32_t l) {
  if constexpr (JB >= 0) {
    constexpr uint32_t hb = 1u << JB;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (e & hb) continue;
      const bool asc = KK == LZ || ((bslot<LZ, G>(l, e) >> KK) & 1u) == 0u;
      cx_r<0>(v[e], v[e | hb], asc);
    }
    lay_stages<LZ, KK, G, JB - 1>(v, l);
  }
}
// Padded LDS slot of register e in layout G, bslot + bslot/16, written as a
// lane base plus e times a constant (immediate offsets, no per-register
// address registers): P 17 l + e, R 272 (l/16) + l mod 16 + 17 e, Q l + l/16
// + e (2^(LZ-4) + 2^(LZ-8)).
template <int LZ, int G>
__device__ __forceinline__ uint32_t pad_base(uint32_t l) {
  if constexpr (G == 0) return 17u * l;
  else if constexpr (G == 1) return 272u * (l >> 4) + (l & 15u);
  else return l + (l >> 4);
}
template <int LZ, int G>
constexpr uint32_t pad_step() {
  return G == 0 ? 1u : G == 1 ? 17u : (1u << (LZ - 4)) + (1u << (LZ - 8));
}
// (the bin's LDS slots hold the ordering words themselves while the network
// runs: no conversion to the record layout between layouts)
template <int LZ, int G, int R>
__device__ __forceinline__ void lay_st(const FE1<R> (&v)[16], FRec<R>* sb, uint32_t l, uint32_t trb) {
  constexpr uint32_t st = pad_step<LZ, G>();
  const uint32_t pb = pad_base<LZ, G>(l);
  FRec<R>* b = sb + pb;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    BOS_TR(0, 4, trb + pb + e * st);
    b[e * st] = v[e].r;
  }
}
template <int LZ, int G, int R>
__device__ __forceinline__ void lay_ld(FE1<R> (&v)[16], const FRec<R>* sb, uint32_t l, uint32_t trb) {
  constexpr uint32_t st = pad_step<LZ, G>();
  const uint32_t pb = pad_base<LZ, G>(l);
  const FRec<R>* b = sb + pb;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    BOS_TR(0, 4, trb + pb + e * st);
    v[e] = FE1<R>{b[e * st]};
  }
}
// Phases KK .. LZ; v holds layout P on entry and exit.
template <int LZ, int KK, int R>
__device__ __forceinline__ void lay_phases(FE1<R> (&v)[16], FRec<R>* sb, uint32_t l, uint32_t trb) {
  if constexpr (KK <= LZ) {
    if constexpr (KK >= 5) {
      lay_st<LZ, 0>(v, sb, l, trb);
      lds_wave_sync();
      if constexpr (KK >= 9) {
        lay_ld<LZ, 2>(v, sb, l, trb);
        lay_stages<LZ, KK, 2, KK - 1 - (LZ - 4)>(v, l);  // slot bits KK-1 .. LZ-4
        lay_st<LZ, 2>(v, sb, l, trb);
        lds_wave_sync();
      }
      lay_ld<LZ, 1>(v, sb, l, trb);
      lay_stages<LZ, KK, 1, (KK >= 9 ? LZ - 9 : KK - 5)>(v, l);  // slot bits min(KK-1, LZ-5) .. 4
      lay_st<LZ, 1>(v, sb, l, trb);
      lds_wave_sync();
      lay_ld<LZ, 0>(v, sb, l, trb);
    }
    lay_stages<LZ, KK, 0, (KK >= 4 ? 3 : KK - 1)>(v, l);  // slot bits min(KK-1, 3) .. 0
    lay_phases<LZ, KK + 1>(v, sb, l, trb);
  }
}

}  // namespace finish_detail

// EXACT = false: the key sort compares the random keys alone and raises
// *a.tie when a bin holds two equal keys among its reals (and its first
// dummy).  EXACT = true runs after it: it returns at once unless *a.tie is
// set, and then redoes every bin with the (key, record) comparator.  The
// flag depends on the keys only, never on the data.
template <int R, int LZ, bool EXACT>
__global__ __launch_bounds__(kFinishThreads) __attribute__((amdgpu_waves_per_eu(R == 8 ? (EXACT ? 3 : 4) : 2))) void orp_finish_kernel(FinishArgs a) {
  using namespace finish_detail;
  using T = typename RecOf<R>::T;
  constexpr uint32_t Z = 1u << LZ, HL = Z >> 4, BPW = kFinishThreads / HL, ZP = Z + (Z >> 4);
  static_assert(LZ >= 4 && LZ <= 11, "Z in [16, 2048]");
  const uint32_t tid = threadIdx.x, S = tid / HL, lq = tid % HL;
  const T* binned = static_cast<const T*>(a.binned);
  T* out = static_cast<T*>(a.out);
  extern __shared__ __align__(16) unsigned char smem[];
  if constexpr (EXACT) {
    if (__hip_atomic_load(a.tie, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0ull) return;
  }
  const uint64_t gend = a.gb_hi ? a.gb_hi : a.nbins;  // bins [gb_lo, gend)
  for (uint64_t g0 = a.gb_lo + uint64_t(blockIdx.x) * BPW; g0 < gend; g0 += uint64_t(gridDim.x) * BPW) {
    const uint64_t gb = g0 + S;
    const bool act = gb < gend;
    uint32_t load = 0;
    uint64_t off = 0;
    if (act) {
      // output offset: the routing block's offset plus the loads of the
      // block's earlier bins
      BOS_TR(0, 22, gb);
      load = a.loads[gb];
      const uint64_t blk = gb >> a.klev;
      BOS_TR(0, 23, blk);
      BOS_TR(0, 23, blk >> 10);
      off = a.boff[blk] + a.coff[blk >> 10];
      for (uint64_t j = blk << a.klev; j < gb; ++j) {
        BOS_TR(0, 22, j);
        off += a.loads[j];
      }
    }
    // slot index of the staged copy (global index minus bin_slot0)
    const uint64_t src = (gb << LZ) + 16u * lq - a.bin_slot0;
    if constexpr (LZ <= 10) {
      // 1. record order, dummies (maximal record) last
      FE1<R> v[16];
      if constexpr (!EXACT && LZ >= 8) {
        // the bin's reals read in layout Q (the bin's lanes take consecutive
        // slots), moved to layout P through the bin's LDS slots, then the
        // layout-switching network
        FRec<R>* sb = reinterpret_cast<FRec<R>*>(smem) + S * ZP;
        static_assert(sizeof(FRec<R>) == sizeof(T), "a slot holds a record or its ordering words");
        const uint64_t b0 = (gb << LZ) - a.bin_slot0;
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t p = bslot<LZ, 2>(lq, e);
          if (act && p < load) BOS_TR(0, 20, b0 + p);
          v[e] = FE1<R>{(act && p < load) ? f_load(binned[b0 + p]) : f_max<R>()};
        }
        lay_st<LZ, 2>(v, sb, lq, S * ZP);
        lds_wave_sync();
        lay_ld<LZ, 0>(v, sb, lq, S * ZP);
        lay_phases<LZ, 1>(v, sb, lq, S * ZP);
      } else {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t p = 16u * lq + e;
          if (act && p < load) BOS_TR(0, 20, src + e);
          v[e] = FE1<R>{(act && p < load) ? f_load(binned[src + e]) : f_max<R>()};
        }
        reg_phases<LZ, 1, 0>(v, lq);
      }
      if constexpr (!EXACT) {
        // the bin in record order to LDS (rank p at padded slot p + p/16;
        // the bin's lanes are one wave's)
        T* sbin = reinterpret_cast<T*>(smem) + S * ZP;
        if (act) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            BOS_TR(0, 4, S * ZP + 17u * lq + e);
            sbin[17u * lq + e] = f_store(v[e].r);
          }
        }
        // 2. rank p's key r(gb*Z + p), its top bits with p below them
        FE3 w[16];
#pragma unroll
        for (uint32_t e4 = 0; e4 < 4; ++e4) {
          const uint32_t p0 = 16u * lq + 4u * e4;
          const Philox4 ph = philox4x64_10(((gb << LZ) + p0) >> 2, a.attempt, a.seed, 1);
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t e = 4u * e4 + q;
            w[e] = FE3{p0 + q < load ? ((ph.v[q] >> LZ) << LZ) | (p0 + q) : ~0ull};
          }
        }
        // 3. order by the words (their ranks then follow the keys)
        reg_phases<LZ, 1, 0>(w, lq);
        lds_wave_sync();
        // 4. output slot j of the bin takes the record of rank w[j] mod Z
        if (act) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            const uint32_t j = 16u * lq + e;
            if (j < load && off + j < a.n) {
              const uint32_t p = uint32_t(w[e].w) & (Z - 1u);
              BOS_TR(0, 4, S * ZP + p + (p >> 4));
              BOS_TR(0, 21, off + j);
              out[off + j - a.out0] = sbin[p + (p >> 4)];
            }
          }
        }
        // two reals with the same top key bits: the exact launch redoes it
        if (act && word_tie<LZ, HL>(w, lq, load)) {
          BOS_TR(0, 24, 0);
          atomicOr(a.tie, 1ull);
        }
      } else {
        // exact launch: 2. the per-bin keys of the reals (reals hold slots
        // 0 .. load-1) with their records
        FE2<R> w[16];
#pragma unroll
        for (uint32_t e4 = 0; e4 < 4; ++e4) {
          const uint32_t p0 = 16u * lq + 4u * e4;
          const Philox4 ph = philox4x64_10(((gb << LZ) + p0) >> 2, a.attempt, a.seed, 1);
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q) {
            const uint32_t e = 4u * e4 + q;
            w[e] = FE2<R>{p0 + q < load ? ph.v[q] : ~0ull, v[e].r};
          }
        }
        // 3. order by (key, record), which is (key, p) as the reals are in
        //    record order
        reg_phases<LZ, 1, 2>(w, lq);
        // 4. the reals to their place in the output
        if (act) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            const uint32_t p = 16u * lq + e;
            if (p < load && off + p < a.n) {
              BOS_TR(0, 21, off + p);
              out[off + p - a.out0] = f_store(w[e].r);
            }
          }
        }
      }
    } else if constexpr (!EXACT) {
      // Z = 2048: two waves per bin, networks through LDS (padded bins), with
      // the (key, rank) comparator
      ElemR<T> v[16];
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint32_t p = 16u * lq + e;
        if (act && p < load) BOS_TR(0, 20, src + e);
        v[e] = ElemR<T>{(act && p < load) ? binned[src + e] : max_rec<T>()};
      }
      T* srec = reinterpret_cast<T*>(smem);
      bin_bitonic<LZ>(v, LdsR<T>{srec}, S * ZP, lq, act);
      ElemRK<T> w[16];
#pragma unroll
      for (uint32_t e4 = 0; e4 < 4; ++e4) {
        const uint32_t p0 = 16u * lq + 4u * e4;
        const Philox4 ph = philox4x64_10(((gb << LZ) + p0) >> 2, a.attempt, a.seed, 1);
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          const uint32_t e = 4u * e4 + q;
          const bool real = p0 + q < load;
          w[e] = ElemRK<T>{v[e].r, real ? uint32_t(ph.v[q]) : ~0u, real ? uint32_t(ph.v[q] >> 32) : ~0u,
                           real ? p0 + q : 0xFFFFu};
        }
      }
      lds_barrier();  // the record sort's last LDS reads are done
      const uint32_t mp = BPW * ZP;
      uint32_t* sklo = reinterpret_cast<uint32_t*>(smem + size_t(mp) * R);
      uint32_t* skhi = sklo + mp;
      uint16_t* saux = reinterpret_cast<uint16_t*>(skhi + mp);
      bin_bitonic<LZ>(w, LdsRK<T>{srec, sklo, skhi, saux}, S * ZP, lq, act);
      if (act) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t p = 16u * lq + e;
          if (p < load && off + p < a.n) {
            BOS_TR(0, 21, off + p);
            out[off + p - a.out0] = w[e].r;
          }
        }
      }
      lds_barrier();  // LDS of this group is no longer read
    }
  }
}

}  // namespace bos
