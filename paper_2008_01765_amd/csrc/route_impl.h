// route_impl.h — register-resident routing passes of bucket ORP
// (Algorithm 3.1 of Asharov et al., SOSA 2020) for gfx950.
//
// Same method and same results as orp_pass_kernel (orp_kernels.hip): one
// launch runs `klev` fused butterfly levels over blocks of 2^klev buckets, every
// MergeSplit a tight-compaction network over the 2Z slots of its two buckets
// (marks = reals whose next label bit is 0 plus the first Z - x dummies, the
// dummy tagging of Section 4.1; network = the offset-compaction recursion of
// Sasy, Johnson and Goldberg, CCS 2022).  This version is specialised on
// log2 Z so that every stage is unrolled with compile-time register pairs:
//
//   * A MergeSplit's 2Z slots live in the registers of 2Z/16 lanes, 16 slots
//     per lane.  In layout A lane l holds positions q = 16 l + e (e = 0..15):
//     stages over q bits 0..3 pair registers, stages over q bits 4 and 5 pair
//     lanes l and l^1 / l^2 through DPP quad permutes.  In layout B a lane holds
//     the 16 positions whose q bits LQ-4..LQ-1 vary (LQ = log2 2Z), so the
//     remaining stages pair registers again.  Each level therefore moves the
//     data through LDS twice: A -> B, and B -> next level's A (whose MergeSplits
//     pair other buckets).
//   * Blocks are persistent: a workgroup walks over several blocks of buckets,
//     and several workgroups share a CU (three at 2^3 Z = 4096 slots of 8-byte
//     records), so one workgroup's HBM loads overlap the others' networks.
//     Barriers wait for LDS traffic only.
//
// Obliviousness: every HBM and LDS address is a function of (n, Z, klev,
// level, block, lane, register) only; labels and records steer register
// selects, never an address.
#pragma once
#include "bos_common.h"

namespace bos {

namespace route_detail {

constexpr uint32_t kDppXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr uint32_t kDppXor2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr uint32_t kDppB0022 = 0xA0; // quad_perm [0,0,2,2]
constexpr uint32_t kDppB1133 = 0xF5; // quad_perm [1,1,3,3]
constexpr uint32_t kDppB0000 = 0x00; // quad_perm [0,0,0,0]
constexpr uint32_t kDppB2222 = 0xAA; // quad_perm [2,2,2,2]

// Barrier that waits for this wave's LDS operations only (global loads issued
// earlier remain in flight).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
}

// Orders this wave's LDS writes before its later LDS reads.  Enough when the
// lanes that exchange data through LDS all belong to one wave: LDS executes a
// wave's instructions in order.
__device__ __forceinline__ void lds_wave_sync() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// LDS exchange among `LANES` consecutive lanes (a power of two): a wave-local
// wait when they fit in one wave, a workgroup barrier otherwise.
template <uint32_t LANES>
__device__ __forceinline__ void lds_group_sync() {
  if constexpr (LANES <= 64u) lds_wave_sync();
  else lds_barrier();
}

template <uint32_t CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return uint32_t(__builtin_amdgcn_mov_dpp(int(v), CTRL, 0xF, 0xF, false));
}
template <uint32_t CTRL>
__device__ __forceinline__ uint2 dpp(uint2 v) {
  return make_uint2(dpp<CTRL>(v.x), dpp<CTRL>(v.y));
}
template <uint32_t CTRL>
__device__ __forceinline__ uint4 dpp(uint4 v) {
  return make_uint4(dpp<CTRL>(v.x), dpp<CTRL>(v.y), dpp<CTRL>(v.z), dpp<CTRL>(v.w));
}

__device__ __forceinline__ uint32_t brev_k(uint32_t x, uint32_t k) { return k ? (__brev(x) >> (32u - k)) : 0u; }

// Halves of a record for two-half LDS exchanges (8 bytes of a 16-byte
// record, 4 of an 8-byte one).
__device__ __forceinline__ uint2 rec_lo(uint4 v) { return make_uint2(v.x, v.y); }
__device__ __forceinline__ uint2 rec_hi(uint4 v) { return make_uint2(v.z, v.w); }
__device__ __forceinline__ void set_lo(uint4& v, uint2 l) {
  v.x = l.x;
  v.y = l.y;
}
__device__ __forceinline__ void set_hi(uint4& v, uint2 h) {
  v.z = h.x;
  v.w = h.y;
}
__device__ __forceinline__ uint32_t rec_lo(uint2 v) { return v.x; }
__device__ __forceinline__ uint32_t rec_hi(uint2 v) { return v.y; }
__device__ __forceinline__ void set_lo(uint2& v, uint32_t l) { v.x = l; }
__device__ __forceinline__ void set_hi(uint2& v, uint32_t h) { v.y = h; }
template <typename T> struct HalfOf;
template <> struct HalfOf<uint4> {
  using H = uint2;
  static __device__ __forceinline__ H zero() { return make_uint2(0u, 0u); }
};
template <> struct HalfOf<uint2> {
  using H = uint32_t;
  static __device__ __forceinline__ H zero() { return 0u; }
};

// Swap decision of the compaction network for the pair at offset i of a node
// of 2*half slots whose marks prefix is P0 at its start and Ph at its middle.
__device__ __forceinline__ bool swap_bit(uint32_t P0, uint32_t Ph, uint32_t half, uint32_t i) {
  if (half == 1u) return (Ph - P0) == (P0 & 1u);  // the rule below with half = 1
  const uint32_t z = P0 & (2u * half - 1u), mm = Ph - P0;
  const bool s = (((z & (half - 1u)) + mm) >= half) != (z >= half);
  const uint32_t t = (z + mm) & (half - 1u);
  return s != (i >= t);
}

// DPP source with lanes outside the pattern (or rows outside ROW_MASK)
// reading 0.
template <uint32_t CTRL, uint32_t ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROW_MASK, 0xF, true));
}

// Inclusive scan over aligned groups of W lanes (W a power of two <= 64):
// row_shr steps inside rows of 16 lanes, then row broadcasts across rows.
template <uint32_t W>
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, uint32_t lane) {
  constexpr uint32_t kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  if constexpr (W >= 2) {
    const uint32_t y = dpp_or_zero<kRowShr + 1>(x);
    x += (W >= 16 || (lane & (W - 1u)) >= 1u) ? y : 0u;
  }
  if constexpr (W >= 4) {
    const uint32_t y = dpp_or_zero<kRowShr + 2>(x);
    x += (W >= 16 || (lane & (W - 1u)) >= 2u) ? y : 0u;
  }
  if constexpr (W >= 8) {
    const uint32_t y = dpp_or_zero<kRowShr + 4>(x);
    x += (W >= 16 || (lane & (W - 1u)) >= 4u) ? y : 0u;
  }
  if constexpr (W >= 16) x += dpp_or_zero<kRowShr + 8>(x);
  if constexpr (W >= 32) x += dpp_or_zero<kRowBcast15, 0xA>(x);  // row 0 -> row 1, row 2 -> row 3
  if constexpr (W >= 64) x += dpp_or_zero<kRowBcast31, 0xC>(x);  // lane 31 -> rows 2 and 3
  return x;
}

// Exclusive scan over aligned segments of SEG lanes (SEG a power of two).
template <uint32_t SEG>
__device__ __forceinline__ uint32_t seg_scan(uint32_t v, uint32_t* swave, uint32_t* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  constexpr uint32_t W = SEG < 64u ? SEG : 64u;
  const uint32_t x = wave_incl_scan<W>(v, lane);
  if constexpr (SEG <= 64u) {
    if constexpr (W == 64u)
      *total = uint32_t(__builtin_amdgcn_readlane(int(x), 63));
    else
      *total = __shfl(x, int(lane | (W - 1u)), 64);
    return x - v;
  } else {
    if (lane == 63u) {
      BOS_TR(0, 9, wave);
      swave[wave] = x;
    }
    lds_barrier();
    constexpr uint32_t WPS = SEG / 64u;
    const uint32_t w0 = wave & ~(WPS - 1u);
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (uint32_t q = 0; q < WPS; ++q) {
      BOS_TR(0, 9, w0 + q);
      const uint32_t t = swave[w0 + q];
      if (w0 + q < wave) pre += t;
      tot += t;
    }
    *total = tot;
    return pre + x - v;
  }
}

}  // namespace route_detail
using namespace route_detail;

// ---- per-bin finish of the last pass (Section 3.2) ---------------------------
//
// Each final bin (Z slots in LDS, padded by one slot per 16) is sorted by a
// bitonic network held in registers: lane lq of the bin's Z/16 lanes holds
// slots 16 lq + e (layout P; stages on slot bits 0..3 pair registers, bits 4
// and 5 pair lanes through DPP).  Stages on slot bits >= 6 run in layout Q,
// where a lane holds the 16 slots whose top four bits vary.  Sort keys:
// record order with dummies last (bos_sort, and the first half of the
// random permutation of bos_orp), then (r, p) with dummies last, r the 64-bit
// Philox key of the p-th real in record order (bos_orp).

// Sort elements.  Dummies are given the maximal record (record order) or the
// maximal key (random-key order), so that comparing keys alone puts them
// last; a real element can only tie with a dummy when both are byte-identical,
// where either order gives the same output bytes.
template <typename T>
struct ElemR {  // a record
  T r;
};
template <typename T>
struct ElemRK {  // a record with its 64-bit random key and rank p (0xFFFF for dummies)
  T r;
  uint32_t klo, khi, aux;
};

template <typename T>
__device__ __forceinline__ bool e_less(const ElemR<T>& a, const ElemR<T>& b) {
  return rec_less(a.r, b.r);
}
template <typename T>
__device__ __forceinline__ bool e_less(const ElemRK<T>& a, const ElemRK<T>& b) {
  const uint64_t ka = (uint64_t(a.khi) << 32) | a.klo, kb = (uint64_t(b.khi) << 32) | b.klo;
  return ka < kb || (ka == kb && a.aux < b.aux);
}
template <typename T>
__device__ __forceinline__ ElemR<T> e_sel(bool c, const ElemR<T>& a, const ElemR<T>& b) {
  return ElemR<T>{sel(c, a.r, b.r)};
}
template <typename T>
__device__ __forceinline__ ElemRK<T> e_sel(bool c, const ElemRK<T>& a, const ElemRK<T>& b) {
  return ElemRK<T>{sel(c, a.r, b.r), c ? a.klo : b.klo, c ? a.khi : b.khi, c ? a.aux : b.aux};
}
template <uint32_t CTRL, typename T>
__device__ __forceinline__ ElemR<T> e_dpp(const ElemR<T>& a) {
  return ElemR<T>{dpp<CTRL>(a.r)};
}
template <uint32_t CTRL, typename T>
__device__ __forceinline__ ElemRK<T> e_dpp(const ElemRK<T>& a) {
  return ElemRK<T>{dpp<CTRL>(a.r), dpp<CTRL>(a.klo), dpp<CTRL>(a.khi), dpp<CTRL>(a.aux)};
}

// LDS views of the bins (padded slot index)
// (tw: the trace buffer its accesses fold into in the digest build: 0 for
// the routing and the per-bin finish, 1 for the comparison sort)
template <typename T>
struct LdsR {
  T* rec;
  uint32_t tw = 0;
  __device__ ElemR<T> ld(uint32_t i) const {
    BOS_TR(tw, 4, i);
    return ElemR<T>{rec[i]};
  }
  __device__ void st(uint32_t i, const ElemR<T>& v) const {
    BOS_TR(tw, 4, i);
    rec[i] = v.r;
  }
};
template <typename T>
struct LdsRK {
  T* rec;
  uint32_t* klo;
  uint32_t* khi;
  uint16_t* aux;
  uint32_t tw = 0;
  __device__ ElemRK<T> ld(uint32_t i) const {
    BOS_TR(tw, 17, i);
    return ElemRK<T>{rec[i], klo[i], khi[i], aux[i]};
  }
  __device__ void st(uint32_t i, const ElemRK<T>& v) const {
    BOS_TR(tw, 17, i);
    rec[i] = v.r;
    klo[i] = v.klo;
    khi[i] = v.khi;
    aux[i] = uint16_t(v.aux);
  }
};

// Compare-exchange with one comparison: equal elements are byte-identical, so
// swapping them or not is the same.
template <typename E>
__device__ __forceinline__ void cx_reg(E& x, E& y, bool asc) {
  const bool sw = e_less(y, x) == asc;
  const E nx = e_sel(sw, y, x), ny = e_sel(sw, x, y);
  x = nx;
  y = ny;
}
template <uint32_t CTRL, typename E>
__device__ __forceinline__ void cx_lane(E& x, bool is_lo, bool asc) {
  const E p = e_dpp<CTRL>(x);
  const bool take = e_less(p, x) == (is_lo == asc);
  x = e_sel(take, p, x);
}

// Bitonic sort (ascending) of every bin; v holds layout P on entry and exit.
// bbase: padded LDS offset of this lane's bin; lq: lane within the bin.
// Phases KK = 1..LZ (merges of 2^KK slots), stages JJ = KK-1..0 (slot bit JJ);
// all indices are template parameters so every register index is static.
struct BinLane {
  uint32_t bbase, pbase, lq, lb0, lb1, lowQ;
  bool active;  // lanes past the block's bins hold no bin and touch no LDS
};

template <int LZ, int KK>
__device__ __forceinline__ bool asc_p(uint32_t e, const BinLane& bl) {
  if constexpr (KK == LZ) return true;
  else if constexpr (KK < 4) return ((e >> KK) & 1u) == 0u;
  else return ((bl.lq >> (KK - 4)) & 1u) == 0u;
}
template <int LZ, int KK>
__device__ __forceinline__ bool asc_q(uint32_t e, const BinLane& bl) {
  if constexpr (KK == LZ) return true;
  else if constexpr (KK >= LZ - 4) return ((e >> (KK - (LZ - 4))) & 1u) == 0u;
  else if constexpr (KK == LZ - 5) return bl.lb1 == 0u;  // lane bits of layout Q (Z >= 2048)
  else return bl.lb0 == 0u;
}

template <int LZ, int KK, int JJ, typename E>
__device__ __forceinline__ void p_stages(E (&v)[16], const BinLane& bl) {
  if constexpr (JJ >= 0) {
    if constexpr (JJ < 4) {
      constexpr uint32_t hb = 1u << JJ;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        if (e & hb) continue;
        cx_reg(v[e], v[e | hb], asc_p<LZ, KK>(e, bl));
      }
    } else if constexpr (JJ == 4) {
      const bool asc = asc_p<LZ, KK>(0, bl);
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) cx_lane<kDppXor1>(v[e], bl.lb0 == 0u, asc);
    } else {
      const bool asc = asc_p<LZ, KK>(0, bl);
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) cx_lane<kDppXor2>(v[e], bl.lb1 == 0u, asc);
    }
    p_stages<LZ, KK, JJ - 1>(v, bl);
  }
}

template <int LZ, int KK, int JJ, typename E>
__device__ __forceinline__ void q_stages(E (&v)[16], const BinLane& bl) {
  if constexpr (JJ >= 6) {
    if constexpr (JJ >= LZ - 4) {
      constexpr uint32_t hb = 1u << (JJ - (LZ - 4));
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        if (e & hb) continue;
        cx_reg(v[e], v[e | hb], asc_q<LZ, KK>(e, bl));
      }
    } else if constexpr (JJ == LZ - 5) {  // lane bit 1 of layout Q (2^LZ >= 2048)
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) cx_lane<kDppXor2>(v[e], bl.lb1 == 0u, asc_q<LZ, KK>(e, bl));
    } else {  // lane bit 0 of layout Q (2^LZ = 4096)
      static_assert(JJ == LZ - 6, "layout Q covers slot bits >= LZ-6");
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) cx_lane<kDppXor1>(v[e], bl.lb0 == 0u, asc_q<LZ, KK>(e, bl));
    }
    q_stages<LZ, KK, JJ - 1>(v, bl);
  }
}

template <int LZ, int KK, typename E, typename V>
__device__ __forceinline__ void bitonic_phase(E (&v)[16], const V& lds, const BinLane& bl) {
  if constexpr (KK <= LZ) {
    if constexpr (KK - 1 >= 6) {
      // layout Q for the stages on slot bits KK-1 .. 6
      if (bl.active) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) lds.st(bl.pbase + e, v[e]);
      }
      lds_group_sync<(1u << LZ) / 16u>();  // a bin's lanes
      if (bl.active) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t sl = (e << (LZ - 4)) | bl.lowQ;
          v[e] = lds.ld(bl.bbase + sl + (sl >> 4));
        }
      }
      q_stages<LZ, KK, KK - 1>(v, bl);
      if (bl.active) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t sl = (e << (LZ - 4)) | bl.lowQ;
          lds.st(bl.bbase + sl + (sl >> 4), v[e]);
        }
      }
      lds_group_sync<(1u << LZ) / 16u>();
      if (bl.active) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) v[e] = lds.ld(bl.pbase + e);
      }
    }
    p_stages<LZ, KK, (KK - 1 < 5 ? KK - 1 : 5)>(v, bl);
    bitonic_phase<LZ, KK + 1>(v, lds, bl);
  }
}

// Ascending bitonic merge of every bin (phase LZ only: stages LZ-1 .. 0), for
// bins that hold a bitonic sequence; v holds layout P on entry and exit.
template <int LZ, typename E, typename V>
__device__ __forceinline__ void bin_bitonic_merge(E (&v)[16], const V& lds, uint32_t bbase, uint32_t lq, bool active) {
  BinLane bl;
  bl.active = active;
  bl.bbase = bbase;
  bl.pbase = bbase + 17u * lq;
  bl.lq = lq;
  bl.lb0 = lq & 1u;
  bl.lb1 = (lq >> 1) & 1u;
  const uint32_t rest = lq >> 2;
  bl.lowQ = LZ >= 11 ? ((bl.lb1 << (LZ - 5)) | (bl.lb0 << (LZ - 6)) | rest) : (LZ >= 6 ? lq : 0u);
  bitonic_phase<LZ, LZ>(v, lds, bl);
}

template <int LZ, typename E, typename V>
__device__ __forceinline__ void bin_bitonic(E (&v)[16], const V& lds, uint32_t bbase, uint32_t lq, bool active) {
  BinLane bl;
  bl.active = active;
  bl.bbase = bbase;
  bl.pbase = bbase + 17u * lq;  // layout P: slots 16 lq .. 16 lq + 15
  bl.lq = lq;
  bl.lb0 = lq & 1u;
  bl.lb1 = (lq >> 1) & 1u;
  const uint32_t rest = lq >> 2;
  // layout Q pairs lanes through DPP only for Z = 2048; otherwise lanes take
  // consecutive slots
  bl.lowQ = LZ >= 11 ? ((bl.lb1 << (LZ - 5)) | (bl.lb0 << (LZ - 6)) | rest) : (LZ >= 6 ? lq : 0u);
  bitonic_phase<LZ, 1>(v, lds, bl);
}

// Per-bin finish of the last pass (Section 3.2): every final bin (LDS bucket
// S, padded slots) is sorted in record order with its dummies (maximal
// record) last, and for fin == 0 then permuted uniformly: the p-th real of
// global bin gb gets the key r(gb*Z + p), word (g mod 4) of Philox block g/4
// with key (seed, 1), and the bin is sorted by (key, p).  On return outr holds
// this lane's 16 slots of its bin (slots 16 lq .. 16 lq + 15) and `load` the
// bin's real count; reals occupy the bin's first `load` slots.  FIN: 0 =
// choose by a.fin at run time, 1 = sort only, 2 = sort and permute.  FULL:
// every lane of the workgroup holds slots (no lane guards).
template <int R, int LZ, int FIN, bool FULL>
__device__ __forceinline__ void sort_bins(const PassArgs& a, uint64_t blk, uint32_t klev,
                                          typename RecOf<R>::T* srec, uint32_t* stag, uint32_t* srhi,
                                          uint16_t* saux, const uint32_t* sload, typename RecOf<R>::T (&outr)[16],
                                          uint32_t* load_out) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t Z = 1u << LZ, ZP = Z + (Z >> 4), HL = Z >> 4;
  const uint32_t tid = threadIdx.x, NB = 1u << klev, m = Z << klev;
  const bool active = FULL || tid < (m >> 4);
  const uint32_t S = active ? tid / HL : 0u, lq = active ? tid % HL : 0u;
  const uint32_t bbase = S * ZP;
  // record order, dummies (maximal record) last
  const LdsR<T> lr{srec};
  ElemR<T> v[16];
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    const uint32_t i = bbase + 17u * lq + e;
    if (active) {
      BOS_TR(0, 5, i);
      BOS_TR(0, 4, i);
    }
    v[e] = ElemR<T>{(active && stag[i] != kDummyTag) ? srec[i] : max_rec<T>()};
  }
  bin_bitonic<LZ>(v, lr, bbase, lq, active);
  if (active) BOS_TR(0, 7, S);
  const uint32_t load = active ? sload[S] : 0u;
  *load_out = load;
  const bool permute = FIN == 2 || (FIN == 0 && a.fin == 0);
  if (FIN != 1 && permute) {
    const uint64_t gb = blk * NB + brev_k(S, klev);
    ElemRK<T> w[16];
#pragma unroll
    for (uint32_t e4 = 0; e4 < 4; ++e4) {
      const uint32_t p0 = 16u * lq + 4u * e4;
      const Philox4 ph = philox4x64_10((gb * Z + p0) >> 2, a.attempt, a.seed, 1);
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t e = 4u * e4 + q;
        const bool real = p0 + q < load;  // reals occupy the first `load` slots
        w[e] = ElemRK<T>{v[e].r, real ? uint32_t(ph.v[q]) : ~0u, real ? uint32_t(ph.v[q] >> 32) : ~0u,
                         real ? p0 + q : 0xFFFFu};
      }
    }
    lds_barrier();  // the record sort's last LDS reads are done
    const LdsRK<T> lrk{srec, stag, srhi, saux};
    bin_bitonic<LZ>(w, lrk, bbase, lq, active);
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) outr[e] = w[e].r;
  } else {
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) outr[e] = v[e].r;
  }
}

// Value of lane (lane ^ X) within each group of 32 lanes (ds_swizzle in bit
// mode: and-mask 31, or-mask 0, xor-mask X; no LDS memory is touched).
template <uint32_t X>
__device__ __forceinline__ uint32_t swz_xor(uint32_t v) {
  static_assert(X >= 1 && X < 32, "xor-mask of 5 bits");
  return uint32_t(__builtin_amdgcn_ds_swizzle(int(v), int((X << 10) | 0x1F)));
}
template <uint32_t X>
__device__ __forceinline__ uint2 swz_xor(uint2 v) {
  return make_uint2(swz_xor<X>(v.x), swz_xor<X>(v.y));
}
template <uint32_t X>
__device__ __forceinline__ uint4 swz_xor(uint4 v) {
  return make_uint4(swz_xor<X>(v.x), swz_xor<X>(v.y), swz_xor<X>(v.z), swz_xor<X>(v.w));
}

// One compaction stage at distance 16 HLX (< 512 slots): the partner slot is
// held by lane lq ^ HLX, reached by a swizzle; P0 and Ph are the reals'
// prefix counts at the node's start and middle (the bin's lane prefixes).
template <uint32_t HLX, typename T>
__device__ __forceinline__ void compact_xstage(T (&rv)[16], uint32_t (&tv)[16], const uint32_t* bpfx, uint32_t lq,
                                               bool active) {
  constexpr uint32_t half = HLX * 16u;
  const uint32_t node0 = lq & ~(2u * HLX - 1u);
  if (active) {
    BOS_TR(0, 6, node0);
    BOS_TR(0, 6, node0 + HLX);
  }
  const uint32_t P0 = active ? bpfx[node0] : 0u, Ph = active ? bpfx[node0 + HLX] : 0u;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    const uint32_t i = 16u * (lq & (HLX - 1u)) + e;  // index in the node's half
    const bool b = active && swap_bit(P0, Ph, half, i);
    const T pr = swz_xor<HLX>(rv[e]);
    const uint32_t pt = swz_xor<HLX>(tv[e]);
    rv[e] = sel(b, pr, rv[e]);
    tv[e] = b ? pt : tv[e];
  }
}

// Oblivious compaction of every final bin in LDS: the bin's reals move to
// its first slots.  The last level leaves each bin's reals interleaved with
// dummies; this is the tight compaction network a MergeSplit level runs
// (conditional swaps at distances 1, 2, .., Z/2, each decided by swap_bit from
// the prefix counts of the reals), over one bin of Z slots with the reals as
// the marks.  Lane lq of the bin's Z/16 lanes holds slots 16 lq + e; stages at
// distances below 16 pair registers, those up to 256 pair lanes by swizzles,
// and longer ones exchange through the bin's own LDS slots.  On return rv
// holds this lane's 16 slots after the compaction.
// LOAD: read the bin's slots from LDS first; else rv and tv already hold
// them (layout P).
template <int R, int LZ, bool FULL, bool LOAD>
__device__ __forceinline__ void compact_bin(typename RecOf<R>::T* srec, uint32_t* stag, uint32_t* spfx,
                                            uint32_t* swave, uint32_t klev, typename RecOf<R>::T (&rv)[16],
                                            uint32_t (&tv)[16]) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t Z = 1u << LZ, ZP = Z + (Z >> 4), HL = Z >> 4;
  const uint32_t tid = threadIdx.x, m = Z << klev;
  const bool active = FULL || tid < (m >> 4);
  const uint32_t S = active ? tid / HL : 0u, lq = active ? tid % HL : 0u;
  const uint32_t bbase = S * ZP;
  if constexpr (LOAD) {
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (active) {
        BOS_TR(0, 4, bbase + 17u * lq + e);
        BOS_TR(0, 5, bbase + 17u * lq + e);
      }
      rv[e] = active ? srec[bbase + 17u * lq + e] : zero_rec<T>();
      tv[e] = active ? stag[bbase + 17u * lq + e] : kDummyTag;
    }
  }
  // prefix counts of the reals
  uint32_t pm[16];
  uint32_t run = 0;
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) {
    pm[e] = run;
    run += tv[e] != kDummyTag ? 1u : 0u;
  }
  uint32_t tot;
  const uint32_t excl = seg_scan<HL>(active ? run : 0u, swave, &tot);
#pragma unroll
  for (uint32_t e = 0; e < 16; ++e) pm[e] += excl;
  if (active) {
    BOS_TR(0, 6, S * HL + lq);
    spfx[S * HL + lq] = pm[0];
  }
  // distances 1, 2, 4, 8: register pairs
#pragma unroll
  for (uint32_t eb = 0; eb < 4; ++eb) {
    const uint32_t half = 1u << eb;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (e & half) continue;
      const uint32_t e2 = e | half, es = e & ~(2u * half - 1u);
      const bool b = swap_bit(pm[es], pm[es | half], half, e & (half - 1u));
      const T r1 = rv[e], r2 = rv[e2];
      const uint32_t t1 = tv[e], t2 = tv[e2];
      rv[e] = sel(b, r2, r1);
      rv[e2] = sel(b, r1, r2);
      tv[e] = b ? t2 : t1;
      tv[e2] = b ? t1 : t2;
    }
  }
  // distances 16 .. 256: the partner lane is lq ^ (half / 16), within 32 lanes
  lds_group_sync<HL>();  // every lane's prefix is in spfx
  const uint32_t* bpfx = spfx + S * HL;
  if constexpr (HL >= 2) compact_xstage<1>(rv, tv, bpfx, lq, active);
  if constexpr (HL >= 4) compact_xstage<2>(rv, tv, bpfx, lq, active);
  if constexpr (HL >= 8) compact_xstage<4>(rv, tv, bpfx, lq, active);
  if constexpr (HL >= 16) compact_xstage<8>(rv, tv, bpfx, lq, active);
  if constexpr (HL >= 32) compact_xstage<16>(rv, tv, bpfx, lq, active);
  // distances 512 .. Z/2 (Z >= 1024): through the bin's LDS slots
  for (uint32_t half = 512; half < Z; half <<= 1) {
    lds_group_sync<HL>();  // spfx written; the previous stage's reads are done
    if (active) {
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        BOS_TR(0, 4, bbase + 17u * lq + e);
        BOS_TR(0, 5, bbase + 17u * lq + e);
        srec[bbase + 17u * lq + e] = rv[e];
        stag[bbase + 17u * lq + e] = tv[e];
      }
    }
    lds_group_sync<HL>();
    const uint32_t hl = half >> 4;                   // lanes per half node
    const uint32_t node0 = lq & ~(2u * hl - 1u);     // first lane of this lane's node
    const uint32_t plq = lq ^ hl;
    if (active) {
      BOS_TR(0, 6, S * HL + node0);
      BOS_TR(0, 6, S * HL + node0 + hl);
    }
    const uint32_t P0 = active ? spfx[S * HL + node0] : 0u, Ph = active ? spfx[S * HL + node0 + hl] : 0u;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint32_t i = 16u * (lq & (hl - 1u)) + e;  // index in the node's half
      const bool b = active && swap_bit(P0, Ph, half, i);
      const uint32_t pi = bbase + 17u * plq + e;
      if (active) {
        BOS_TR(0, 4, pi);
        BOS_TR(0, 5, pi);
      }
      const T pr = active ? srec[pi] : zero_rec<T>();
      const uint32_t pt = active ? stag[pi] : kDummyTag;
      rv[e] = sel(b, pr, rv[e]);
      tv[e] = b ? pt : tv[e];
    }
  }
}

// Last pass, split form: after the per-bin finish, global bin gb keeps its
// reals in slots gb*Z .. gb*Z + load - 1 of rec_out, its real count in
// loads[gb] and the block's total in scan[blk]; a scan and a strip kernel then
// concatenate the bins (the addresses of both depend on the loads only, which
// the method reveals).  FIN = 3: the bins are compacted, not sorted (their
// reals keep the order the last level left).
// LOADED (FIN = 3): rv and tv already hold every bin's slots (layout P:
// lane lq of bin S holds slots 16 lq .. 16 lq + 15); else they are read from
// LDS.  rv and tv are scratch registers of the caller.
template <int R, int LZ, int FIN, bool FULL, bool LOADED>
__device__ __forceinline__ void finish_split(const PassArgs& a, uint32_t blk, uint32_t klev,
                                             typename RecOf<R>::T* srec, uint32_t* stag, uint32_t* srhi,
                                             uint16_t* saux, const uint32_t* sload, uint32_t* spfx,
                                             uint32_t* swave, typename RecOf<R>::T (&rv)[16],
                                             uint32_t (&tv)[16]) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t Z = 1u << LZ, HL = Z >> 4;
  const uint32_t tid = threadIdx.x, NB = 1u << klev, m = Z << klev;
  const bool active = FULL || tid < (m >> 4);
  const uint32_t S = active ? tid / HL : 0u, lq = active ? tid % HL : 0u;
  if (tid == 0) {
    uint64_t agg = 0;
    for (uint32_t b = 0; b < NB; ++b) {
      BOS_TR(0, 7, b);
      agg += sload[b] < Z ? sload[b] : Z;
    }
    BOS_TR(0, 14, blk);
    a.scan[blk] = agg;
  }
  T (&outr)[16] = rv;
  uint32_t load = 0;
  if constexpr (FIN == 3) {
    compact_bin<R, LZ, FULL, !LOADED>(srec, stag, spfx, swave, klev, outr, tv);
    if (active) BOS_TR(0, 7, S);
    load = active ? sload[S] : 0u;
  } else {
    static_assert(!LOADED, "the per-bin sorts read their bins from LDS");
    sort_bins<R, LZ, FIN, FULL>(a, blk, klev, srec, stag, srhi, saux, sload, outr, &load);
  }
  if (active) {
    // a bin holds at most Z reals (an overflowing attempt is discarded)
    const uint32_t kept = load < Z ? load : Z;
    const uint64_t gb = uint64_t(blk) * NB + brev_k(S, klev);
    T* BO = static_cast<T*>(a.rec_out);
    if (lq == 0) {
      BOS_TR(0, 13, gb);
      a.loads[gb] = kept;
    }
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint32_t p = 16u * lq + e;
      if (p < kept) {
        BOS_TR(0, 12, (gb << LZ) + p);
        BO[(gb << LZ) + p - a.out_slot0] = outr[e];
      }
    }
  }
}

// Last pass, fused form: sort (or randomly permute) every bin, then strip the
// dummies and write the bins' reals to their place in the output, found with
// a decoupled look-back over the blocks (block index = ticket order).
template <int R, int LZ, bool FULL>
__device__ __forceinline__ void finish_bins(const PassArgs& a, uint32_t blk, uint32_t klev,
                                            typename RecOf<R>::T* srec, uint32_t* stag, uint32_t* srhi,
                                            uint16_t* saux, uint32_t* sload, uint32_t* soff) {
  using T = typename RecOf<R>::T;
  constexpr uint32_t Z = 1u << LZ, HL = Z >> 4;
  const uint32_t tid = threadIdx.x, NB = 1u << klev, m = Z << klev;
  const bool active = FULL || tid < (m >> 4);
  const uint32_t S = active ? tid / HL : 0u, lq = active ? tid % HL : 0u;
  // The bin loads (sload, written by the last level) are known before the
  // bins are sorted: publish the block's aggregate now so that later blocks'
  // look-back does not wait for this block's sort.
  uint64_t agg = 0;
  if (tid == 0) {
    for (uint32_t b = 0; b < NB; ++b) {
      BOS_TR(0, 7, b);
      agg += sload[b];
    }
    BOS_TR(0, 14, blk);
    __hip_atomic_store(&a.scan[blk], ((blk == 0 ? 2ull : 1ull) << 62) | agg, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  T outr[16];
  uint32_t load = 0;
  sort_bins<R, LZ, 0, FULL>(a, blk, klev, srec, stag, srhi, saux, sload, outr, &load);
  // look back for the block's output offset (reals occupy the first slots of
  // every sorted bin).  Wave 0 inspects 64 predecessors per step: it sums
  // their aggregates back to the nearest one whose inclusive prefix is known.
  if (tid < 64) {
    const uint32_t lane = tid;
    const uint64_t kVal = (1ull << 62) - 1ull;
    uint64_t excl = 0;
    int64_t p = int64_t(blk) - 1;
    while (p >= 0) {
      const int64_t idx = p - int64_t(lane);
      const unsigned long long w =
          idx >= 0 ? __hip_atomic_load(&a.scan[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) : (2ull << 62);
      const uint32_t flag = uint32_t(w >> 62);
      const unsigned long long inc = __ballot(flag == 2u), none = __ballot(flag == 0u);
      const uint32_t first2 = inc ? uint32_t(__ffsll((long long)inc) - 1) : 64u;
      const unsigned long long need = first2 < 63u ? ((2ull << first2) - 1ull) : ~0ull;
      if (none & need) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      uint64_t v = lane <= first2 ? (w & kVal) : 0ull;
#pragma unroll
      for (uint32_t o = 32; o > 0; o >>= 1) v += __shfl_xor(v, int(o), 64);
      excl += v;
      if (first2 < 64u) break;
      p -= 64;
    }
    if (lane == 0) {
      if (blk != 0)
        __hip_atomic_store(&a.scan[blk], (2ull << 62) | (excl + agg), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t off = excl;
      for (uint32_t u = 0; u < NB; ++u) {
        const uint32_t b = brev_k(u, klev);
        BOS_TR(0, 8, b);
        BOS_TR(0, 7, b);
        soff[2 * b] = uint32_t(off);
        soff[2 * b + 1] = uint32_t(off >> 32);
        off += sload[b];
      }
    }
  }
  lds_barrier();
  if (active) {
    T* OUT = static_cast<T*>(a.out);
    BOS_TR(0, 8, S);
    const uint64_t off = (uint64_t(soff[2 * S + 1]) << 32) | soff[2 * S];
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint32_t p = 16u * lq + e;
      if (p < load && off + p < a.n) {
        BOS_TR(0, 16, off + p);
        OUT[off + p] = outr[e];
      }
    }
  }
}

// R: record bytes; LZ: log2 Z (4..11); MODE bit 0 = first pass, bit 1 = last,
// bit 2 = split form of the last pass (bins compacted and written to rec_out,
// then scan + strip; the sorts only), bit 4 = the launch has exactly Z 2^klev / 16 lanes
// (all of them hold slots, so no lane needs a guard), bit 5 = a first pass whose
// groups all start on a multiple of 8 elements (no staged loads).
// Body of one routing launch.  BATCH = false: a persistent workgroup walks
// over items blockIdx.x, + gridDim.x, ... (last pass: tickets).  BATCH = true:
// the workgroup runs the single item `item0` of one instance of a batch.
template <int R, int LZ, int MODE, bool BATCH>
__device__ __forceinline__ void route_run(const PassArgs& a, uint32_t nitems, uint32_t item0) {
  using T = typename RecOf<R>::T;
  constexpr bool FIRST = (MODE & 1) != 0, LAST = (MODE & 2) != 0, SPLIT = (MODE & 4) != 0;
  constexpr bool FULL = (MODE & 16) != 0;  // every lane holds slots: no lane guards
  // a first pass whose groups all start on a multiple of 8 elements: built
  // without the staged loads (and their registers)
  constexpr bool ALIGNED = (MODE & 32) != 0;
  static_assert(!ALIGNED || (FIRST && !LAST), "the aligned form is a first pass that is not also the last");
  static_assert(!SPLIT || (LAST && !FIRST), "the split form is a last pass that is not also the first");
  // the split form serves the sorts: it compacts its bins, and the strip puts
  // in order the bins that straddle a tile of the comparison sort's first
  // phase (the tile sort orders every other bin with its tile); bos_orp's
  // permuting finish keeps the fused form
  constexpr int SPLIT_FIN = 3;
  constexpr uint32_t Z = 1u << LZ, LQ = LZ + 1, TPM = 1u << (LQ - 4), ZP = Z + (Z >> 4);
  constexpr bool HAS_B = LQ > 6;
  constexpr uint32_t HALF_LANES = TPM / 2;  // lanes per bucket in layout A

  // Records exchange through LDS in two halves (the tags go with the
  // first): LDS holds half a record and a tag per slot, so more workgroups
  // share a CU.
  constexpr bool HALF = lds_rec_bytes(R, Z, LAST && !SPLIT) < uint32_t(R);
  static_assert(!HALF || HAS_B, "two-half exchanges use layout B (Z >= 64)");
  using H = typename HalfOf<T>::H;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t klev = a.klev, NB = 1u << klev, m = Z << klev, mp = NB * ZP;
  T* srec = reinterpret_cast<T*>(smem);
  H* shalf = reinterpret_cast<H*>(smem);  // HALF: one half record per slot
  uint32_t* stag = reinterpret_cast<uint32_t*>(smem + size_t(mp) * lds_rec_bytes(R, Z, LAST && !SPLIT));
  uint32_t* spfx = stag + mp;          // m/16 marks-prefix entries (16-slot granularity)
  uint32_t* sload = spfx + (m >> 4);   // NB bin loads (last pass)
  uint32_t* soff = sload + NB;         // 2*NB words: output offsets (last pass)
  uint32_t* swave = soff + 2 * NB;     // 64 scan words
  uint32_t* smisc = swave + 64;        // 16 words
  uint32_t* srhi = smisc + 16;         // last pass, shuffle
  uint16_t* saux = reinterpret_cast<uint16_t*>(srhi + mp);

  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint64_t n = a.n, B = a.buckets;
  const uint32_t L = a.levels, i0 = a.level0;
  const bool active = FULL || tid < (m >> 4);
  const uint32_t ms = active ? tid / TPM : 0u, lt = active ? tid % TPM : 0u;
  const T* RI = static_cast<const T*>(a.rec_in);
  const T* X = static_cast<const T*>(a.x_in);
  // first pass: all groups start on a multiple of 8 elements (labels come from
  // whole Philox blocks); otherwise inputs are staged through LDS
  // (B = 2^L: divisions by B are shifts; a 64-bit division by a run-time
  // value would be a long software sequence in every lane)
  const bool aligned = ALIGNED || (n & ((8ull << L) - 1ull)) == 0;

  // ---- load one block into layout-A registers of level 0 -------------------
  // level 0 pairs LDS buckets 2ms and 2ms+1; lane lt holds slots 16*(lt mod
  // TPM/2) .. +15 of bucket 2ms + lt / (TPM/2).
  const uint32_t S_load = 2u * ms + (lt >= HALF_LANES ? 1u : 0u);
  const uint32_t sb_load = 16u * (lt % HALF_LANES);
  T rv[16];
  uint32_t tv[16];

  auto issue_load = [&](uint32_t item, T* dr, uint32_t* dt) {
    const uint64_t r = uint64_t(item) & ((1ull << i0) - 1ull), h = uint64_t(item) >> i0;
    if constexpr (!FIRST) {
      const uint64_t bucket = (h << (i0 + klev)) + (uint64_t(S_load) << i0) + r;
      const uint64_t gi = (bucket << LZ) + sb_load;
      // staged chunk: input segment S_load holds buckets (S_load, r in0 ..)
      const uint64_t si = a.staged ? ((((h - a.in_h0) << (i0 + klev)) + (uint64_t(S_load) << a.in_lseg) +
                                       (r - a.in_r0)) << LZ) + sb_load
                                   : gi;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        if (active) {
          BOS_TR(0, 1, gi + e);
          BOS_TR(0, 2, gi + e);
        }
        dr[e] = active ? RI[si + e] : zero_rec<T>();
        dt[e] = active ? a.tag_in[si + e] : kDummyTag;
      }
    } else {
      // group j = h*NB + S_load holds X[floor(jn/B), floor((j+1)n/B))
      const uint64_t j = h * NB + S_load;
      const uint64_t gs = (j * n) >> L, gz = (((j + 1) * n) >> L) - gs;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const bool real = active && (sb_load + e) < gz;
        if (real) BOS_TR(0, 3, gs + sb_load + e);
        dr[e] = real ? X[gs + sb_load + e - a.x_off] : zero_rec<T>();
        dt[e] = real ? 0u : kDummyTag;  // label filled in by finish_load
      }
    }
  };
  // first pass: labels of the loaded reals (word x mod 8 of Philox block x/8)
  auto finish_load = [&](uint32_t item, uint32_t* dt) {
    constexpr uint32_t QH = HALF_LANES / 2;  // lanes of a bucket that can hold reals
    if constexpr (FIRST && QH >= 1 && QH < 64) {
      // A group has at most Z/2 elements, so its reals sit in the first QH
      // lanes of the bucket (16 slots each, two Philox blocks).  Every lane
      // computes one block: lane q labels the block (q / QH) of lane q mod QH,
      // and lane q < QH takes its second block from lane q + QH.
      const uint64_t h = uint64_t(item) >> i0;
      const uint64_t j = h * NB + S_load;
      const uint64_t gs = (j * n) >> L;
      const uint32_t q = lt % HALF_LANES;
      const uint64_t xo = gs + 16u * (q % QH);  // first element of the owning lane, a multiple of 8
      const Philox4 ph = philox4x64_10((xo >> 3) + q / QH, a.attempt, a.seed, 0);
      uint32_t w[8], wp[8];
#pragma unroll
      for (uint32_t e = 0; e < 8; ++e) {
        w[e] = uint32_t(ph.v[e >> 1] >> (32u * (e & 1u)));
        wp[e] = uint32_t(__shfl_xor(int(w[e]), int(QH), 64));
      }
      if (active) {
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e) {
          if (dt[e] != kDummyTag) dt[e] = L ? (w[e] >> (32u - L)) : 0u;
          if (dt[8 + e] != kDummyTag) dt[8 + e] = L ? (wp[e] >> (32u - L)) : 0u;
        }
      }
    } else if constexpr (FIRST) {
      const uint64_t h = uint64_t(item) >> i0;
      const uint64_t j = h * NB + S_load;
      const uint64_t gs = (j * n) >> L;
      const uint64_t x0 = gs + sb_load;  // multiple of 8
      if (active && dt[0] != kDummyTag) {
        const Philox4 p0 = philox4x64_10(x0 >> 3, a.attempt, a.seed, 0);
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e) {
          const uint32_t word = uint32_t(p0.v[e >> 1] >> (32u * (e & 1u)));
          if (dt[e] != kDummyTag) dt[e] = L ? (word >> (32u - L)) : 0u;
        }
      }
      if (active && dt[8] != kDummyTag) {
        const Philox4 p1 = philox4x64_10((x0 >> 3) + 1, a.attempt, a.seed, 0);
#pragma unroll
        for (uint32_t e = 0; e < 8; ++e) {
          const uint32_t word = uint32_t(p1.v[e >> 1] >> (32u * (e & 1u)));
          if (dt[8 + e] != kDummyTag) dt[8 + e] = L ? (word >> (32u - L)) : 0u;
        }
      }
    }
  };
  // first pass, groups not aligned to 8: stage the block through LDS and read
  // layout A back (the generic placement of Algorithm 3.1)
  auto staged_first_load = [&](uint32_t item) {
    const uint64_t h = uint64_t(item) >> i0;
    const uint64_t j_lo = h * NB;
    const uint64_t x_lo = (j_lo * n) >> L, x_hi = ((j_lo + NB) * n) >> L;
    const uint64_t c_lo = x_lo >> 3, c_hi = (x_hi + 7) >> 3;
    // HALF: round 0 stages the first halves and the tags, round 1 the second
    // halves; otherwise one round stages whole records
    for (uint32_t round = 0; round < (HALF ? 2u : 1u); ++round) {
      for (uint32_t t = tid; t < mp; t += nthr) {
        BOS_TR(0, 4, t);
        if constexpr (HALF) {
          shalf[t] = HalfOf<T>::zero();
        } else {
          srec[t] = zero_rec<T>();
        }
        if (round == 0) {
          BOS_TR(0, 5, t);
          stag[t] = kDummyTag;
        }
      }
      lds_barrier();
      for (uint64_t c = c_lo + tid; c < c_hi; c += nthr) {
        const Philox4 ph = philox4x64_10(c, a.attempt, a.seed, 0);
#pragma unroll
        for (uint32_t w = 0; w < 8; ++w) {
          const uint64_t x = c * 8 + w;
          if (x < x_lo || x >= x_hi) continue;
          const uint32_t word = uint32_t(ph.v[w >> 1] >> (32u * (w & 1u)));
          const uint64_t j = ((x + 1) * B - 1) / n;
          const uint64_t gs = (j * n) >> L;
          const uint32_t S = uint32_t(j - j_lo), s = uint32_t(x - gs);
          const uint32_t pi = S * ZP + s + (s >> 4);
          BOS_TR(0, 3, x);
          BOS_TR(0, 4, pi);
          if constexpr (HALF) {
            shalf[pi] = round == 0 ? rec_lo(X[x - a.x_off]) : rec_hi(X[x - a.x_off]);
          } else {
            srec[pi] = X[x - a.x_off];
          }
          if (round == 0) {
            BOS_TR(0, 5, pi);
            stag[pi] = L ? (word >> (32u - L)) : 0u;
          }
        }
      }
      lds_barrier();
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint32_t s = sb_load + e;
        const uint32_t pi = S_load * ZP + s + (s >> 4);
        if (active) BOS_TR(0, 4, pi);
        if constexpr (HALF) {
          if (round == 0) {
            if (active) BOS_TR(0, 5, pi);
            set_lo(rv[e], active ? shalf[pi] : HalfOf<T>::zero());
            tv[e] = active ? stag[pi] : kDummyTag;
          } else {
            set_hi(rv[e], active ? shalf[pi] : HalfOf<T>::zero());
          }
        } else {
          if (active) BOS_TR(0, 5, pi);
          rv[e] = active ? srec[pi] : zero_rec<T>();
          tv[e] = active ? stag[pi] : kDummyTag;
        }
      }
      lds_barrier();
    }
  };

  // ---- one block -----------------------------------------------------------
  // padded LDS index of this lane's slot e in layout B of the MergeSplit of
  // buckets at base0 / base1 (bB0, bB1: their layout-B lane bases; lB: the
  // lane's low slot bits)
  auto b_index = [&](uint32_t e, uint32_t b0, uint32_t b1, uint32_t bB0, uint32_t bB1, uint32_t lB) -> uint32_t {
    const uint32_t sl = (e & 7u) << (LQ - 4);
    // padded index of slot s = sl + lB: s + s/16 = sl + sl/16 + lB + lB/16
    // holds because sl is a multiple of 16 whenever LQ >= 8; for smaller Z
    // compute it directly
    if constexpr (LQ >= 8) {
      return ((e < 8) ? bB0 : bB1) + sl + (sl >> 4);
    } else {
      const uint32_t s2 = sl + lB;
      return (e < 8 ? b0 : b1) + s2 + (s2 >> 4);
    }
  };
  // HALF: second half of an exchange whose first halves (and tags) every
  // lane has stored at its indices src(e): read the first halves and tags at
  // dst(e), wait for the group, store this lane's second halves (still in rv)
  // at src(e), wait, read them at dst(e).
  // (the new first halves replace the stored ones in rv, which keeps the
  // second halves until they are stored: no extra registers)
  auto half_finish = [&](auto src, auto dst, auto sync) {
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (active) {
        BOS_TR(0, 4, dst(e));
        BOS_TR(0, 5, dst(e));
      }
      set_lo(rv[e], active ? shalf[dst(e)] : HalfOf<T>::zero());
      tv[e] = active ? stag[dst(e)] : kDummyTag;
    }
    sync();
    if (active) {
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        BOS_TR(0, 4, src(e));
        shalf[src(e)] = rec_hi(rv[e]);
      }
    }
    sync();
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      if (active) BOS_TR(0, 4, dst(e));
      set_hi(rv[e], active ? shalf[dst(e)] : HalfOf<T>::zero());
    }
  };
  // where the previous level left this lane's slots (layout B), for HALF
  uint32_t pb0 = 0, pb1 = 0, pbB0 = 0, pbB1 = 0, plB = 0;

  auto process = [&](uint32_t item) {
    const uint64_t r = uint64_t(item) & ((1ull << i0) - 1ull), h = uint64_t(item) >> i0;
    for (uint32_t d = 0; d < klev; ++d) {
      const uint32_t lev = i0 + d, shift = L - 1u - lev;
      const uint32_t S0 = ((ms >> d) << (d + 1)) | (ms & ((1u << d) - 1u)), S1 = S0 | (1u << d);
      const uint32_t base0 = S0 * ZP, base1 = S1 * ZP;
      // layout A: this lane's 16 slots are bucket (lt < TPM/2 ? S0 : S1),
      // slots 16*(lt mod TPM/2) + e
      const uint32_t baseA = (lt < HALF_LANES ? base0 : base1) + 17u * (lt % HALF_LANES);
      if (d > 0) {
        if constexpr (HALF) {
          half_finish([&](uint32_t e) { return b_index(e, pb0, pb1, pbB0, pbB1, plB); },
                      [&](uint32_t e) { return baseA + e; }, [] { lds_barrier(); });
        } else {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            if (active) {
              BOS_TR(0, 4, baseA + e);
              BOS_TR(0, 5, baseA + e);
            }
            rv[e] = active ? srec[baseA + e] : zero_rec<T>();
            tv[e] = active ? stag[baseA + e] : kDummyTag;
          }
        }
      }
      // prefix counts of (class-0 reals, dummies) in 16-bit halves
      uint32_t pk[16];
      uint32_t run = 0;
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint32_t tg = tv[e];
        const bool real = tg != kDummyTag;
        const bool c0 = real && ((tg >> shift) & 1u) == 0u;
        pk[e] = run;
        run += (c0 ? 1u : 0u) | (real ? 0u : 0x10000u);
      }
      uint32_t tot;
      const uint32_t excl = seg_scan<TPM>(active ? run : 0u, swave, &tot);
      const uint32_t x = tot & 0xFFFFu, nd = tot >> 16, y = 2u * Z - x - nd;
      const uint32_t need = x <= Z ? Z - x : 0u;
      uint32_t pm[16];
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint32_t pe = excl + pk[e];
        pm[e] = (pe & 0xFFFFu) + min(pe >> 16, need);
      }
      if (active) {
        BOS_TR(0, 6, ms * TPM + lt);
        spfx[ms * TPM + lt] = pm[0];
        if (LAST && lt == 0 && d + 1 == klev) {
          // bin loads of this block: S0 keeps min(x, Z) reals, S1 the rest of
          // the pair's reals (exact even when the MergeSplit overflowed)
          const uint32_t k0 = x < Z ? x : Z;
          BOS_TR(0, 7, S0);
          BOS_TR(0, 7, S1);
          sload[S0] = k0;
          sload[S1] = x + y - k0;
        }
        if (lt == 0 && (x > Z || y > Z)) {
          const uint64_t G = S0 >> (d + 1);
          const uint64_t v = brev_k(S0 & ((1u << d) - 1u), d);
          const uint64_t j = (((h << (klev - d - 1)) + G) << lev) + (r << d) + v;
          BOS_TR(0, 15, 0);
          atomicMin(a.status, (unsigned long long)((uint64_t(lev) << 32) | j));
        }
      }
      // -- layout A, q bits 0..3: register pairs
#pragma unroll
      for (uint32_t eb = 0; eb < 4; ++eb) {
        const uint32_t half = 1u << eb;
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          if (e & half) continue;
          const uint32_t e2 = e | half, es = e & ~(2u * half - 1u);
          const bool b = swap_bit(pm[es], pm[es | half], half, e & (half - 1u));
          const T r1 = rv[e], r2 = rv[e2];
          const uint32_t t1 = tv[e], t2 = tv[e2];
          rv[e] = sel(b, r2, r1);
          rv[e2] = sel(b, r1, r2);
          tv[e] = b ? t2 : t1;
          tv[e2] = b ? t1 : t2;
        }
      }
      // -- layout A, q bit 4: lanes l and l^1 (node = 2 lanes, half = 16)
      if constexpr (LQ >= 5) {
        const uint32_t P0 = dpp<kDppB0022>(pm[0]), Ph = dpp<kDppB1133>(pm[0]);
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const bool b = swap_bit(P0, Ph, 16u, e);
          const T pr = dpp<kDppXor1>(rv[e]);
          const uint32_t pt = dpp<kDppXor1>(tv[e]);
          rv[e] = sel(b, pr, rv[e]);
          tv[e] = b ? pt : tv[e];
        }
      }
      // -- layout A, q bit 5: lanes l and l^2 (node = 4 lanes, half = 32)
      if constexpr (LQ >= 6) {
        const uint32_t P0 = dpp<kDppB0000>(pm[0]), Ph = dpp<kDppB2222>(pm[0]);
        const uint32_t ioff = 16u * (lt & 1u);
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const bool b = swap_bit(P0, Ph, 32u, ioff + e);
          const T pr = dpp<kDppXor2>(rv[e]);
          const uint32_t pt = dpp<kDppXor2>(tv[e]);
          rv[e] = sel(b, pr, rv[e]);
          tv[e] = b ? pt : tv[e];
        }
      }
      // lane lt in layout B: q = e << (LQ-4) | lb1 << (LQ-5) | lb0 << (LQ-6) | rest
      uint32_t baseB0 = 0, baseB1 = 0, lowB = 0;
      if constexpr (HAS_B) {
        // A -> LDS (HALF: the first halves)
        if (active) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            BOS_TR(0, 4, baseA + e);
            BOS_TR(0, 5, baseA + e);
            if constexpr (HALF)
              shalf[baseA + e] = rec_lo(rv[e]);
            else
              srec[baseA + e] = rv[e];
            stag[baseA + e] = tv[e];
          }
        }
        lds_group_sync<TPM>();  // layouts A and B of one MergeSplit share its lanes
        // Layout B pairs lanes through DPP only for Z >= 1024; below that the
        // lanes simply take consecutive slots (conflict-free LDS access).
        const uint32_t lb0 = lt & 1u, lb1 = (lt >> 1) & 1u, rest = lt >> 2;
        lowB = (LQ >= 11) ? ((lb1 << (LQ - 5)) | (lb0 << (LQ - 6)) | rest) : lt;
        baseB0 = base0 + lowB + (lowB >> 4);
        baseB1 = base1 + lowB + (lowB >> 4);
        // HALF: the exchange first (its registers are free before the prefixes load)
        if constexpr (HALF) {
          half_finish([&](uint32_t e) { return baseA + e; },
                      [&](uint32_t e) { return b_index(e, base0, base1, baseB0, baseB1, lowB); },
                      [] { lds_group_sync<TPM>(); });
        }
        // marks prefix at node boundaries (multiples of 16 slots)
        uint32_t pv[16], pvh[16];
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t q = e << (LQ - 4);
          const uint32_t i1 = (q & 15u) == 0u ? (q >> 4) : 0u;
          if (active) BOS_TR(0, 6, ms * TPM + i1);
          pv[e] = active ? spfx[ms * TPM + i1] : 0u;
          if constexpr (LQ >= 11) {
            const uint32_t qh = q | (1u << (LQ - 5));
            if (active) BOS_TR(0, 6, ms * TPM + (qh >> 4));
            pvh[e] = active ? spfx[ms * TPM + (qh >> 4)] : 0u;
          } else {
            pvh[e] = 0;
          }
        }
        if constexpr (!HALF) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            const uint32_t pi = b_index(e, base0, base1, baseB0, baseB1, lowB);
            if (active) {
              BOS_TR(0, 4, pi);
              BOS_TR(0, 5, pi);
            }
            rv[e] = active ? srec[pi] : zero_rec<T>();
            tv[e] = active ? stag[pi] : kDummyTag;
          }
        }
        // -- layout B, q bit LQ-6 (lane bit 0), only for Z = 2048
        if constexpr (LQ - 6 >= 6) {
          const uint32_t half = 1u << (LQ - 6);
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            // node: q bits 0..LQ-6 cleared; its start and middle are 16-aligned
            const uint32_t qn = (e << (LQ - 4)) | (lb1 << (LQ - 5));
            BOS_TR(0, 6, ms * TPM + (qn >> 4));
            BOS_TR(0, 6, ms * TPM + ((qn | half) >> 4));
            const uint32_t P0 = spfx[ms * TPM + (qn >> 4)];
            const uint32_t Ph = spfx[ms * TPM + ((qn | half) >> 4)];
            const bool b = swap_bit(P0, Ph, half, rest);
            const T pr = dpp<kDppXor1>(rv[e]);
            const uint32_t pt = dpp<kDppXor1>(tv[e]);
            rv[e] = sel(b, pr, rv[e]);
            tv[e] = b ? pt : tv[e];
          }
        }
        // -- layout B, q bit LQ-5 (lane bit 1), for Z >= 1024
        if constexpr (LQ - 5 >= 6) {
          const uint32_t half = 1u << (LQ - 5);
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            const bool b = swap_bit(pv[e], pvh[e], half, (lb0 << (LQ - 6)) | rest);
            const T pr = dpp<kDppXor2>(rv[e]);
            const uint32_t pt = dpp<kDppXor2>(tv[e]);
            rv[e] = sel(b, pr, rv[e]);
            tv[e] = b ? pt : tv[e];
          }
        }
        // -- layout B, q bits LQ-4 .. LQ-1: register pairs (those >= 6)
#pragma unroll
        for (uint32_t eb = 0; eb < 4; ++eb) {
          if (LQ - 4 + eb < 6) continue;
          const uint32_t hb = 1u << eb;
          const uint32_t half = 1u << (LQ - 4 + eb);
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            if (e & hb) continue;
            const uint32_t e2 = e | hb, es = e & ~(2u * hb - 1u);
            const uint32_t i = ((e & (hb - 1u)) << (LQ - 4)) | lowB;
            const bool b = swap_bit(pv[es], pv[es | hb], half, i);
            const T r1 = rv[e], r2 = rv[e2];
            const uint32_t t1 = tv[e], t2 = tv[e2];
            rv[e] = sel(b, r2, r1);
            rv[e2] = sel(b, r1, r2);
            tv[e] = b ? t2 : t1;
            tv[e2] = b ? t1 : t2;
          }
        }
      }
      // -- hand the level's output to LDS (next level or last-pass finish)
      if (d + 1 < klev || LAST) {
        if constexpr (HAS_B) {
          // every lane rewrites exactly the layout-B slots it read: no
          // barrier (HALF: the first halves; the next level's start, or the
          // last pass's finish, completes the exchange)
          if (active) {
#pragma unroll
            for (uint32_t e = 0; e < 16; ++e) {
              const uint32_t pi = b_index(e, base0, base1, baseB0, baseB1, lowB);
              BOS_TR(0, 4, pi);
              BOS_TR(0, 5, pi);
              if constexpr (HALF)
                shalf[pi] = rec_lo(rv[e]);
              else
                srec[pi] = rv[e];
              stag[pi] = tv[e];
            }
          }
          pb0 = base0;
          pb1 = base1;
          pbB0 = baseB0;
          pbB1 = baseB1;
          plB = lowB;
        } else {
          if (active) {
#pragma unroll
            for (uint32_t e = 0; e < 16; ++e) {
              BOS_TR(0, 4, baseA + e);
              BOS_TR(0, 5, baseA + e);
              srec[baseA + e] = rv[e];
              stag[baseA + e] = tv[e];
            }
          }
        }
        lds_barrier();
      } else {
        // last level of a non-last pass: write the 2^klev output buckets
        // (LDS bucket S is output digit bitrev(S)) straight from registers
        T* RO = static_cast<T*>(a.rec_out);
        const uint64_t ob0 = (h << (i0 + klev)) + (r << klev) + brev_k(S0, klev);
        const uint64_t ob1 = (h << (i0 + klev)) + (r << klev) + brev_k(S1, klev);
        if (active) {
#pragma unroll
          for (uint32_t e = 0; e < 16; ++e) {
            uint64_t gi;
            if constexpr (HAS_B) {
              const uint32_t s = ((e & 7u) << (LQ - 4)) | lowB;
              gi = (((e < 8) ? ob0 : ob1) << LZ) + s;
            } else {
              gi = (((lt < HALF_LANES) ? ob0 : ob1) << LZ) + sb_load + e;
            }
            BOS_TR(0, 10, gi);
            BOS_TR(0, 11, gi);
            RO[gi - a.out_slot0] = rv[e];
            a.tag_out[gi - a.out_slot0] = tv[e];
          }
        }
      }
    }
  };

  // split last pass: every bin's slots in layout P, then compaction and
  // the write of its reals
  auto finish_bins_split = [&](uint32_t blk) {
    if constexpr (HALF) {
      const uint32_t HLn = Z >> 4;
      const uint32_t S = active ? tid / HLn : 0u, lq = active ? tid % HLn : 0u;
      const uint32_t pbase = S * ZP + 17u * lq;
      half_finish([&](uint32_t e) { return b_index(e, pb0, pb1, pbB0, pbB1, plB); },
                  [&](uint32_t e) { return pbase + e; }, [] { lds_barrier(); });
      finish_split<R, LZ, SPLIT_FIN, FULL, true>(a, blk, klev, srec, stag, srhi, saux, sload, spfx, swave, rv, tv);
    } else {
      finish_split<R, LZ, SPLIT_FIN, FULL, false>(a, blk, klev, srec, stag, srhi, saux, sload, spfx, swave, rv, tv);
    }
  };

  if constexpr (BATCH && (!LAST || SPLIT)) {
    item0 += a.item_off;
    if (FIRST && !aligned) {
      staged_first_load(item0);
    } else {
      issue_load(item0, rv, tv);
      finish_load(item0, tv);
    }
    process(item0);
    if constexpr (SPLIT) finish_bins_split(item0);
  } else if constexpr (!LAST || SPLIT) {
    // persistent walk over blocks: item = blockIdx.x, + gridDim.x, ...  The
    // next block's loads are issued after the current one is done: with no
    // prefetch registers a pass runs three workgroups per CU at 2^3 Z slots
    // per block, and their interleaving hides the loads better than a
    // register prefetch with fewer workgroups did.
    // items are global block indices: a staged launch runs blocks
    // item_off .. item_off + nitems - 1
    const uint32_t ioff = a.item_off, iend = ioff + nitems;
    uint32_t item = item0 + ioff;
    if (item >= iend) return;
    if (FIRST && !aligned) {
      staged_first_load(item);
    } else {
      issue_load(item, rv, tv);
      finish_load(item, tv);
    }
    for (;;) {
      const uint32_t next = item + gridDim.x;
      const bool has_next = next < iend;
      process(item);
      if constexpr (SPLIT) finish_bins_split(item);
      if (!has_next) break;
      item = next;
      lds_barrier();  // LDS of the previous block is no longer read
      if (FIRST && !aligned) {
        staged_first_load(item);
      } else {
        issue_load(item, rv, tv);
        finish_load(item, tv);
      }
    }
  } else {
    // Last pass: one block per launch block; the block index is a ticket so
    // that the look-back of the strip only waits on blocks that started
    // earlier.
    if (tid == 0) smisc[0] = atomicAdd(a.ticket, 1u);
    lds_barrier();
    const uint32_t blk = smisc[0];
    if (FIRST && !aligned) {
      staged_first_load(blk);
    } else {
      issue_load(blk, rv, tv);
      finish_load(blk, tv);
    }
    process(blk);
    // every final bin (LDS bucket S) now sits in LDS with padded slots
    finish_bins<R, LZ, FULL>(a, blk, klev, srec, stag, srhi, saux, sload, soff);
  }
  (void)nitems;
}

template <int R, int LZ, int MODE>
__global__ __launch_bounds__(kMaxThreads) void route_kernel(PassArgs a, uint32_t nitems) {
  route_run<R, LZ, MODE, false>(a, nitems, blockIdx.x);
}

// The passes after the first whose LDS exchanges go in two halves (kW3
// below) are compiled for a register budget that lets as many workgroups
// share a CU as their LDS allows: three waves per SIMD (at most 168 VGPRs)
// for 16-byte records, four (at most 128) for 8-byte ones.  The first pass,
// which also computes the labels, keeps the default allocation (it would
// spill).
template <int R, int LZ, int MODE>
constexpr bool kW3 = lds_rec_bytes(R, 1u << LZ, (MODE & 2) && !(MODE & 4)) < uint32_t(R) && LZ >= 6 && !(MODE & 1);
template <int R>
constexpr int kWavesPerSimd = R == 16 ? 3 : 4;

template <int R, int LZ, int MODE>
__global__ __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<R>, 8))) void
route_kernel_w3(PassArgs a, uint32_t nitems) {
  route_run<R, LZ, MODE, false>(a, nitems, blockIdx.x);
}

// Batched routing: segment s of the launch is one instance's pass; its blocks
// are blockIdx.x in [blk_start[s], blk_start[s+1]).
template <int R, int LZ, int MODE, bool W3>
__device__ __forceinline__ void route_b_body(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs) {
  uint32_t lo = 0, hi = nsegs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (blk_start[mid] <= blockIdx.x)
      lo = mid;
    else
      hi = mid;
  }
  const PassArgs a = segs[lo];
  route_run<R, LZ, MODE, true>(a, 0u, blockIdx.x - blk_start[lo]);
}
template <int R, int LZ, int MODE>
__global__ __launch_bounds__(kMaxThreads) void route_kernel_b(const PassArgs* segs, const uint32_t* blk_start,
                                                              uint32_t nsegs) {
  route_b_body<R, LZ, MODE, false>(segs, blk_start, nsegs);
}
template <int R, int LZ, int MODE>
__global__ __launch_bounds__(kMaxThreads) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd<R>, 8))) void
route_kernel_b_w3(const PassArgs* segs, const uint32_t* blk_start, uint32_t nsegs) {
  route_b_body<R, LZ, MODE, true>(segs, blk_start, nsegs);
}

}  // namespace bos
