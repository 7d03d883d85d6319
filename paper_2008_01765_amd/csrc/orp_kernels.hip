// orp_kernels.hip — gfx950 kernels of the routing phase of bucket ORP
// (Algorithm 3.1 and Section 3.2 of Asharov et al., SOSA 2020).
//
// One launch runs one *pass*: `klev` consecutive butterfly levels fused in one
// block.  A block owns the 2^klev buckets that the pass's MergeSplits connect:
// it reads them from HBM into LDS (coalesced, Z contiguous slots per bucket),
// runs the klev levels in LDS and writes 2^klev contiguous output buckets.
// The first pass reads the input records and draws the labels (Philox4x64-10)
// on chip instead of reading a slot array; the last pass also finishes every
// bin (random permutation or oblivious sort of the bin, Section 3.2) and strips
// the dummies.
//
// Obliviousness: every HBM and LDS address below is a function of
// (n, Z, klev, level, block, thread) only.  Labels and record contents enter
// the computation only through comparisons whose results drive register
// selects, never an address.  The strip writes depend on the bin loads, which
// the paper reveals on purpose (Lemma 3.3).
//
// MergeSplit inside LDS: the two input buckets of a MergeSplit form a 2Z-slot
// array; real elements whose next label bit is 0 are "marked", and so are the
// first Z - x dummies (x = marked reals), the dummy tagging of Section 4.1.  An
// oblivious tight-compaction network then moves exactly Z marked slots into the
// lower bucket and the rest into the upper one.  The network is the
// offset-compaction recursion of Sasy, Johnson and Goldberg (CCS 2022): a node
// of 2^j slots compacts its halves with cyclic offsets z mod 2^(j-1) and
// (z + m) mod 2^(j-1), then conditionally swaps slot i with slot i + 2^(j-1);
// every offset follows from the exclusive prefix count of marks at the node's
// start, so all control bits come from one prefix scan.  The 2Z slots are
// spread over 2Z/16 threads holding 16 slots each; the log2(2Z) swap stages run
// four at a time inside registers, the slot-to-register assignment changing
// through LDS between groups of four.  Bucket contents are sets (Algorithm 3.1);
// the order of slots inside a bucket is the network's.
#include "bos_common.h"

namespace bos {

__device__ __forceinline__ uint32_t padidx(uint32_t s) { return s + (s >> 4); }

__device__ __forceinline__ uint32_t bitrev(uint32_t x, uint32_t k) {
  return k ? (__brev(x) >> (32u - k)) : 0u;
}

// Exclusive scan of v over aligned segments of `seg` consecutive threads
// (seg a power of two); *total receives the segment's sum.  Every thread of the
// block must call it (it may synchronize).
__device__ __forceinline__ uint32_t segmented_excl_scan(uint32_t v, uint32_t seg, uint32_t* swave,
                                                        uint32_t* total) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t w = seg < 64u ? seg : 64u;
  uint32_t x = v;
#pragma unroll
  for (uint32_t off = 1; off < 64u; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (off < w && (lane & (w - 1u)) >= off) x += y;
  }
  if (seg <= 64u) {
    *total = __shfl(x, int(lane | (w - 1u)), 64);
    return x - v;
  }
  if (lane == 63u) swave[wave] = x;
  __syncthreads();
  const uint32_t wps = seg >> 6, w0 = wave & ~(wps - 1u);
  uint32_t pre = 0, tot = 0;
  for (uint32_t q = 0; q < wps; ++q) {
    const uint32_t t = swave[w0 + q];
    if (w0 + q < wave) pre += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return pre + x - v;
}

// Bitonic sort of every Z-slot bin of the block's LDS (ascending), with the
// order supplied by `less(a_index, b_index)` on padded slot indices.  Addresses
// depend on (m, Z) only.
template <typename Less, typename Swap>
__device__ __forceinline__ void bitonic_bins(uint32_t m, uint32_t Z, Less less, Swap swp) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x, half_m = m >> 1;
  for (uint32_t k2 = 2; k2 <= Z; k2 <<= 1) {
    for (uint32_t j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
      for (uint32_t p = tid; p < half_m; p += nthr) {
        const uint32_t lo = ((p & ~(j2 - 1u)) << 1) | (p & (j2 - 1u));
        const uint32_t hi = lo + j2;
        const bool up = (k2 == Z) || ((lo & k2) == 0);
        const uint32_t a = padidx(lo), b = padidx(hi);
        const bool sw = up ? less(b, a) : less(a, b);
        swp(a, b, sw);
      }
      __syncthreads();
    }
  }
}

// MODE bit 0: first pass (reads the input records), bit 1: last pass (finishes
// the bins and strips).  Separate instantiations keep the passes apart in
// kernel traces and let the compiler drop the unused phases.
template <int R, int MODE>
__global__ __launch_bounds__(kMaxThreads) void orp_pass_kernel(PassArgs a) {
  using T = typename RecOf<R>::T;
  constexpr bool first = (MODE & 1) != 0, last = (MODE & 2) != 0;
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t Z = a.z, lz = a.lz, klev = a.klev, NB = 1u << klev;
  const uint32_t m = Z << klev, mp = m + (m >> 4);
  T* srec = reinterpret_cast<T*>(smem);
  uint32_t* stag = reinterpret_cast<uint32_t*>(smem + size_t(mp) * R);
  uint32_t* spfx = stag + mp;          // m/16 marks-prefix entries
  uint32_t* sload = spfx + (m >> 4);   // NB bin loads
  uint32_t* soff = sload + NB;         // 2*NB words: 64-bit output offset of every bin
  uint32_t* swave = soff + 2 * NB;     // 64 scan words
  uint32_t* smisc = swave + 64;        // 16 words
  uint32_t* srhi = smisc + 16;         // last pass, shuffle: high words of the random keys
  uint16_t* saux = reinterpret_cast<uint16_t*>(srhi + mp);  // last pass, shuffle: p | dummy<<15

  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint64_t n = a.n, B = a.buckets;
  const uint32_t L = a.levels, i0 = a.level0;

  // Block index.  The last pass takes a ticket so that the look-back of the
  // strip only ever waits on blocks that started earlier.
  uint32_t blk = blockIdx.x;
  if constexpr (last) {
    if (tid == 0) smisc[0] = atomicAdd(a.ticket, 1u);
    __syncthreads();
    blk = smisc[0];
  }
  const uint64_t r = uint64_t(blk) & ((1ull << i0) - 1ull);
  const uint64_t h = uint64_t(blk) >> i0;

  // ---- load the block's 2^klev buckets into LDS -------------------------
  if constexpr (first) {
    for (uint32_t t = tid; t < m; t += nthr) {
      srec[padidx(t)] = zero_rec<T>();
      stag[padidx(t)] = kDummyTag;
    }
    __syncthreads();
    // Groups j = h*NB + g hold X[floor(jn/B), floor((j+1)n/B)) (Algorithm 3.1,
    // initial placement); labels: 32-bit word (x mod 8) of Philox block x/8.
    const T* X = static_cast<const T*>(a.x_in);
    const uint64_t j_lo = h * NB;
    const uint64_t x_lo = (j_lo * n) / B, x_hi = ((j_lo + NB) * n) / B;
    const uint64_t c_lo = x_lo >> 3, c_hi = (x_hi + 7) >> 3;
    for (uint64_t c = c_lo + tid; c < c_hi; c += nthr) {
      const Philox4 ph = philox4x64_10(c, a.attempt, a.seed, 0);
#pragma unroll
      for (uint32_t w = 0; w < 8; ++w) {
        const uint64_t x = c * 8 + w;
        if (x < x_lo || x >= x_hi) continue;
        const uint32_t word = uint32_t(ph.v[w >> 1] >> (32u * (w & 1u)));
        const uint32_t lab = L ? (word >> (32u - L)) : 0u;
        const uint64_t j = ((x + 1) * B - 1) / n;
        const uint64_t gs = (j * n) / B;
        const uint32_t s = uint32_t((j - j_lo) << lz) + uint32_t(x - gs);
        srec[padidx(s)] = X[x];
        stag[padidx(s)] = lab;
      }
    }
  } else {
    const T* RI = static_cast<const T*>(a.rec_in);
    for (uint32_t t = tid; t < m; t += nthr) {
      const uint32_t g = t >> lz, s = t & (Z - 1u);
      const uint64_t bucket = (h << (i0 + klev)) + (uint64_t(g) << i0) + r;
      const uint64_t gi = (bucket << lz) + s;
      srec[padidx(t)] = RI[gi];
      stag[padidx(t)] = a.tag_in[gi];
    }
  }
  __syncthreads();

  // ---- klev butterfly levels, each MergeSplit an in-LDS compaction --------
  const uint32_t LQ = lz + 1, S2 = 2u * Z, TPM = S2 >> 4;
  const bool active = tid < (m >> 4);
  const uint32_t ms = active ? tid / TPM : 0u, lt = active ? tid % TPM : 0u;
  for (uint32_t d = 0; d < klev; ++d) {
    const uint32_t lev = i0 + d, shift = L - 1u - lev;
    const uint32_t S0 = ((ms >> d) << (d + 1)) | (ms & ((1u << d) - 1u)), S1 = S0 | (1u << d);
    const uint32_t base0 = S0 << lz, base1 = S1 << lz;
    // Slot index (unpadded) of position q of this MergeSplit.
#define QSLOT(q) (((q) < Z ? base0 : base1) + ((q) & (Z - 1u)))

    // prefix counts of (class-0 reals, dummies), packed in 16-bit halves
    uint32_t pk[16];
    uint32_t run = 0;
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint32_t q = lt * 16u + e;
      const uint32_t tg = active ? stag[padidx(QSLOT(q))] : kDummyTag;
      const bool real = tg != kDummyTag;
      const bool c0 = real && ((tg >> shift) & 1u) == 0u;
      pk[e] = run;
      run += (c0 ? 1u : 0u) | (real ? 0u : 0x10000u);
    }
    uint32_t tot;
    const uint32_t excl = segmented_excl_scan(active ? run : 0u, TPM, swave, &tot);
    const uint32_t x = tot & 0xFFFFu, nd = tot >> 16, y = S2 - x - nd;
    const uint32_t need = x <= Z ? Z - x : 0u;
    uint32_t pm[16];
#pragma unroll
    for (uint32_t e = 0; e < 16; ++e) {
      const uint32_t pe = excl + pk[e];
      pm[e] = (pe & 0xFFFFu) + min(pe >> 16, need);
    }
    if (active) {
      spfx[ms * TPM + lt] = pm[0];
      if (lt == 0 && (x > Z || y > Z)) {
        // first overflow: MergeSplit (lev, j) with
        // j = 2^lev * (2^(klev-d-1) h + S0 >> (d+1)) + r 2^d + bitrev_d(S0 mod 2^d)
        const uint64_t G = S0 >> (d + 1);
        const uint64_t v = bitrev(S0 & ((1u << d) - 1u), d);
        const uint64_t j = (((h << (klev - d - 1)) + G) << lev) + (r << d) + v;
        atomicMin(a.status, (unsigned long long)((uint64_t(lev) << 32) | j));
      }
    }
    __syncthreads();

    const uint32_t NL = (LQ + 3u) >> 2;
    for (uint32_t l = 0; l < NL; ++l) {
      const uint32_t bb = min(4u * l, LQ - 4u);
      const uint32_t low = lt & ((1u << bb) - 1u), high = lt >> bb;
      T rv[16];
      uint32_t tv[16], pv[16];
#pragma unroll
      for (uint32_t e = 0; e < 16; ++e) {
        const uint32_t q = (high << (bb + 4u)) | (e << bb) | low;
        const uint32_t si = padidx(QSLOT(q));
        rv[e] = active ? srec[si] : zero_rec<T>();
        tv[e] = active ? stag[si] : kDummyTag;
        if (l == 0) {
          pv[e] = pm[e];
        } else {
          const uint32_t pq = (high << (bb + 4u)) | (e << bb);
          pv[e] = (active && (pq & 15u) == 0u) ? spfx[ms * TPM + (pq >> 4)] : 0u;
        }
      }
#pragma unroll
      for (uint32_t eb = 0; eb < 4; ++eb) {
        const uint32_t j = bb + eb + 1u;
        if (j < 4u * l + 1u) continue;  // stage done in an earlier layout
        const uint32_t half = 1u << (j - 1u);
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          if (e & (1u << eb)) continue;
          const uint32_t e2 = e | (1u << eb);
          const uint32_t ep = e & ~((2u << eb) - 1u);
          const uint32_t Pp = pv[ep], Pph = pv[ep | (1u << eb)];
          const uint32_t z = Pp & ((half << 1) - 1u), mm = Pph - Pp;
          const bool s = (((z & (half - 1u)) + mm) >= half) != (z >= half);
          const uint32_t tt = (z + mm) & (half - 1u);
          const uint32_t i = ((e & ((1u << eb) - 1u)) << bb) | low;
          const bool b = s != (i >= tt);
          const T r1 = rv[e], r2 = rv[e2];
          const uint32_t t1 = tv[e], t2 = tv[e2];
          rv[e] = sel(b, r2, r1);
          rv[e2] = sel(b, r1, r2);
          tv[e] = b ? t2 : t1;
          tv[e2] = b ? t1 : t2;
        }
      }
      if (active) {
#pragma unroll
        for (uint32_t e = 0; e < 16; ++e) {
          const uint32_t q = (high << (bb + 4u)) | (e << bb) | low;
          const uint32_t si = padidx(QSLOT(q));
          srec[si] = rv[e];
          stag[si] = tv[e];
        }
      }
      __syncthreads();
    }
#undef QSLOT
  }

  // ---- not the last pass: write 2^klev contiguous output buckets ----------
  if constexpr (!last) {
    T* RO = static_cast<T*>(a.rec_out);
    for (uint32_t t = tid; t < m; t += nthr) {
      const uint32_t S = t >> lz, s = t & (Z - 1u);
      const uint64_t bucket = (h << (i0 + klev)) + (r << klev) + bitrev(S, klev);
      const uint64_t gi = (bucket << lz) + s;
      RO[gi] = srec[padidx(t)];
      a.tag_out[gi] = stag[padidx(t)];
    }
    return;
  } else {
  // ---- last pass: finish every bin (Section 3.2) --------------------------
  // Record order with dummies last.
  auto less_rec = [&](uint32_t ia, uint32_t ib) {
    const bool da = stag[ia] == kDummyTag, db = stag[ib] == kDummyTag;
    if (da || db) return !da && db;
    return rec_less(srec[ia], srec[ib]);
  };
  auto swap_rt = [&](uint32_t ia, uint32_t ib, bool sw) {
    const T ra = srec[ia], rb = srec[ib];
    const uint32_t ta = stag[ia], tb = stag[ib];
    srec[ia] = sel(sw, rb, ra);
    srec[ib] = sel(sw, ra, rb);
    stag[ia] = sw ? tb : ta;
    stag[ib] = sw ? ta : tb;
  };
  bitonic_bins(m, Z, less_rec, swap_rt);

  // Bin loads: the bin's reals now occupy its first slots.
  for (uint32_t S = tid; S < NB; S += nthr) sload[S] = 0;
  __syncthreads();
  for (uint32_t t = tid; t < m; t += nthr)
    if (stag[padidx(t)] != kDummyTag) atomicAdd(&sload[t >> lz], 1u);
  __syncthreads();

  if (a.fin == 0) {
    // Random permutation of each bin: the p-th real of global bin b (in record
    // order) gets key r(b*Z + p) = word (g mod 4) of Philox block g/4 with key
    // (seed, 1); the bin is then sorted by (r, p), dummies last.
    for (uint32_t t4 = tid * 4u; t4 < m; t4 += nthr * 4u) {
      const uint32_t S = t4 >> lz, p0 = t4 & (Z - 1u);
      const uint64_t gb = uint64_t(blk) * NB + bitrev(S, klev);
      const uint64_t g0 = gb * Z + p0;  // Z >= 8, so g0 is a multiple of 4
      const Philox4 ph = philox4x64_10(g0 >> 2, a.attempt, a.seed, 1);
#pragma unroll
      for (uint32_t w = 0; w < 4; ++w) {
        const uint32_t si = padidx(t4 + w);
        const bool dummy = stag[si] == kDummyTag;
        stag[si] = uint32_t(ph.v[w]);
        srhi[si] = uint32_t(ph.v[w] >> 32);
        saux[si] = uint16_t((p0 + w) | (dummy ? 0x8000u : 0u));
      }
    }
    __syncthreads();
    auto less_key = [&](uint32_t ia, uint32_t ib) {
      const uint32_t xa = saux[ia], xb = saux[ib];
      const bool da = xa & 0x8000u, db = xb & 0x8000u;
      if (da || db) return !da && db;
      const uint64_t ka = (uint64_t(srhi[ia]) << 32) | stag[ia];
      const uint64_t kb = (uint64_t(srhi[ib]) << 32) | stag[ib];
      return ka < kb || (ka == kb && xa < xb);
    };
    auto swap_key = [&](uint32_t ia, uint32_t ib, bool sw) {
      const T ra = srec[ia], rb = srec[ib];
      const uint32_t ta = stag[ia], tb = stag[ib], ha = srhi[ia], hb = srhi[ib];
      const uint16_t xa = saux[ia], xb = saux[ib];
      srec[ia] = sel(sw, rb, ra);
      srec[ib] = sel(sw, ra, rb);
      stag[ia] = sw ? tb : ta;
      stag[ib] = sw ? ta : tb;
      srhi[ia] = sw ? hb : ha;
      srhi[ib] = sw ? ha : hb;
      saux[ia] = sw ? xb : xa;
      saux[ib] = sw ? xa : xb;
    };
    bitonic_bins(m, Z, less_key, swap_key);
  }

  // ---- strip and concatenate: decoupled look-back over blocks -------------
  if (tid == 0) {
    uint64_t agg = 0;
    for (uint32_t S = 0; S < NB; ++S) agg += sload[S];
    uint64_t excl = 0;
    const uint64_t kVal = (1ull << 62) - 1ull;
    if (blk == 0) {
      __hip_atomic_store(&a.scan[0], (2ull << 62) | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(&a.scan[blk], (1ull << 62) | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      int64_t p = int64_t(blk) - 1;
      while (p >= 0) {
        const unsigned long long w =
            __hip_atomic_load(&a.scan[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t flag = uint32_t(w >> 62);
        if (flag == 0) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += w & kVal;
        if (flag == 2) break;
        --p;
      }
      __hip_atomic_store(&a.scan[blk], (2ull << 62) | (excl + agg), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    // bin offsets in global bin order u = 0..NB-1 (LDS bucket bitrev(u))
    uint64_t off = excl;
    for (uint32_t u = 0; u < NB; ++u) {
      const uint32_t S = bitrev(u, klev);
      soff[2 * S] = uint32_t(off);
      soff[2 * S + 1] = uint32_t(off >> 32);
      off += sload[S];
    }
  }
  __syncthreads();
  T* OUT = static_cast<T*>(a.out);
  for (uint32_t t = tid; t < m; t += nthr) {
    const uint32_t S = t >> lz, p = t & (Z - 1u);
    if (p < sload[S]) {
      const uint64_t dst = (uint64_t(soff[2 * S + 1]) << 32 | soff[2 * S]) + p;
      if (dst < n) OUT[dst] = srec[padidx(t)];
    }
  }
  }  // last pass
}

// status := no overflow; scan words and tickets := 0 (a kernel rather than a
// memset so that the sequence can be captured into a graph).
__global__ void fill_u64_kernel(unsigned long long* p, uint64_t count, unsigned long long v) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void labels_kernel(uint32_t* out, uint64_t n, uint32_t L, uint64_t seed, uint32_t attempt) {
  const uint64_t c = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c * 8 >= n) return;
  const Philox4 ph = philox4x64_10(c, attempt, seed, 0);
#pragma unroll
  for (uint32_t w = 0; w < 8; ++w) {
    const uint64_t x = c * 8 + w;
    if (x >= n) break;
    const uint32_t word = uint32_t(ph.v[w >> 1] >> (32u * (w & 1u)));
    out[x] = L ? (word >> (32u - L)) : 0u;
  }
}

// ---- host-side launchers -------------------------------------------------

hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint32_t threads = 256;
  uint64_t blocks = (count + threads - 1) / threads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(uint32_t(blocks)), dim3(threads), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t launch_labels(uint32_t* out, uint64_t n, uint32_t L, uint64_t seed, uint32_t attempt,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t chunks = (n + 7) / 8;
  const uint32_t threads = 256;
  hipLaunchKernelGGL(labels_kernel, dim3(uint32_t((chunks + threads - 1) / threads)), dim3(threads), 0,
                     s, out, n, L, seed, attempt);
  return hipGetLastError();
}

template <int R, int MODE>
static hipError_t launch_pass_t(const PassArgs& a, uint32_t nblocks, hipStream_t s) {
  const uint32_t m = a.z << a.klev;
  uint32_t threads = m >> 4;
  if (threads < 64) threads = 64;
  const uint32_t lds = pass_lds_bytes(R, a.z, a.klev, (MODE & 2) && a.fin == 0, true);  // whole records in LDS
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&orp_pass_kernel<R, MODE>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((orp_pass_kernel<R, MODE>), dim3(nblocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

template <int R>
static hipError_t launch_pass_r(const PassArgs& a, int mode, uint32_t nblocks, hipStream_t s) {
  switch (mode) {
    case 0: return launch_pass_t<R, 0>(a, nblocks, s);
    case 1: return launch_pass_t<R, 1>(a, nblocks, s);
    case 2: return launch_pass_t<R, 2>(a, nblocks, s);
    default: return launch_pass_t<R, 3>(a, nblocks, s);
  }
}

hipError_t launch_pass(int rec, const PassArgs& a, bool first, bool last, uint32_t nblocks, hipStream_t s) {
  const int mode = (first ? 1 : 0) | (last ? 2 : 0);
  return rec == 8 ? launch_pass_r<8>(a, mode, nblocks, s) : launch_pass_r<16>(a, mode, nblocks, s);
}

}  // namespace bos
