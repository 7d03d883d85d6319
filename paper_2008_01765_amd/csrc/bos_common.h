// bos_common.h — device-side building blocks shared by the gfx950 kernels of
// libbos: record types and comparisons, the Philox4x64-10 generator, and the
// argument blocks of the routing kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bos {

constexpr uint32_t kDummyTag = 0xFFFFFFFFu;  // tag of a dummy slot; real tags are labels < 2^31
constexpr uint64_t kNoOverflow = ~0ull;      // status word when no MergeSplit overflowed
constexpr int kMaxThreads = 512;             // threads per routing block
// Outputs per workgroup of a merge pass: 4096 records of 8 bytes, 2048 of 16
// (the tile and its staging copy fit four workgroups' LDS per CU either way).
__host__ __device__ constexpr uint32_t merge_tile_records(int rec) { return rec == 8 ? 4096u : 2048u; }

// Record of BOS_REC_U32U32 (8 bytes) or BOS_REC_U64U64 (16 bytes).
template <int R> struct RecOf;
template <> struct RecOf<8> { using T = uint2; };
template <> struct RecOf<16> { using T = uint4; };

// Native vector types of the records, for arrays that must stay in registers
// (arrays of the uint2/uint4 structs can end up in scratch memory).
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
template <typename T> struct NativeOf;
template <> struct NativeOf<uint2> { using V = v2u; };
template <> struct NativeOf<uint4> { using V = v4u; };

__device__ __forceinline__ uint64_t key_of(uint2 r) { return r.x; }
__device__ __forceinline__ uint64_t pay_of(uint2 r) { return r.y; }
__device__ __forceinline__ uint64_t key_of(uint4 r) { return uint64_t(r.x) | (uint64_t(r.y) << 32); }
__device__ __forceinline__ uint64_t pay_of(uint4 r) { return uint64_t(r.z) | (uint64_t(r.w) << 32); }

// Unsigned lexicographic order on (key, payload).
__device__ __forceinline__ bool rec_less(uint2 a, uint2 b) {
  const uint64_t ka = (uint64_t(a.x) << 32) | a.y, kb = (uint64_t(b.x) << 32) | b.y;
  return ka < kb;
}
__device__ __forceinline__ bool rec_less(uint4 a, uint4 b) {
  const uint64_t ka = key_of(a), kb = key_of(b);
  return (ka < kb) | ((ka == kb) & (pay_of(a) < pay_of(b)));  // no short-circuit branches
}

template <typename T> __device__ __forceinline__ T zero_rec();
template <> __device__ __forceinline__ uint2 zero_rec<uint2>() { return make_uint2(0, 0); }
template <> __device__ __forceinline__ uint4 zero_rec<uint4>() { return make_uint4(0, 0, 0, 0); }
template <typename T> __device__ __forceinline__ T max_rec();
template <> __device__ __forceinline__ uint2 max_rec<uint2>() { return make_uint2(~0u, ~0u); }
template <> __device__ __forceinline__ uint4 max_rec<uint4>() { return make_uint4(~0u, ~0u, ~0u, ~0u); }

template <typename T> __device__ __forceinline__ T sel(bool c, T a, T b) { return c ? a : b; }
template <> __device__ __forceinline__ uint2 sel<uint2>(bool c, uint2 a, uint2 b) {
  return make_uint2(c ? a.x : b.x, c ? a.y : b.y);
}
template <> __device__ __forceinline__ uint4 sel<uint4>(bool c, uint4 a, uint4 b) {
  return make_uint4(c ? a.x : b.x, c ? a.y : b.y, c ? a.z : b.z, c ? a.w : b.w);
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128
// bit multiplications with the published multipliers and Weyl key increments.
struct Philox4 {
  uint64_t v[4];
};
__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = c0, x1 = c1, x2 = 0, x3 = 0;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t lo0 = M0 * x0, hi0 = __umul64hi(M0, x0);
    const uint64_t lo1 = M1 * x2, hi1 = __umul64hi(M1, x2);
    const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  Philox4 r;
  r.v[0] = x0;
  r.v[1] = x1;
  r.v[2] = x2;
  r.v[3] = x3;
  return r;
}

// Arguments of one routing pass (levels [level0, level0 + klev) of Algorithm 3.1).
struct PassArgs {
  const void* x_in;           // first pass: the n input records
  void* out;                  // last pass: n output records
  const void* rec_in;         // slot records of level level0 (not first pass)
  const uint32_t* tag_in;     // slot tags of level level0
  void* rec_out;              // slot records of level level0 + klev (not last pass)
  uint32_t* tag_out;
  unsigned long long* status; // first overflow: (level << 32) | pair, min over MergeSplits
  unsigned long long* scan;   // last pass: per-block look-back words
  uint32_t* ticket;           // last pass: dynamic block index counter
  uint64_t n;
  uint64_t buckets;           // B
  uint64_t seed;
  uint32_t z, lz;             // Z and log2 Z
  uint32_t levels;            // L
  uint32_t level0, klev;      // first level of this pass, levels in this pass
  uint32_t attempt;
  uint32_t fin;               // fused last pass: 0 = random permutation of each bin, 1 = sort each bin
  uint32_t pad;
  uint32_t* loads;            // split last pass: real count of every final bin
  // Staged (out-of-core) launches run a chunk of the pass's blocks on copies
  // of its slots; all zero otherwise.  Blocks keep their global index
  // (item_off + launch index) for labels, overflow pairs and bins.
  uint32_t item_off;          // global index of the launch's first block
  uint32_t staged;            // 1: rec_in/tag_in hold the chunk's input segments (in_h0, in_r0, in_lseg)
  uint64_t in_h0, in_r0;      // the chunk's first group h and (for a chunk inside one group) first r
  uint32_t in_lseg, pad2;     // log2 of the buckets per staged input segment
  uint64_t x_off;             // first pass: global index of the first staged input record
  uint64_t out_slot0;         // global index of the first staged output slot (rec_out, tag_out)
};

// One instance of a batched comparison-sort launch (tile sort or merge pass).
struct SortSeg {
  void* src;         // tile sort: the buffer sorted in place; merge pass: source runs
  void* dst;         // merge pass: destination; tile sort: the first four-way pass's samples (or null)
  uint64_t n;        // records of the instance
  uint64_t w;        // merge pass: run width
  uint64_t* split;   // merge pass: this instance's split array
  uint32_t first;    // first block (and first partition thread) of the segment in the launch
  uint32_t count;    // blocks of the instance in the launch (tiles of the tile sort or merge)
};

// One instance of a batched four-way merge pass (two merge levels in one HBM
// pass).  Launch k of the pass (0 sample gather, 1 per-sample ranks,
// 2 workgroup-wide ranks, 3 tile starts, 4 tile merges) gives the instance
// its blocks first[k] .. first[k] + count - 1 (count 0: not in that launch).
struct M4Seg {
  const void* src;            // runs of width 2^lw
  void* dst;
  void* smp;                  // samples of src (every 2^kSmpLog-th record)
  void* next_smp;             // the next pass's samples, written by the tiles (null: none)
  uint64_t* spl;              // sample ranks, then tile starts
  unsigned long long* err;    // the instance's comparison-sort error word
  uint64_t n, ntf, ng, ntl, total;  // records; tiles per full group, groups, tiles of the last group, all tiles
  uint32_t lw, pad;
  uint32_t first[5];
  uint32_t pad2;
};

// One instance of a batched scan + strip after a split last pass.
struct StripSeg {
  const void* binned;            // bin gb's reals in slots gb*Z .. (the last pass's rec_out)
  const uint32_t* loads;         // real count per bin
  unsigned long long* bsum;      // real count per routing block; scanned in place
  void* out;
  uint64_t n;
  uint32_t nblocks, klev, lz;
  uint32_t first;                // first strip workgroup of the segment in the launch
  uint32_t tile;                 // records per tile of the comparison sort's first phase
  uint32_t pad;
};

// Per-bin finish of bos_orp after a split last pass.
struct FinishArgs {
  const void* binned;               // bin gb's reals in slots gb*Z .. gb*Z + loads[gb] - 1
  const uint32_t* loads;            // real count per bin
  const unsigned long long* boff;   // exclusive scan of the block counts within 1024-block chunks
  const unsigned long long* coff;   // offset of every chunk of 1024 blocks
  void* out;                        // n output records
  uint64_t n;
  uint64_t nbins;                   // B
  uint64_t seed;
  uint32_t klev;                    // levels of the last pass: a block holds 2^klev bins
  uint32_t attempt;
  unsigned long long* tie;          // raised when a bin's random keys tie (cleared before the finish)
  // Staged (out-of-core) launches finish bins [gb_lo, gb_hi) from a copy of
  // their slots (binned index minus bin_slot0) into a copy of their output
  // range (out index minus out0); 0, 0, nbins, 0 otherwise.
  uint64_t gb_lo, gb_hi, bin_slot0, out0;
};

// One instance's status words to initialise before its first routing pass.
struct FillSeg {
  unsigned long long* p;  // status word, ticket, look-back words (or an error word)
  uint32_t count;
  uint32_t zero_first;    // 1: p[0] = 0 too (an error word), else p[0] = no overflow
};

// ---- address digests (test build) ------------------------------------------
//
// Built with BOS_TRACE_DIGEST, every HBM and LDS access of the routing, the
// per-bin finish, the strip (trace buffer 0) and the comparison sort (trace
// buffer 1) folds (array class, index) into a 64-bit slot of its thread, in
// program order: slot[g] = mix(slot[g], class, index), g = the thread's
// global index in its launch (modulo the buffer's slot count).  Two runs
// leave equal buffers when every thread of every launch touched the same
// arrays at the same indices in the same order, which is what a data-
// independent access pattern means (Definition 2.1) at the granularity of
// array elements.  The normal build compiles every hook to nothing.
//
// Device code reads the buffers through a file-scope pointer pair of its own
// translation unit, which the host sets (trace_bind) before each launch when
// bos_trace_bind has changed them.
struct TraceHost {
  void* buf[2];
  uint64_t slots;
  uint64_t gen;
};
extern TraceHost g_trace;  // host side, defined in bos_api.hip

#ifdef BOS_TRACE_DIGEST
static __device__ unsigned long long* bos_trace_buf[2];
static __device__ uint64_t bos_trace_mask;
[[maybe_unused]] static uint64_t g_trace_bound = 0;  // host: the generation this translation unit was bound to

__device__ __forceinline__ void trace_idx(uint32_t which, uint32_t cls, uint64_t idx) {
  unsigned long long* b = bos_trace_buf[which];
  if (!b) return;
  const uint64_t g = (uint64_t(blockIdx.x) * blockDim.x + threadIdx.x) & bos_trace_mask;
  uint64_t h = b[g];
  h ^= idx + (uint64_t(cls) << 56) + 0x9E3779B97F4A7C15ull;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 31;
  h *= 0x94D049BB133111EBull;
  h ^= h >> 29;
  b[g] = h;
}

[[maybe_unused]] static inline hipError_t trace_bind() {
  if (g_trace_bound == g_trace.gen) return hipSuccess;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(bos_trace_buf), g_trace.buf, sizeof(g_trace.buf));
  const uint64_t mask = g_trace.slots ? g_trace.slots - 1 : 0;
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(bos_trace_mask), &mask, sizeof(mask));
  if (e == hipSuccess) g_trace_bound = g_trace.gen;
  return e;
}
#define BOS_TR(which, cls, idx) ::bos::trace_idx((which), (cls), uint64_t(idx))
#define BOS_TRACE_BIND()                             \
  do {                                               \
    const hipError_t te_ = ::bos::trace_bind();      \
    if (te_ != hipSuccess) return te_;               \
  } while (0)
#else
#define BOS_TR(which, cls, idx) ((void)0)
#define BOS_TRACE_BIND() ((void)0)
#endif

// Dynamic LDS bytes of a routing block (must match the carve in the kernel).
// LDS bytes per slot of a routing pass's records.  At 64 <= Z <= 512 records
// go through LDS in two halves (the second after the first has been read),
// so a block needs half a record and a tag of LDS per slot; the fused last
// pass keeps whole records (its per-bin sorts hold them in LDS).
__host__ __device__ constexpr uint32_t lds_rec_bytes(int rec, uint32_t z, bool fused) {
  return (z >= 64 && z <= 512 && !fused) ? uint32_t(rec) / 2u : uint32_t(rec);
}

__host__ __device__ inline uint32_t pass_lds_bytes(int rec, uint32_t z, uint32_t klev, bool last_shuffle,
                                                   bool fused) {
  const uint32_t m = z << klev;
  const uint32_t mp = m + (m >> 4);
  uint32_t b = mp * lds_rec_bytes(rec, z, fused) + mp * 4u + (m >> 4) * 4u + (1u << klev) * 12u + 64u * 4u + 64u;
  if (last_shuffle) b += mp * 4u + mp * 2u;
  return (b + 15u) & ~15u;
}

}  // namespace bos
