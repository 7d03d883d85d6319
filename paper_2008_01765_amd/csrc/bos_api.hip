// bos_api.hip — planner, launch sequencing and the C ABI of libbos (include/bos.h).
//
// Planner (Algorithm 3.1): B = smallest power of two >= 2n/Z, L = log2 B; the
// L levels are cut into passes of at most k levels (k fused levels = 2^k
// buckets per block, bounded by LDS); the workspace holds two slot arrays
// (records + 4-byte tags, ping-pong), the overflow status word and the
// look-back words of the strip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "bos.h"
#include "bos_common.h"
#include "bos_prof.h"

namespace bos {
hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s);
hipError_t launch_labels(uint32_t* out, uint64_t n, uint32_t L, uint64_t seed, uint32_t attempt, hipStream_t s);
hipError_t launch_pass(int rec, const PassArgs& a, bool first, bool last, uint32_t nblocks, hipStream_t s);
hipError_t launch_route(int rec, const PassArgs& a, bool first, bool last, uint32_t nitems, uint32_t grid,
                        hipStream_t s, bool split);
hipError_t launch_strip(int rec, const void* binned, const uint32_t* loads, unsigned long long* bsum,
                        unsigned long long* coff, void* out, uint64_t n, uint32_t nblocks, uint32_t klev, uint32_t lz,
                        uint32_t tile, hipStream_t s);
constexpr uint32_t kScanChunk = 1024;  // block counts per workgroup of the strip's first scan
hipError_t launch_comparison_sort(int rec, void* buf0, void* buf1, uint64_t n, uint32_t ts, uint64_t* split,
                                  hipStream_t s, void** result, bool multiway);
uint32_t comparison_sort_hbm_passes(int rec, uint64_t n, uint32_t ts, bool multiway);
size_t comparison_sort_split_bytes(uint64_t n, int rec);
unsigned long long* comparison_sort_err_word(uint64_t* split, uint64_t n, int rec);
hipError_t launch_route_batched(int rec, uint32_t lz, bool first, bool last, const PassArgs* segs,
                                const uint32_t* blk_start, uint32_t nsegs, uint32_t blocks, uint32_t threads,
                                uint32_t lds, hipStream_t s, bool split);
hipError_t launch_strip_batched(int rec, const StripSeg* segs, uint32_t nsegs, uint32_t blocks, hipStream_t s);
hipError_t launch_block_scan(unsigned long long* bsum, unsigned long long* coff, uint32_t nblocks, hipStream_t s);
hipError_t launch_strip_staged(int rec, const void* binned, const uint32_t* loads, const unsigned long long* bsum,
                               const unsigned long long* coff, void* out, uint64_t n, uint32_t klev, uint32_t lz,
                               uint32_t tile, uint64_t blk0, uint32_t nblk, uint64_t bin_slot0, uint64_t out0,
                               hipStream_t s);
hipError_t launch_or_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s);
hipError_t launch_orp_finish(int rec, uint32_t lz, const FinishArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_sort_batched(int rec, int kind, uint32_t tile, const SortSeg* segs, uint32_t nsegs, uint32_t total,
                               hipStream_t s);
hipError_t launch_fill_status_batched(const FillSeg* segs, uint32_t nsegs, hipStream_t s);
bool sort_tile_ok(int rec, uint32_t t);
hipError_t launch_batch_status(unsigned long long* const* status, unsigned long long* const* err, uint32_t* out,
                               uint32_t count, hipStream_t s);
bool merge_pass_at(int rec, uint64_t n, uint32_t ts, uint32_t p, uint64_t* w_out, bool* four, bool* next_four);
void* first_pass_samples(int rec, uint64_t n, uint32_t ts, uint64_t* split);
void merge4_seg(int rec, const void* src, void* dst, uint64_t n, uint64_t* split, uint64_t w, bool gather,
                bool next_four, M4Seg* sg, uint32_t counts[5]);
hipError_t launch_merge4_batched(int rec, const M4Seg* segs, uint32_t nsegs, const uint32_t totals[5],
                                 hipStream_t s);
uint32_t bitonic_tile(int rec);
hipError_t launch_bitonic(int rec, const void* in, void* out, uint64_t n, void* ws, uint64_t N,
                          hipStream_t s);
}  // namespace bos

namespace {

struct ProfRec {
  uint32_t kind, index;
  uint64_t bytes;
  hipEvent_t start, stop;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;
ProfRec g_prof_open;
bool g_prof_pending = false;

hipEvent_t prof_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace bos {
TraceHost g_trace = {{nullptr, nullptr}, 0, 0};

void prof_begin(uint32_t kind, uint32_t index, uint64_t bytes, hipStream_t s) {
  if (!g_prof_on) return;
  g_prof_open.kind = kind;
  g_prof_open.index = index;
  g_prof_open.bytes = bytes;
  g_prof_open.start = prof_event();
  g_prof_open.stop = prof_event();
  g_prof_pending = g_prof_open.start && g_prof_open.stop;
  if (g_prof_pending) (void)hipEventRecord(g_prof_open.start, s);
}
void prof_end(hipStream_t s) {
  if (!g_prof_on || !g_prof_pending) return;
  (void)hipEventRecord(g_prof_open.stop, s);
  g_prof.push_back(g_prof_open);
  g_prof_pending = false;
}
}  // namespace bos

namespace {

using namespace bos;

constexpr uint64_t kMaxN = 1ull << 31;
constexpr uint32_t kMaxPasses = 32;
constexpr uint32_t kDefaultTile = 4096;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  uint64_t n = 0, B = 1;
  int rec = 8;
  uint32_t Z = 512, lz = 9, L = 0, P = 1, k = 0, tile = kDefaultTile;
  uint32_t klev[kMaxPasses] = {0}, lev0[kMaxPasses] = {0};
  size_t off_rec[2] = {0, 0}, off_tag[2] = {0, 0}, off_status = 0, off_split = 0, off_loads = 0, off_coff = 0;
  size_t total = 0;
  uint32_t nblocks_last = 1;
  bool generic = false;
};

uint32_t g_lds_max = 0;

uint32_t lds_max() {
  if (g_lds_max == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      g_lds_max = uint32_t(v);
    else
      g_lds_max = 64 * 1024;
  }
  return g_lds_max;
}

void fill_defaults(bos_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->z = 512;
  p->max_retries = 3;
  p->min_security_bits = 80;
  p->flags = BOS_SYNC;
}

bos_params resolve(const bos_params* p) {
  bos_params q;
  if (p) {
    q = *p;
  } else {
    fill_defaults(&q);
  }
  return q;
}

// ---- tuning table: (record size, size class) -> Z, k, tile -----------------
// Filled by bos_set_tuning (the autotuner); consulted by make_plan wherever
// the caller leaves z, k or tile at 0.
std::mutex g_tune_mu;
std::vector<bos_tune_entry> g_tune;
uint64_t g_tune_gen = 0;  // bumped by every bos_set_tuning

uint32_t size_class(uint64_t n) {
  uint32_t c = 0;
  while (c < 63 && (1ull << c) < n) ++c;
  return c;
}

// The entry for this record size whose size class is nearest to n's (the
// smaller class on a tie).
bool tuned_for(uint64_t n, int rec, bos_tune_entry* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const int64_t c = size_class(n);
  const bos_tune_entry* best = nullptr;
  int64_t bd = 0;
  for (const bos_tune_entry& e : g_tune) {
    if (int(e.rec) != rec) continue;
    const int64_t d = int64_t(e.log2n) - c, ad = d < 0 ? -d : d;
    if (!best || ad < bd || (ad == bd && e.log2n < best->log2n)) {
      best = &e;
      bd = ad;
    }
  }
  if (!best) return false;
  *out = *best;
  return true;
}

// Largest k such that a block of 2^k buckets fits in LDS and in 512 threads.
// Most levels per pass whose block fits a workgroup and its LDS (full_rec:
// whole records in LDS, as in the fused last pass and the generic kernel).
uint32_t max_klev(int rec, uint32_t z, bool last_shuffle, bool full_rec) {
  uint32_t best = 0;
  for (uint32_t k = 1; k <= 12; ++k) {
    const uint64_t m = uint64_t(z) << k;
    if (m / 16 > uint64_t(kMaxThreads)) break;
    if (pass_lds_bytes(rec, z, k, last_shuffle, full_rec) > lds_max()) break;
    best = k;
  }
  return best;
}


// Lemma 3.2: overflow probability <= B log2 B e^(-Z/6) (B = 2^L)
bool insecure(uint32_t L, uint32_t Z, uint32_t bits) {
  if (!bits || L == 0) return false;
  const double log2eps = double(L) + std::log2(double(L)) - double(Z) / (6.0 * std::log(2.0));
  return log2eps > -double(bits);
}

uint32_t levels_for(uint64_t n, uint32_t Z, uint64_t* B_out) {
  uint64_t B = 1;
  uint32_t L = 0;
  while (B * Z < 2 * n) {
    B *= 2;
    ++L;
  }
  *B_out = B;
  return L;
}

bos_status make_plan(uint64_t n, int rec, const bos_params& q, bool shuffle_last, Plan* pl, uint64_t max_n = kMaxN) {
  if (rec != 8 && rec != 16) return BOS_ERR_INVALID_ARG;
  if (n > max_n) return BOS_ERR_INVALID_ARG;
  bos_tune_entry te;
  std::memset(&te, 0, sizeof(te));
  const bool tuned = (q.z == 0 || q.k == 0 || q.tile == 0) && tuned_for(n, rec, &te);
  uint32_t Z = q.z ? q.z : (tuned && te.z ? te.z : 512u);
  if (Z < 2 || (Z & (Z - 1))) return BOS_ERR_INVALID_ARG;
  // the kernels hold 16 slots per lane and draw per-bin keys four at a
  // time: Z in [8, 2048] (Z = 2 or 4 fails Lemma 3.2's bound at any n > 1)
  if (Z < 8 || Z > 2048) return BOS_ERR_UNSUPPORTED;
  uint64_t B = 1;
  uint32_t L = levels_for(n, Z, &B);
  if (q.z == 0) {
    // a tuned Z below the caller's security floor gives way to a larger one
    while (insecure(L, Z, q.min_security_bits) && Z < 2048) {
      Z *= 2;
      L = levels_for(n, Z, &B);
    }
  }
  if (L > 31) return BOS_ERR_INVALID_ARG;
  if (insecure(L, Z, q.min_security_bits)) return BOS_ERR_INSECURE_Z;
  pl->n = n;
  pl->rec = rec;
  pl->Z = Z;
  pl->generic = (q.flags & BOS_GENERIC_ROUTING) != 0;
  pl->lz = 0;
  while ((1u << pl->lz) < Z) ++pl->lz;
  pl->B = B;
  pl->L = L;
  // the last pass is sized as the fused form (whole records in LDS)
  const uint32_t kmid = max_klev(rec, Z, false, pl->generic), klast = max_klev(rec, Z, shuffle_last, true);
  if (kmid == 0 || klast == 0) return BOS_ERR_UNSUPPORTED;
  // default: 3 levels per pass (a block of 2^3 Z slots leaves LDS for three
  // workgroups per CU at Z = 512, which outruns fewer, larger passes)
  // An explicit k must fit a block of 2^k buckets in LDS and in one
  // workgroup; the tuned or default k is capped at what fits.
  if (q.k > 12) return BOS_ERR_INVALID_ARG;
  if (q.k > kmid) return BOS_ERR_UNSUPPORTED;
  // strict mode (Section 4.1's client of O(1) buckets): one level per pass,
  // so a workgroup holds one MergeSplit's 2Z slots and nothing across levels
  const bool strict = (q.flags & BOS_STRICT) != 0;
  if (strict && q.k > 1) return BOS_ERR_INVALID_ARG;
  const uint32_t kreq = strict ? 1u : q.k ? q.k : (tuned && te.k && te.z == Z ? te.k : 3u);
  const uint32_t k = std::min(kreq, kmid);
  pl->k = k;
  pl->tile = q.tile ? q.tile : (tuned && te.tile ? te.tile : kDefaultTile);
  if (!sort_tile_ok(rec, pl->tile)) return BOS_ERR_INVALID_ARG;
  if (L == 0) {
    pl->P = 1;
    pl->klev[0] = 0;
    pl->lev0[0] = 0;
  } else {
    // fewest passes of at most k levels, balanced; the larger passes go last
    // (the last pass, whose per-bin finish is amortized over its bins, gets
    // as many levels as it may)
    uint32_t P = (L + k - 1) / k;
    for (;; ++P) {
      if (P > kMaxPasses) return BOS_ERR_UNSUPPORTED;
      const uint32_t base = L / P, extra = L % P;
      if (base == 0) return BOS_ERR_UNSUPPORTED;
      if (base + (extra ? 1u : 0u) > k) continue;
      const bool big_last = extra > 0 && base + 1 <= klast;
      if (!big_last && base > klast) continue;
      uint32_t lv = 0;
      for (uint32_t t = 0; t < P; ++t) {
        const bool big = big_last ? (t >= P - extra) : (t < extra);
        pl->klev[t] = base + (big ? 1u : 0u);
        pl->lev0[t] = lv;
        lv += pl->klev[t];
      }
      pl->P = P;
      break;
    }
  }
  pl->nblocks_last = uint32_t(B >> pl->klev[pl->P - 1]);
  const size_t slots = size_t(B) * Z;
  size_t off = 0;
  for (int t = 0; t < 2; ++t) {
    pl->off_rec[t] = off;
    off = align_up(off + slots * rec);
  }
  for (int t = 0; t < 2; ++t) {
    pl->off_tag[t] = off;
    off = align_up(off + slots * 4);
  }
  pl->off_status = off;  // status word, ticket, then look-back words
  off = align_up(off + 16 + size_t(pl->nblocks_last) * 8);
  pl->off_split = off;   // merge-path splits of the comparison sort
  off = align_up(off + comparison_sort_split_bytes(n, rec));
  pl->off_loads = off;   // split last pass: real count of every final bin
  off = align_up(off + size_t(B) * 4);
  pl->off_coff = off;    // split last pass: offset of every chunk of kScanChunk block counts,
                         // then bos_orp's key-tie flag
  off = align_up(off + (size_t(pl->nblocks_last) / kScanChunk + 2) * 8);
  pl->total = off;
  return BOS_OK;
}

uint64_t routing_bytes(const Plan& pl) {
  // first pass reads n records and writes B*Z slots; middle passes read and
  // write B*Z slots; the last reads B*Z slots and writes n records.
  const uint64_t slot = uint64_t(pl.rec) + 4, bz = pl.B * pl.Z;
  if (pl.P == 1) return 2 * pl.n * pl.rec;
  return 2 * pl.n * pl.rec + 2 * bz * slot * (pl.P - 1);
}

bos_status hip_status(hipError_t e) { return e == hipSuccess ? BOS_OK : BOS_ERR_HIP; }

// Plans of the step engine, which re-plans every resident job on every step:
// memoised on everything make_plan reads (size, record, the parameters it
// uses and the tuning table's generation).
struct PlanKey {
  uint64_t n, gen;
  uint32_t rec, z, k, tile, bits, flags;
  bool operator==(const PlanKey& o) const {
    return n == o.n && gen == o.gen && rec == o.rec && z == o.z && k == o.k && tile == o.tile && bits == o.bits &&
           flags == o.flags;
  }
};
struct PlanKeyHash {
  size_t operator()(const PlanKey& x) const {
    uint64_t h = x.n * 0x9E3779B97F4A7C15ull ^ x.gen;
    for (uint32_t v : {x.rec, x.z, x.k, x.tile, x.bits, x.flags}) h = (h ^ v) * 0x100000001B3ull;
    return size_t(h ^ (h >> 29));
  }
};
std::mutex g_plan_mu;
std::unordered_map<PlanKey, std::pair<bos_status, Plan>, PlanKeyHash> g_plans;

bos_status make_plan_cached(uint64_t n, int rec, const bos_params& q, Plan* pl) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    gen = g_tune_gen;
  }
  const PlanKey key{n, gen, uint32_t(rec), q.z, q.k, q.tile, q.min_security_bits, q.flags};
  {
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
      *pl = it->second.second;
      return it->second.first;
    }
  }
  const bos_status st = make_plan(n, rec, q, true, pl);
  std::lock_guard<std::mutex> lock(g_plan_mu);
  if (g_plans.size() >= 4096) g_plans.clear();  // bounded: a server sees a limited set of sizes at a time
  g_plans.emplace(key, std::make_pair(st, *pl));
  return st;
}

uint32_t g_num_cus = 0;
uint32_t num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      g_num_cus = uint32_t(v);
    else
      g_num_cus = 256;
  }
  return g_num_cus;
}

// The register-resident routing kernel covers Z in [16, 2048] with at least one
// level per pass; Z = 8 and the single-bin case (L = 0) use the generic kernel,
// as does every pass when the caller sets BOS_GENERIC_ROUTING.
bool use_route_kernel(const Plan& pl, uint32_t t) {
  return !pl.generic && pl.lz >= 4 && pl.lz <= 11 && pl.klev[t] >= 1;
}

// The split form of the last pass (a last pass that leaves the compacted bins
// in slot array (P + 1) & 1, then scan + strip, which sorts the bins that
// straddle a tile of the comparison sort) applies to sorting plans of two or
// more passes routed by the register-resident kernel.
bool split_last(const Plan& pl) { return pl.P >= 2 && pl.L > 0 && use_route_kernel(pl, pl.P - 1); }

// Where a sort's comparison phase ping-pongs besides `out`: with the split
// last pass, the two tag arrays (2 B Z 4 >= n R bytes; the bins sit in slot
// array (P + 1) & 1 until the strip); otherwise slot array (P + 1) & 1 itself
// (the fused last pass reads slot array P & 1 and writes `out` directly).
char* sort_tmp(const Plan& pl, char* ws) {
  return ws + (split_last(pl) ? pl.off_tag[0] : pl.off_rec[(pl.P + 1) & 1]);
}

// One instance's entry of a batched strip after its split last pass.
StripSeg strip_seg(const Plan& pl, char* ws, void* out, uint32_t first) {
  const uint32_t t = pl.P - 1;
  StripSeg g;
  std::memset(&g, 0, sizeof(g));
  g.binned = ws + pl.off_rec[t & 1];
  g.loads = reinterpret_cast<const uint32_t*>(ws + pl.off_loads);
  g.bsum = reinterpret_cast<unsigned long long*>(ws + pl.off_status) + 2;
  g.out = out;
  g.n = pl.n;
  g.nblocks = pl.nblocks_last;
  g.klev = pl.klev[t];
  g.lz = pl.lz;
  g.first = first;
  g.tile = pl.tile;
  return g;
}

// Enqueue one attempt of the routing phase; `out` receives the stripped bins.
// split: last pass in split form (requires split_last(pl); `out` must not be
// slot array (P + 1) & 1, which holds the bins until the strip).
hipError_t enqueue_routing(const Plan& pl, const void* in, void* out, uint64_t seed, uint32_t attempt,
                           uint32_t fin, char* ws, hipStream_t s, int stop_after = -1, bool split = false,
                           uint32_t flags = 0) {
  unsigned long long* status = reinterpret_cast<unsigned long long*>(ws + pl.off_status);
  hipError_t e = launch_fill_u64(status, 2 + pl.nblocks_last, 0, s);
  if (e != hipSuccess) return e;
  e = launch_fill_u64(status, 1, kNoOverflow, s);
  if (e != hipSuccess) return e;
  for (uint32_t t = 0; t < pl.P; ++t) {
    if (stop_after >= 0 && int(t) > stop_after) break;
    PassArgs a;
    std::memset(&a, 0, sizeof(a));
    const bool first = t == 0, last = t + 1 == pl.P && stop_after < 0;
    a.x_in = in;
    a.out = out;
    a.rec_in = ws + pl.off_rec[(t + 1) & 1];
    a.tag_in = reinterpret_cast<const uint32_t*>(ws + pl.off_tag[(t + 1) & 1]);
    a.rec_out = ws + pl.off_rec[t & 1];
    a.tag_out = reinterpret_cast<uint32_t*>(ws + pl.off_tag[t & 1]);
    a.status = status;
    a.ticket = reinterpret_cast<uint32_t*>(status + 1);
    a.scan = status + 2;
    a.n = pl.n;
    a.buckets = pl.B;
    a.seed = seed;
    a.z = pl.Z;
    a.lz = pl.lz;
    a.levels = pl.L;
    a.level0 = pl.lev0[t];
    a.klev = pl.klev[t];
    a.attempt = attempt;
    const bool split_pass = split && last;
    // the split last pass compacts every bin whatever the finish; the fused
    // one permutes (fin 0) or sorts (fin 1) its bins itself
    a.fin = split_pass ? 1u : fin;
    if (split_pass) a.loads = reinterpret_cast<uint32_t*>(ws + pl.off_loads);
    const uint64_t slot_bytes = pl.B * pl.Z * (uint64_t(pl.rec) + 4), rec_bytes = pl.n * pl.rec;
    const uint32_t kind = first && last ? BOS_K_ROUTE_SINGLE
                          : first       ? BOS_K_ROUTE_FIRST
                          : last        ? BOS_K_ROUTE_LAST
                                        : BOS_K_ROUTE_MID;
    const uint64_t bytes = (first ? rec_bytes : slot_bytes) + (last ? rec_bytes : slot_bytes);
    prof_begin(kind, t, bytes, s);
    const uint32_t nitems = uint32_t(pl.B >> pl.klev[t]);
    if (use_route_kernel(pl, t))
      e = launch_route(pl.rec, a, first, last, nitems, num_cus(), s, split_pass);
    else
      e = launch_pass(pl.rec, a, first, last, nitems, s);
    prof_end(s);
    if (e != hipSuccess) return e;
    if (split_pass && fin != 0) {
      prof_begin(BOS_K_STRIP, 0, 2 * rec_bytes, s);
      e = launch_strip(pl.rec, a.rec_out, a.loads, a.scan, reinterpret_cast<unsigned long long*>(ws + pl.off_coff),
                       out, pl.n, nitems, pl.klev[t], pl.lz, pl.tile, s);
      prof_end(s);
      if (e != hipSuccess) return e;
    } else if (split_pass) {
      // bos_orp: scan of the block counts, then the per-bin permutation and
      // strip (Section 3.2)
      unsigned long long* coff = reinterpret_cast<unsigned long long*>(ws + pl.off_coff);
      unsigned long long* tie = coff + nitems / kScanChunk + 1;
      prof_begin(BOS_K_ORP_FINISH, 0, 2 * rec_bytes, s);
      e = launch_fill_u64(tie, 1, (flags & BOS_EXACT_FINISH) ? 1ull : 0ull, s);
      if (e == hipSuccess) e = launch_block_scan(a.scan, coff, nitems, s);
      if (e == hipSuccess) {
        FinishArgs f;
        std::memset(&f, 0, sizeof(f));
        f.binned = a.rec_out;
        f.loads = a.loads;
        f.boff = a.scan;
        f.coff = coff;
        f.out = out;
        f.n = pl.n;
        f.nbins = pl.B;
        f.seed = seed;
        f.klev = pl.klev[t];
        f.attempt = attempt;
        f.tie = tie;
        e = launch_orp_finish(pl.rec, pl.lz, f, num_cus(), s);
      }
      prof_end(s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

void fill_report(bos_report* rep, const Plan& pl, uint32_t attempts, uint64_t ovf, uint64_t extra_bytes) {
  if (!rep) return;
  std::memset(rep, 0, sizeof(*rep));
  rep->attempts = attempts;
  rep->z = pl.Z;
  rep->k = pl.k;
  rep->tile = pl.tile;
  rep->levels = pl.L;
  rep->passes = pl.P;
  rep->buckets = pl.B;
  rep->first_overflow_level = ovf == kNoOverflow ? -1 : int32_t(ovf >> 32);
  rep->first_overflow_pair = ovf == kNoOverflow ? -1 : int64_t(ovf & 0xFFFFFFFFull);
  rep->algorithmic_bytes = routing_bytes(pl) + extra_bytes;
}

// Runs the routing phase with the retry loop; *attempts_out / *ovf_out report.
bos_status run_routing(const Plan& pl, const bos_params& q, const void* in, void* out, uint32_t fin, char* ws,
                       hipStream_t s, uint32_t* attempts_out, uint64_t* ovf_out, uint32_t first_attempt = 0,
                       uint64_t prev_ovf = kNoOverflow, bool split = false) {
  uint64_t last_ovf = prev_ovf;
  // with BOS_SYNC: attempts first_attempt .. max_retries (at least one);
  // without: first_attempt alone, its status left on the device
  const uint32_t last = (q.flags & BOS_SYNC) ? std::max(q.max_retries, first_attempt) : first_attempt;
  for (uint32_t att = first_attempt; att <= last; ++att) {
    hipError_t e = enqueue_routing(pl, in, out, q.seed, att, fin, ws, s, -1, split, q.flags);
    if (e != hipSuccess) return BOS_ERR_HIP;
    *attempts_out = att + 1;
    if (!(q.flags & BOS_SYNC)) {
      *ovf_out = kNoOverflow;
      return BOS_OK;
    }
    uint64_t st = 0;
    e = hipMemcpyAsync(&st, ws + pl.off_status, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return BOS_ERR_HIP;
    if (st == kNoOverflow) {
      *ovf_out = last_ovf;
      return BOS_OK;
    }
    last_ovf = st;
  }
  *ovf_out = last_ovf;
  return BOS_ERR_OVERFLOW;
}

bool has_gpu() {
  int c = 0;
  return hipGetDeviceCount(&c) == hipSuccess && c > 0;
}

// ---- batched engine -----------------------------------------------------
//
// bos_sort_batched plans every instance on its own (its own Z, k and tile when
// they come from the tuning table), gives each a workspace region, and runs
// all of them pass-major: one launch per routing pass index, pass kind
// (first / middle / last / single) and Z over a table of per-instance pass
// arguments, then one batched tile sort per tile size and one batched launch
// pair per merge pass.  The launch sequence is captured once into a hipGraph
// per batch shape (sizes, record type, plans, workspace) and replayed; the
// tables (pointers, seeds) are re-uploaded before every replay.

// Z values with batched routing kernels.
bool batched_lz(uint32_t lz) { return lz == 5 || lz == 8 || lz == 9 || lz == 10; }

// The comparison sort's error word and first four-way samples of a job whose
// workspace (plan pl) starts at w.
unsigned long long* err_word(const Plan& pl, char* w, uint64_t n) {
  return w ? comparison_sort_err_word(reinterpret_cast<uint64_t*>(w + pl.off_split), n, pl.rec) : nullptr;
}
void* split_smp(const Plan& pl, char* w, uint64_t n) {
  return w ? first_pass_samples(pl.rec, n, pl.tile, reinterpret_cast<uint64_t*>(w + pl.off_split)) : nullptr;
}

// Merge pass `pass` of several instances, launched together: two-way passes
// as one table of SortSeg, four-way passes as one table of M4Seg.
struct MergeRound {
  std::vector<SortSeg> two;
  std::vector<M4Seg> four;
  uint32_t two_tiles = 0, m4[5] = {0, 0, 0, 0, 0};
  void add(int rec, void* src, void* dst, uint64_t n, uint32_t tile, uint32_t pass, uint64_t* split) {
    uint64_t w = 0;
    bool f = false, nf = false;
    if (!merge_pass_at(rec, n, tile, pass, &w, &f, &nf)) return;
    if (!f) {
      const uint32_t mt = merge_tile_records(rec);
      const uint32_t c = uint32_t((n + mt - 1) / mt);
      two.push_back(SortSeg{src, dst, n, w, split, two_tiles, c});
      two_tiles += c;
      return;
    }
    // the samples exist unless a two-way pass came just before
    uint64_t pw = 0;
    bool pf = true, pnf = false;
    const bool gather = pass > 0 && merge_pass_at(rec, n, tile, pass - 1, &pw, &pf, &pnf) && !pf;
    M4Seg sg;
    uint32_t c[5];
    merge4_seg(rec, src, dst, n, split, w, gather, nf, &sg, c);
    for (int k = 0; k < 5; ++k) {
      sg.first[k] = m4[k];
      m4[k] += c[k];
    }
    four.push_back(sg);
  }
};

struct BatchJob {
  const void* in = nullptr;
  void* out = nullptr;
  uint64_t n = 0, seed = 0;
  Plan pl;
  char* ws = nullptr;
  void* start = nullptr;  // routing output (where the comparison sort starts)
  void* other = nullptr;
  uint32_t merges = 0;     // HBM passes of the comparison sort's merge phase (two- and four-way)
  bool special = false;   // routed on its own (single bin, or a Z without batched kernels)
  bool split = false;     // last pass in split form, then the batched strip
};

struct BLaunch {
  int kind = 0;  // 0 fill, 1 route, 2 tile sort, 3 two-way merge pass, 4 status, 5 plain routing of one job,
                 // 6 strip, 7 four-way merge pass
  int mode = 0;  // route: bit 0 first, bit 1 last, bit 2 split last pass
  uint32_t lz = 0;    // route: log2 Z of the launch
  uint32_t tile = 0;  // tile sort: records per tile
  uint32_t nsegs = 0, blocks = 0, threads = 0, lds = 0, total = 0, job = 0;
  uint32_t m4[5] = {0, 0, 0, 0, 0};  // four-way pass: blocks of each of its launches
  size_t tab = 0, aux = 0;
};

struct Batch {
  std::vector<BatchJob> jobs;
  std::vector<BLaunch> launches;
  std::vector<char> tables;
  size_t tab_base = 0;  // offset of the tables in the workspace
  size_t total = 0;
  bool batched = true;
  int rec = 8;
};

template <typename V>
size_t push_table(std::vector<char>& tab, const std::vector<V>& v) {
  size_t off = align_up(tab.size());
  tab.resize(off + v.size() * sizeof(V));
  if (!v.empty()) std::memcpy(tab.data() + off, v.data(), v.size() * sizeof(V));
  return off;
}

bos_status build_batch(const bos_instance* inst, const uint64_t* ns, uint32_t count, int rec, const bos_params& q,
                       char* ws, Batch* b) {
  b->jobs.assign(count, BatchJob());
  b->rec = rec;
  b->batched = !(q.flags & BOS_GENERIC_ROUTING);
  size_t off = 0;
  for (uint32_t i = 0; i < count; ++i) {
    BatchJob& j = b->jobs[i];
    j.n = ns[i];
    if (inst) {
      j.in = inst[i].in;
      j.out = inst[i].out;
      j.seed = inst[i].seed;
    }
    const bos_status st = make_plan(j.n, rec, q, true, &j.pl);
    if (st != BOS_OK) return st;
    j.ws = ws ? ws + off : nullptr;
    off = align_up(off + j.pl.total);
    j.merges = comparison_sort_hbm_passes(rec, j.n, j.pl.tile, true);
    char* tmp = j.ws ? sort_tmp(j.pl, j.ws) : nullptr;
    j.start = (j.merges % 2 == 0) ? j.out : static_cast<void*>(tmp);
    j.other = (j.merges % 2 == 0) ? static_cast<void*>(tmp) : j.out;
    j.special = j.pl.L == 0 || !use_route_kernel(j.pl, 0) || !batched_lz(j.pl.lz);
    j.split = split_last(j.pl);
  }
  b->tab_base = align_up(off);
  if (!b->batched) {
    b->total = b->tab_base;
    return BOS_OK;
  }
  std::vector<char>& tab = b->tables;
  tab.clear();
  auto dev = [&](size_t o) -> char* { return ws ? ws + b->tab_base + o : nullptr; };
  // 0. status words
  {
    std::vector<FillSeg> f;
    for (const BatchJob& j : b->jobs)
      if (j.n && !j.special)
        f.push_back(FillSeg{reinterpret_cast<unsigned long long*>(j.ws + j.pl.off_status), 2 + j.pl.nblocks_last, 0});
    // comparison-sort error words (set by a four-way tile that fails its bound checks)
    for (const BatchJob& j : b->jobs)
      if (j.n > 1) f.push_back(FillSeg{err_word(j.pl, j.ws, j.n), 1, 1});
    BLaunch l;
    l.kind = 0;
    l.nsegs = uint32_t(f.size());
    l.tab = push_table(tab, f);
    if (l.nsegs) b->launches.push_back(l);
  }
  // 1. routing passes, pass-major
  uint32_t maxP = 0;
  for (const BatchJob& j : b->jobs)
    if (j.n && !j.special) maxP = std::max(maxP, j.pl.P);
  for (uint32_t t = 0; t < maxP; ++t) {
    // one launch per (pass kind, Z, levels of the pass): every block of a
    // launch has the same LDS size, so none is held to a larger block's
    // occupancy.  Groups are keyed (kind rank, log2 Z, levels) and launched
    // in key order.
    struct Group {
      std::vector<PassArgs> segs;
      std::vector<uint32_t> starts;
      uint32_t blocks = 0, threads = 64, lds = 0;
      int mode = 0;
      uint32_t lz = 0;
    };
    std::map<uint32_t, Group> groups;
    for (const BatchJob& j : b->jobs) {
      if (!j.n || j.special || t >= j.pl.P) continue;
      const bool first = t == 0, last = t + 1 == j.pl.P;
      const int mode = (first ? 1 : 0) | (last ? 2 : 0) | (last && j.split ? 4 : 0);
      const uint32_t rank = mode == 3 ? 0u : mode == 1 ? 1u : mode == 0 ? 2u : mode == 2 ? 3u : 4u;
      const Plan& pl = j.pl;
      Group& g = groups[(rank * 16u + pl.lz) * 16u + pl.klev[t]];
      g.mode = mode;
      g.lz = pl.lz;
      PassArgs a;
      std::memset(&a, 0, sizeof(a));
      unsigned long long* status = reinterpret_cast<unsigned long long*>(j.ws + pl.off_status);
      a.x_in = j.in;
      a.out = j.start;
      a.rec_in = j.ws + pl.off_rec[(t + 1) & 1];
      a.tag_in = reinterpret_cast<const uint32_t*>(j.ws + pl.off_tag[(t + 1) & 1]);
      a.rec_out = j.ws + pl.off_rec[t & 1];
      a.tag_out = reinterpret_cast<uint32_t*>(j.ws + pl.off_tag[t & 1]);
      a.status = status;
      a.ticket = reinterpret_cast<uint32_t*>(status + 1);
      a.scan = status + 2;
      a.n = pl.n;
      a.buckets = pl.B;
      a.seed = j.seed;
      a.z = pl.Z;
      a.lz = pl.lz;
      a.levels = pl.L;
      a.level0 = pl.lev0[t];
      a.klev = pl.klev[t];
      a.attempt = 0;
      a.fin = 1;
      if (last && j.split) a.loads = reinterpret_cast<uint32_t*>(j.ws + pl.off_loads);
      g.segs.push_back(a);
      g.starts.push_back(g.blocks);
      g.blocks += uint32_t(pl.B >> pl.klev[t]);
      g.threads = std::max(g.threads, uint32_t((pl.Z << pl.klev[t]) >> 4));
      g.lds = std::max(g.lds, pass_lds_bytes(rec, pl.Z, pl.klev[t], false, (mode & 2) && !(mode & 4)));
    }
    for (const auto& kv : groups) {
      const Group& g = kv.second;
      BLaunch l;
      l.kind = 1;
      l.mode = g.mode;
      l.lz = g.lz;
      l.nsegs = uint32_t(g.segs.size());
      l.blocks = g.blocks;
      l.threads = g.threads;
      l.lds = g.lds;
      l.tab = push_table(tab, g.segs);
      l.aux = push_table(tab, g.starts);
      b->launches.push_back(l);
    }
  }
  {
    // strip after the split last passes (all of them are done by now)
    std::vector<StripSeg> f;
    uint32_t blocks = 0;
    for (const BatchJob& j : b->jobs)
      if (j.n && !j.special && j.split) {
        f.push_back(strip_seg(j.pl, j.ws, j.start, blocks));
        blocks += j.pl.nblocks_last;
      }
    BLaunch l;
    l.kind = 6;
    l.nsegs = uint32_t(f.size());
    l.blocks = blocks;
    l.tab = push_table(tab, f);
    if (l.nsegs) b->launches.push_back(l);
  }
  for (uint32_t i = 0; i < count; ++i)
    if (b->jobs[i].n && b->jobs[i].special) {
      BLaunch l;
      l.kind = 5;
      l.job = i;
      b->launches.push_back(l);
    }
  // 2. tile sort, one launch per tile size
  for (uint32_t T : {16384u, 8192u, 4096u, 2048u, 1024u}) {
    std::vector<SortSeg> segs;
    uint32_t tiles = 0;
    for (const BatchJob& j : b->jobs) {
      if (j.n <= 1 || j.pl.tile != T) continue;
      const uint32_t c = uint32_t((j.n + T - 1) / T);
      segs.push_back(SortSeg{j.start, split_smp(j.pl, j.ws, j.n), j.n, 0, nullptr, tiles, c});
      tiles += c;
    }
    BLaunch l;
    l.kind = 2;
    l.tile = T;
    l.nsegs = uint32_t(segs.size());
    l.total = tiles;
    l.tab = push_table(tab, segs);
    if (l.nsegs) b->launches.push_back(l);
  }
  // 3. merge passes, pass-major: pass p of every instance that has one, as a
  //    two-way pass (merge tiles of merge_tile_records(rec) outputs) or a
  //    four-way pass (two merge levels)
  uint32_t maxM = 0;
  for (const BatchJob& j : b->jobs) maxM = std::max(maxM, j.merges);
  for (uint32_t pass = 0; pass < maxM; ++pass) {
    MergeRound mr;
    for (const BatchJob& j : b->jobs) {
      if (pass >= j.merges) continue;
      void* src = (pass % 2 == 0) ? j.start : j.other;
      void* dst = (pass % 2 == 0) ? j.other : j.start;
      mr.add(rec, src, dst, j.n, j.pl.tile, pass, reinterpret_cast<uint64_t*>(j.ws + j.pl.off_split));
    }
    if (!mr.two.empty()) {
      BLaunch l;
      l.kind = 3;
      l.nsegs = uint32_t(mr.two.size());
      l.total = mr.two_tiles;
      l.tab = push_table(tab, mr.two);
      b->launches.push_back(l);
    }
    if (!mr.four.empty()) {
      BLaunch l;
      l.kind = 7;
      l.nsegs = uint32_t(mr.four.size());
      std::memcpy(l.m4, mr.m4, sizeof(l.m4));
      l.tab = push_table(tab, mr.four);
      b->launches.push_back(l);
    }
  }
  // 4. per-instance status (overflow, then the comparison sort's error word)
  {
    std::vector<unsigned long long*> st, er;
    for (const BatchJob& j : b->jobs) {
      st.push_back(j.n ? reinterpret_cast<unsigned long long*>(j.ws + j.pl.off_status) : nullptr);
      er.push_back(j.n > 1 ? err_word(j.pl, j.ws, j.n) : nullptr);
    }
    BLaunch l;
    l.kind = 4;
    l.nsegs = count;
    l.tab = push_table(tab, st);
    l.aux = push_table(tab, er);
    b->launches.push_back(l);
  }
  (void)dev;
  b->total = b->tab_base + align_up(tab.size());
  return BOS_OK;
}

hipError_t enqueue_batch(const Batch& b, char* tables, hipStream_t s, uint32_t* d_status) {
  for (const BLaunch& l : b.launches) {
    hipError_t e = hipSuccess;
    switch (l.kind) {
      case 0:
        e = launch_fill_status_batched(reinterpret_cast<const FillSeg*>(tables + l.tab), l.nsegs, s);
        break;
      case 1:
        e = launch_route_batched(b.rec, l.lz, (l.mode & 1) != 0, (l.mode & 2) != 0,
                                 reinterpret_cast<const PassArgs*>(tables + l.tab),
                                 reinterpret_cast<const uint32_t*>(tables + l.aux), l.nsegs, l.blocks, l.threads,
                                 l.lds, s, (l.mode & 4) != 0);
        break;
      case 2:
        e = launch_sort_batched(b.rec, 0, l.tile, reinterpret_cast<const SortSeg*>(tables + l.tab), l.nsegs, l.total,
                                s);
        break;
      case 3:
        e = launch_sort_batched(b.rec, 1, 0, reinterpret_cast<const SortSeg*>(tables + l.tab), l.nsegs, l.total, s);
        if (e == hipSuccess)
          e = launch_sort_batched(b.rec, 2, 0, reinterpret_cast<const SortSeg*>(tables + l.tab), l.nsegs, l.total,
                                  s);
        break;
      case 4:
        e = launch_batch_status(reinterpret_cast<unsigned long long* const*>(tables + l.tab),
                                reinterpret_cast<unsigned long long* const*>(tables + l.aux), d_status, l.nsegs, s);
        break;
      case 7:
        e = launch_merge4_batched(b.rec, reinterpret_cast<const M4Seg*>(tables + l.tab), l.nsegs, l.m4, s);
        break;
      case 5: {
        const BatchJob& j = b.jobs[l.job];
        e = enqueue_routing(j.pl, j.in, j.start, j.seed, 0, 1, j.ws, s, -1, j.split);
        break;
      }
      case 6:
        e = launch_strip_batched(b.rec, reinterpret_cast<const StripSeg*>(tables + l.tab), l.nsegs, l.blocks, s);
        break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  char* pinned = nullptr;          // pinned host copy of the tables, uploaded before each replay
  size_t pinned_cap = 0;
  hipEvent_t uploaded = nullptr;   // recorded after the upload: the copy may be rewritten once it completes
  bool upload_pending = false;
};
std::mutex g_graph_mu;
std::map<std::string, GraphEntry> g_graphs;

// Frees a cache entry once its last upload has completed.
void release_entry(GraphEntry& ge) {
  if (ge.upload_pending && ge.uploaded) (void)hipEventSynchronize(ge.uploaded);
  ge.upload_pending = false;
  if (ge.uploaded) (void)hipEventDestroy(ge.uploaded);
  if (ge.pinned) (void)hipHostFree(ge.pinned);
  if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
  ge = GraphEntry();
}
hipStream_t g_cap_stream = nullptr;
hipEvent_t g_ev_in = nullptr, g_ev_out = nullptr;

std::string batch_key(const Batch& b, const bos_params& q, const char* tables, const uint32_t* d_status) {
  std::string k;
  auto add = [&](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  const uint32_t cnt = uint32_t(b.jobs.size());
  add(&cnt, 4);
  add(&b.rec, sizeof(b.rec));
  add(&q.z, 4);
  add(&q.k, 4);
  add(&tables, sizeof(tables));
  add(&d_status, sizeof(d_status));
  for (const BatchJob& j : b.jobs) {
    add(&j.n, 8);
    add(&j.pl.Z, 4);
    add(&j.pl.tile, 4);
    add(&j.pl.P, 4);
    add(j.pl.klev, sizeof(uint32_t) * j.pl.P);
  }
  // jobs whose routing is launched directly carry their pointers in kernel
  // arguments, not in the tables
  for (const BatchJob& j : b.jobs)
    if (j.special) {
      add(&j.in, sizeof(j.in));
      add(&j.start, sizeof(j.start));
      add(&j.seed, 8);
    }
  return k;
}

bos_status run_batch(Batch& b, const bos_params& q, hipStream_t s, uint32_t* d_status) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  // the tables live right after the per-instance regions of the workspace
  char* tables = b.jobs[0].ws + b.tab_base;
  if (!g_cap_stream) {
    if (hipStreamCreateWithFlags(&g_cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g_ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g_ev_out, hipEventDisableTiming) != hipSuccess)
      return BOS_ERR_HIP;
  }
  const std::string key = batch_key(b, q, tables, d_status);
  GraphEntry& ge = g_graphs[key];
  hipStream_t cs = g_cap_stream;
  // The tables go to the device from a pinned host copy, so the call returns
  // without waiting for the upload; the copy is rewritten only once the
  // previous upload from it has completed.
  if (!b.tables.empty()) {
    if (ge.upload_pending && hipEventSynchronize(ge.uploaded) != hipSuccess) return BOS_ERR_HIP;
    ge.upload_pending = false;
    if (ge.pinned_cap < b.tables.size()) {
      if (ge.pinned) (void)hipHostFree(ge.pinned);
      ge.pinned = nullptr;
      ge.pinned_cap = 0;
      void* ph = nullptr;
      if (hipHostMalloc(&ph, b.tables.size(), hipHostMallocDefault) != hipSuccess) return BOS_ERR_HIP;
      ge.pinned = static_cast<char*>(ph);
      ge.pinned_cap = b.tables.size();
    }
    if (!ge.uploaded && hipEventCreateWithFlags(&ge.uploaded, hipEventDisableTiming) != hipSuccess)
      return BOS_ERR_HIP;
    std::memcpy(ge.pinned, b.tables.data(), b.tables.size());
  }
  if (hipEventRecord(g_ev_in, s) != hipSuccess || hipStreamWaitEvent(cs, g_ev_in, 0) != hipSuccess) return BOS_ERR_HIP;
  if (!b.tables.empty()) {
    if (hipMemcpyAsync(tables, ge.pinned, b.tables.size(), hipMemcpyHostToDevice, cs) != hipSuccess ||
        hipEventRecord(ge.uploaded, cs) != hipSuccess)
      return BOS_ERR_HIP;
    ge.upload_pending = true;
  }
  if (!ge.exec) {
    const bool prof = g_prof_on;
    g_prof_on = false;  // no event records inside the captured graph
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      const hipError_t e1 = enqueue_batch(b, tables, cs, d_status);
      e = hipStreamEndCapture(cs, &graph);
      if (e1 != hipSuccess) e = e1;
    }
    g_prof_on = prof;
    if (e == hipSuccess) e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      release_entry(ge);
      g_graphs.erase(key);
      return BOS_ERR_HIP;
    }
  }
  prof_begin(BOS_K_OTHER, 0, 0, cs);
  hipError_t e = hipGraphLaunch(ge.exec, cs);
  prof_end(cs);
  if (e != hipSuccess) return BOS_ERR_HIP;
  if (hipEventRecord(g_ev_out, cs) != hipSuccess || hipStreamWaitEvent(s, g_ev_out, 0) != hipSuccess)
    return BOS_ERR_HIP;
  return BOS_OK;
}

bos_status sort_batched_sequential(const bos_instance* inst, uint32_t count, bos_rec rec, bos_params q, void* ws,
                                   size_t ws_bytes, hipStream_t s, uint32_t* d_status, bos_report* rep);

}  // namespace

extern "C" {

void bos_default_params(bos_params* p) {
  if (p) fill_defaults(p);
}

size_t bos_workspace_bytes(uint64_t n, bos_rec rec, const bos_params* p) {
  if (!has_gpu()) return 0;
  Plan pl;
  bos_params q = resolve(p);
  q.min_security_bits = 0;  // the size does not depend on the security floor
  if (make_plan(n, int(rec), q, true, &pl) != BOS_OK) return 0;
  return pl.total;
}

bos_status bos_trace_bind(void* route_buf, void* sort_buf, uint64_t slots) {
#ifdef BOS_TRACE_DIGEST
  if (slots && (slots & (slots - 1))) return BOS_ERR_INVALID_ARG;
  g_trace.buf[0] = route_buf;
  g_trace.buf[1] = sort_buf;
  g_trace.slots = slots;
  ++g_trace.gen;
  return BOS_OK;
#else
  (void)route_buf;
  (void)sort_buf;
  (void)slots;
  return BOS_ERR_UNSUPPORTED;
#endif
}

size_t bos_status_offset(uint64_t n, bos_rec rec, const bos_params* p) {
  if (!has_gpu()) return SIZE_MAX;
  Plan pl;
  bos_params q = resolve(p);
  q.min_security_bits = 0;  // the layout does not depend on the security floor
  if (make_plan(n, int(rec), q, true, &pl) != BOS_OK) return SIZE_MAX;
  return pl.off_status;
}

bos_status bos_plan(uint64_t n, bos_rec rec, const bos_params* p, uint64_t* buckets, uint32_t* levels,
                    uint32_t* passes_out) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  Plan pl;
  const bos_params q = resolve(p);
  const bos_status st = make_plan(n, int(rec), q, true, &pl);
  if (st != BOS_OK) return st;
  if (buckets) *buckets = pl.B;
  if (levels) *levels = pl.L;
  if (passes_out) {
    passes_out[0] = pl.P;
    for (uint32_t t = 0; t < pl.P; ++t) passes_out[1 + t] = pl.klev[t];
  }
  return BOS_OK;
}

bos_status bos_orp(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* ws,
                   size_t ws_bytes, void* stream, bos_report* rep) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  const bos_params q = resolve(p);
  Plan pl;
  bos_status st = make_plan(n, int(rec), q, true, &pl);
  if (st != BOS_OK) return st;
  if (n == 0) {
    fill_report(rep, pl, 0, kNoOverflow, 0);
    return BOS_OK;
  }
  if (!in || !out) return BOS_ERR_INVALID_ARG;
  if (!ws || ws_bytes < pl.total) return BOS_ERR_WORKSPACE;
  uint32_t attempts = 0;
  uint64_t ovf = kNoOverflow;
  // plans of two or more passes: split last pass, scan, then the per-bin
  // finish kernel; single-pass plans keep the fused last pass
  st = run_routing(pl, q, in, out, 0, static_cast<char*>(ws), static_cast<hipStream_t>(stream), &attempts, &ovf,
                   q.attempt, kNoOverflow, split_last(pl));
  fill_report(rep, pl, attempts, ovf, 0);
  return st;
}

}  // extern "C"

// Workspace of bos_sort_noalloc (see below).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

bos_status sort_impl(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* ws,
                     size_t ws_bytes, void* stream, bos_report* rep) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  const bos_params q = resolve(p);
  Plan pl;
  bos_status st = make_plan(n, int(rec), q, true, &pl);
  if (st != BOS_OK) return st;
  if (n == 0) {
    fill_report(rep, pl, 0, kNoOverflow, 0);
    return BOS_OK;
  }
  if (!in || !out) return BOS_ERR_INVALID_ARG;
  if (!ws || ws_bytes < pl.total) return BOS_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // The comparison sort ping-pongs between `out` and a free region of the
  // workspace (sort_tmp); the routing output goes where the sort must start
  // so that the result lands in `out`.
  const uint32_t passes = comparison_sort_hbm_passes(pl.rec, n, pl.tile, true);
  const bool split = split_last(pl);
  void* tmp = sort_tmp(pl, w);
  void* start = (passes % 2 == 0) ? out : tmp;
  void* other = (passes % 2 == 0) ? tmp : out;
  uint32_t attempts = 0;
  uint64_t ovf = kNoOverflow;
  st = run_routing(pl, q, in, start, 1, w, s, &attempts, &ovf, q.attempt, kNoOverflow, split);
  if (st != BOS_OK) {
    fill_report(rep, pl, attempts, ovf, 0);
    return st;
  }
  void* result = nullptr;
  hipError_t e = launch_comparison_sort(pl.rec, start, other, n, pl.tile,
                                        reinterpret_cast<uint64_t*>(w + pl.off_split), s, &result, true);
  if (e != hipSuccess) return BOS_ERR_HIP;
  if (result != out) {
    e = hipMemcpyAsync(out, result, n * pl.rec, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return BOS_ERR_HIP;
  }
  if (q.flags & BOS_SYNC) {
    unsigned long long err = 0;
    if (hipMemcpyAsync(&err, comparison_sort_err_word(reinterpret_cast<uint64_t*>(w + pl.off_split), n, pl.rec), 8,
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return BOS_ERR_HIP;
    if (err) return BOS_ERR_INTERNAL;
  }
  fill_report(rep, pl, attempts, ovf, uint64_t(2 + 2 * passes) * n * pl.rec);
  return BOS_OK;
}

// ---- workspace held by the library, for callers that cannot allocate ------
//
// bos_sort_noalloc runs bos_sort with its workspace in this array.  Each GPU
// the library runs on holds its own copy for the life of the process.  In
// host code the array's name is only a host-side stand-in: its device address
// is looked up once per device (with that device current) and only that
// address is handed to kernels and copies.
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {nullptr};

bos_status scratch_of_current_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BOS_ERR_HIP;
  if (dev < 0 || dev >= kScratchDevices) return BOS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BOS_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BOS_OK;
}

}  // namespace

extern "C" {

bos_status bos_sort(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* ws,
                    size_t ws_bytes, void* stream, bos_report* rep) {
  return sort_impl(in, out, n, rec, p, ws, ws_bytes, stream, rep);
}

bos_status bos_sort_noalloc(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* stream,
                            bos_report* rep) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  void* ws = nullptr;
  const bos_status st = scratch_of_current_device(&ws);
  if (st != BOS_OK) return st;
  // sort_impl rejects a plan whose workspace exceeds the array with
  // BOS_ERR_WORKSPACE before it launches anything
  return sort_impl(in, out, n, rec, p, ws, kScratchBytes, stream, rep);
}

size_t bos_batched_workspace_bytes(const uint64_t* n, uint32_t count, bos_rec rec, const bos_params* p) {
  if (!has_gpu() || (count && !n)) return 0;
  bos_params q = resolve(p);
  q.min_security_bits = 0;
  Batch b;
  if (build_batch(nullptr, n, count, int(rec), q, nullptr, &b) != BOS_OK) return 0;
  return b.total;
}

bos_status bos_sort_batched(const bos_instance* inst, uint32_t count, bos_rec rec, const bos_params* p,
                            void* ws, size_t ws_bytes, void* stream, uint32_t* d_status, bos_report* rep) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  if (count && !inst) return BOS_ERR_INVALID_ARG;
  const bos_params q = resolve(p);
  hipStream_t s = static_cast<hipStream_t>(stream);
  std::vector<uint64_t> ns(count);
  for (uint32_t i = 0; i < count; ++i) ns[i] = inst[i].n;
  Batch b;
  bos_status st = build_batch(inst, ns.data(), count, int(rec), q, static_cast<char*>(ws), &b);
  if (st != BOS_OK) return st;
  if (!ws || ws_bytes < b.total) return BOS_ERR_WORKSPACE;
  if (rep) {
    // Z, k and tile when every instance shares them, else 0
    std::memset(rep, 0, sizeof(*rep));
    for (uint32_t i = 0; i < count; ++i) {
      const Plan& pl = b.jobs[i].pl;
      rep->z = (i == 0 || rep->z == pl.Z) ? pl.Z : 0;
      rep->k = (i == 0 || rep->k == pl.k) ? pl.k : 0;
      rep->tile = (i == 0 || rep->tile == pl.tile) ? pl.tile : 0;
    }
    rep->first_overflow_level = -1;
    rep->first_overflow_pair = -1;
  }
  if (count == 0) return BOS_OK;
  if (!b.batched) return sort_batched_sequential(inst, count, rec, q, ws, ws_bytes, s, d_status, rep);
  if (!d_status) return BOS_ERR_INVALID_ARG;
  st = run_batch(b, q, s, d_status);
  if (st != BOS_OK) return st;
  uint32_t attempts = 0;
  uint64_t bytes = 0;
  bos_status worst = BOS_OK;
  std::vector<uint32_t> hs(count, 0);
  if (q.flags & BOS_SYNC) {
    if (hipMemcpyAsync(hs.data(), d_status, count * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return BOS_ERR_HIP;
    // Instances whose first attempt overflowed continue alone from attempt 1
    // (the same attempts and labels bos_sort would use).
    for (uint32_t i = 0; i < count; ++i) {
      const BatchJob& j = b.jobs[i];
      uint32_t att = j.n ? 1u : 0u;
      if (hs[i] != BOS_OK && hs[i] != BOS_ERR_OVERFLOW) {
        if (worst == BOS_OK) worst = bos_status(hs[i]);  // a comparison-sort consistency check failed
      } else if (hs[i] == BOS_ERR_OVERFLOW) {
        uint64_t ovf = kNoOverflow, prev = kNoOverflow;
        if (hipMemcpyAsync(&prev, j.ws + j.pl.off_status, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return BOS_ERR_HIP;
        bos_params qi = q;
        qi.seed = inst[i].seed;
        const bos_status rs = run_routing(j.pl, qi, j.in, j.start, 1, j.ws, s, &att, &ovf, 1, prev, j.split);
        bos_status fs = rs;
        if (rs == BOS_OK) {
          void* result = nullptr;
          unsigned long long err = 0;
          uint64_t* split = reinterpret_cast<uint64_t*>(j.ws + j.pl.off_split);
          if (launch_comparison_sort(j.pl.rec, j.start, j.other, j.n, j.pl.tile, split, s, &result, true) !=
                  hipSuccess ||
              hipMemcpyAsync(&err, err_word(j.pl, j.ws, j.n), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess)
            return BOS_ERR_HIP;
          if (err) fs = BOS_ERR_INTERNAL;
        }
        hs[i] = fs;
        if (hipMemcpyAsync(d_status + i, &hs[i], 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return BOS_ERR_HIP;
        if (fs != BOS_OK && worst == BOS_OK) worst = fs;
      }
      attempts += att;
      bytes += routing_bytes(j.pl) + uint64_t(2 + 2 * j.merges) * j.n * j.pl.rec;
    }
  }
  if (rep) {
    rep->attempts = attempts;
    rep->algorithmic_bytes = bytes;
    rep->buckets = count;
  }
  return worst;
}


// ---- continuous batching --------------------------------------------------
//
// A step is a budget of device work, handed out in array order (the caller
// puts its oldest job first).  The first unfinished job always runs at least
// one phase (several if they are cheap: up to kStepMinQuantum); later jobs
// backfill a budget of twice that, capped at kStepBackfillCap, each as many
// phases as fit, so small requests run several phases next to one phase of a
// large request, large requests keep their order, and a large head request
// keeps at least two thirds of the device (its latency sets the tail).  The phase cost model is
// n + kStepFixed records (kStepFixed stands for the launch overhead of a
// phase).  The overflow check of an attempt is
// speculative: a job that finished its routing passes goes on to the
// comparison sort in the same step, and the status words of those jobs are
// read once at the end of the step; a job whose attempt overflowed goes back
// to pass 0 with the next attempt, and whatever it wrote is redone.

constexpr uint32_t kStepRounds = 32;           // sub-rounds per step at most
constexpr uint64_t kStepFixed = 1ull << 17;    // launch overhead, in records
constexpr uint64_t kStepMinQuantum = 1ull << 21;
constexpr uint64_t kStepBackfillCap = 1ull << 23;

size_t step_round_bytes(uint32_t count) {
  // every job adds at most one entry of each kind; each table starts aligned
  // (fill, 2 per route group -- at most one group per job, and at most 5
  // kinds x 8 Z x 12 levels --, strip, 5 tile sizes, two-way and four-way
  // merge passes)
  const size_t groups = std::min<size_t>(count, 5 * 8 * 12);
  return size_t(count) * (2 * sizeof(FillSeg) + sizeof(PassArgs) + 4 + sizeof(StripSeg) + 2 * sizeof(SortSeg) +
                          sizeof(M4Seg)) +
         (2 * groups + 12) * kAlign;
}

size_t bos_step_workspace_bytes(uint32_t count) {
  // the rounds' tables, then two status entries per job (routing checked, or
  // comparison sort ended): two pointers and one result word each
  return align_up(kStepRounds * step_round_bytes(count) + size_t(count) * 40 + 6 * kAlign);
}

}  // extern "C"

// State of a pipelined sequence of steps (bos_sort_step_async): the previous
// step, still in flight when a call returns, and the pinned host buffers of
// the two alternating steps.
struct bos_stepper {
  struct Routed {
    void* ws;
    uint32_t attempt, slot;  // slot: index in the step's status words
  };
  struct Finished {
    void* ws;
    uint32_t attempt, slot;  // slot: index of its error-word check in the step's status words
  };
  struct Half {
    char* tab = nullptr;  // pinned: the step's tables
    size_t tab_cap = 0;
    uint32_t* st = nullptr;  // pinned: the step's status words
    size_t st_cap = 0;
    hipEvent_t ev = nullptr;
    std::vector<Routed> routed;
    std::vector<Finished> finished;
  };
  Half half[2];
  uint64_t calls = 0;
  bool pending = false;  // the previous call's step is in flight
  int device = -1;
};

namespace {

// Grow a pinned host buffer (its previous contents are not kept).
bool grow_pinned(void** p, size_t* cap, size_t need) {
  if (*cap >= need) return true;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  const size_t n = std::max<size_t>(need + need / 2, 4096);
  if (hipHostMalloc(p, n, hipHostMallocDefault) != hipSuccess) return false;
  *cap = n;
  return true;
}

// The last phase index of a job plus one: in a pipelined sequence, the phase
// of a job whose every phase has been enqueued and whose result is not yet
// known.
uint32_t after_last_phase(const Plan& pl, uint32_t merges) { return pl.P + 1 + merges; }

bos_status step_impl(bos_job* jobs, uint32_t count, bos_rec rec, const bos_params* p, void* step_ws_arg,
                     size_t step_ws_bytes_arg, void* stream, bos_stepper* ctx) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  if (count && !jobs) return BOS_ERR_INVALID_ARG;
  const bos_params q = resolve(p);
  const int R = int(rec);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (count == 0 && !(ctx && ctx->pending)) return BOS_OK;
  // a pipelined step uses one half of step_ws; the other may still be read
  // by the step in flight
  const uint32_t par = ctx ? uint32_t(ctx->calls & 1) : 0u;
  const size_t step_ws_bytes = ctx ? (step_ws_bytes_arg / 2) & ~(kAlign - 1) : step_ws_bytes_arg;
  void* step_ws = ctx && step_ws_arg ? static_cast<char*>(step_ws_arg) + par * step_ws_bytes : step_ws_arg;
  if (count && (!step_ws || step_ws_bytes < bos_step_workspace_bytes(count))) return BOS_ERR_WORKSPACE;
  const bool batchable = !(q.flags & BOS_GENERIC_ROUTING);
  std::vector<Plan> plans(count);
  std::vector<uint32_t> merges(count, 0), allowed(count, 0);
  std::vector<char> routed(count, 0);  // finished an attempt's routing in this step
  uint64_t quantum = kStepMinQuantum;
  for (uint32_t i = 0; i < count; ++i) {
    bos_job& j = jobs[i];
    if (j.phase == BOS_PHASE_DONE) continue;
    if (j.n == 0) {
      j.phase = BOS_PHASE_DONE;
      j.status = BOS_OK;
      continue;
    }
    if (!j.in || !j.out || j.in == j.out) return BOS_ERR_INVALID_ARG;
    const bos_status st = make_plan_cached(j.n, R, q, &plans[i]);
    if (st != BOS_OK) return st;
    if (!j.ws || j.ws_bytes < plans[i].total) return BOS_ERR_WORKSPACE;
    merges[i] = comparison_sort_hbm_passes(R, j.n, plans[i].tile, true);
    if (j.phase > plans[i].P + merges[i] + (ctx ? 1u : 0u)) return BOS_ERR_INVALID_ARG;
  }
  {
    bool head = true;
    uint64_t left = 0;
    for (uint32_t i = 0; i < count; ++i) {
      const bos_job& j = jobs[i];
      if (j.phase == BOS_PHASE_DONE) continue;
      const uint64_t c = j.n + kStepFixed;
      const uint64_t remaining = uint64_t(plans[i].P) + 1 + merges[i] - j.phase;
      if (remaining == 0) continue;  // every phase enqueued (pipelined), awaiting its result
      uint64_t k;
      if (head) {
        quantum = std::max(quantum, c);
        k = std::max<uint64_t>(1, kStepMinQuantum / c);
        left = std::min<uint64_t>(2 * quantum, kStepBackfillCap);
        head = false;
      } else {
        k = left / c;
      }
      k = std::min<uint64_t>({k, remaining, kStepRounds});
      allowed[i] = uint32_t(k);
      left -= std::min(left, k * c);
    }
  }
  auto tmp_buf = [&](uint32_t i) -> void* { return sort_tmp(plans[i], static_cast<char*>(jobs[i].ws)); };
  auto start_buf = [&](uint32_t i) -> void* { return (merges[i] % 2 == 0) ? jobs[i].out : tmp_buf(i); };
  auto other_buf = [&](uint32_t i) -> void* { return (merges[i] % 2 == 0) ? tmp_buf(i) : jobs[i].out; };

  // Build every sub-round's tables on the host, then upload them at once.
  // route launches of a round: one per (pass kind, log2 Z); tile sorts: one
  // per tile size (index 0..4 = 4096, 2048, 1024, 8192, 16384)
  struct RouteGroup {
    std::vector<PassArgs> args;
    std::vector<uint32_t> starts;
    size_t o_args = 0, o_starts = 0;
    uint32_t blocks = 0, threads = 64, lds = 0, items0 = 0;
  };
  struct Round {
    size_t o_fill = 0, o_strip = 0, o_tile[5] = {0, 0, 0, 0, 0}, o_merge = 0, o_m4 = 0;
    uint32_t nfill = 0, nstrip = 0, ntile[5] = {0, 0, 0, 0, 0}, nmerge = 0, nm4 = 0;
    uint32_t sblocks = 0, tiles[5] = {0, 0, 0, 0, 0}, mtiles = 0, m4[5] = {0, 0, 0, 0, 0};
    std::map<uint32_t, RouteGroup> route;  // key: (mode * 16 + lz) * 16 + levels of the pass
    std::vector<uint32_t> whole;  // jobs routed by the per-job path in this round
  };
  const uint32_t kTiles[5] = {4096, 2048, 1024, 8192, 16384};
  std::vector<Round> rounds;
  std::vector<char> tab;
  std::vector<uint32_t> phase(count);
  for (uint32_t i = 0; i < count; ++i) phase[i] = jobs[i].phase;
  // a job's last phase: done (synchronous step), or enqueued with its result
  // pending until the step has run (pipelined)
  std::vector<uint32_t> finished;
  auto finish = [&](uint32_t i) -> uint32_t {
    finished.push_back(i);
    if (!ctx) return BOS_PHASE_DONE;
    return after_last_phase(plans[i], merges[i]);
  };
  for (uint32_t r = 0; r < kStepRounds; ++r) {
    Round rd;
    std::vector<FillSeg> fills;
    std::vector<StripSeg> strips;
    std::vector<SortSeg> tiles[5];
    MergeRound mr;
    bool any = false;
    for (uint32_t i = 0; i < count; ++i) {
      if (phase[i] == BOS_PHASE_DONE || allowed[i] <= r) continue;
      bos_job& j = jobs[i];
      const Plan& pl = plans[i];
      char* w = static_cast<char*>(j.ws);
      any = true;
      const uint32_t ph = phase[i];
      if (ph < pl.P) {
        if (pl.L == 0 || !batchable || !batched_lz(pl.lz) || !use_route_kernel(pl, ph)) {
          if (ph != 0) return BOS_ERR_INVALID_ARG;  // per-job routing runs a whole attempt at once
          rd.whole.push_back(i);
          phase[i] = pl.P;
          routed[i] = 1;
          continue;
        }
        unsigned long long* status = reinterpret_cast<unsigned long long*>(w + pl.off_status);
        if (ph == 0) fills.push_back(FillSeg{status, 2 + pl.nblocks_last, 0});
        const bool first = ph == 0, last = ph + 1 == pl.P;
        const bool split = last && split_last(pl);
        const int mode = (first ? 1 : 0) | (last ? 2 : 0) | (split ? 4 : 0);
        PassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.x_in = j.in;
        a.out = start_buf(i);
        a.rec_in = w + pl.off_rec[(ph + 1) & 1];
        a.tag_in = reinterpret_cast<const uint32_t*>(w + pl.off_tag[(ph + 1) & 1]);
        a.rec_out = w + pl.off_rec[ph & 1];
        a.tag_out = reinterpret_cast<uint32_t*>(w + pl.off_tag[ph & 1]);
        a.status = status;
        a.ticket = reinterpret_cast<uint32_t*>(status + 1);
        a.scan = status + 2;
        a.n = pl.n;
        a.buckets = pl.B;
        a.seed = j.seed;
        a.z = pl.Z;
        a.lz = pl.lz;
        a.levels = pl.L;
        a.level0 = pl.lev0[ph];
        a.klev = pl.klev[ph];
        a.attempt = j.attempt;
        a.fin = 1;
        if (split) {
          a.loads = reinterpret_cast<uint32_t*>(w + pl.off_loads);
          strips.push_back(strip_seg(pl, w, start_buf(i), rd.sblocks));
          rd.sblocks += pl.nblocks_last;
        }
        const uint32_t items = uint32_t(pl.B >> pl.klev[ph]);
        RouteGroup& g = rd.route[(uint32_t(mode) * 16u + pl.lz) * 16u + pl.klev[ph]];
        if (g.args.empty()) g.items0 = items;
        g.args.push_back(a);
        g.starts.push_back(g.blocks);
        g.blocks += items;
        g.threads = std::max(g.threads, uint32_t((pl.Z << pl.klev[ph]) >> 4));
        g.lds = std::max(g.lds, pass_lds_bytes(R, pl.Z, pl.klev[ph], false, (mode & 2) && !(mode & 4)));
        if (last) {
          phase[i] = pl.P;  // on to the tile sort; the check is at the end of the step
          routed[i] = 1;
        } else {
          ++phase[i];
        }
      } else if (ph == pl.P) {
        uint32_t ti = 0;
        while (kTiles[ti] != pl.tile) ++ti;  // the plan's tile is one of kTiles
        const uint32_t T = pl.tile;
        const uint32_t c = uint32_t((j.n + T - 1) / T);
        if (j.n > 1) {
          tiles[ti].push_back(SortSeg{start_buf(i), split_smp(pl, w, j.n), j.n, 0, nullptr, rd.tiles[ti], c});
          rd.tiles[ti] += c;
          fills.push_back(FillSeg{err_word(pl, w, j.n), 1, 1});  // before this round's tile sorts
        }
        phase[i] = merges[i] == 0 ? finish(i) : pl.P + 1;
      } else {
        const uint32_t pass = ph - (pl.P + 1);
        void* src = (pass % 2 == 0) ? start_buf(i) : other_buf(i);
        void* dst = (pass % 2 == 0) ? other_buf(i) : start_buf(i);
        mr.add(R, src, dst, j.n, pl.tile, pass, reinterpret_cast<uint64_t*>(w + pl.off_split));
        phase[i] = pass + 1 >= merges[i] ? finish(i) : ph + 1;
      }
    }
    if (!any) break;
    rd.nfill = uint32_t(fills.size());
    rd.o_fill = push_table(tab, fills);
    rd.nstrip = uint32_t(strips.size());
    rd.o_strip = push_table(tab, strips);
    for (auto& kv : rd.route) {
      kv.second.o_args = push_table(tab, kv.second.args);
      kv.second.o_starts = push_table(tab, kv.second.starts);
    }
    for (int ti = 0; ti < 5; ++ti) {
      rd.ntile[ti] = uint32_t(tiles[ti].size());
      rd.o_tile[ti] = push_table(tab, tiles[ti]);
    }
    rd.nmerge = uint32_t(mr.two.size());
    rd.mtiles = mr.two_tiles;
    rd.o_merge = push_table(tab, mr.two);
    rd.nm4 = uint32_t(mr.four.size());
    std::memcpy(rd.m4, mr.m4, sizeof(rd.m4));
    rd.o_m4 = push_table(tab, mr.four);
    rounds.push_back(std::move(rd));
  }
  // status checks: the overflow word of every job whose routing finished in
  // this step (entries 0 .. st_job.size() - 1), then the comparison sort's
  // error word of every job that ended in it
  std::vector<unsigned long long*> st_ptr, er_ptr;
  std::vector<uint32_t> st_job;
  for (uint32_t i = 0; i < count; ++i)
    if (routed[i]) {
      st_ptr.push_back(reinterpret_cast<unsigned long long*>(static_cast<char*>(jobs[i].ws) + plans[i].off_status));
      er_ptr.push_back(nullptr);
      st_job.push_back(i);
    }
  for (uint32_t i : finished) {
    st_ptr.push_back(nullptr);
    er_ptr.push_back(jobs[i].n > 1 ? err_word(plans[i], static_cast<char*>(jobs[i].ws), jobs[i].n) : nullptr);
  }
  const size_t o_stp = push_table(tab, st_ptr);
  const size_t o_erp = push_table(tab, er_ptr);
  const size_t o_sto = align_up(tab.size());
  if (o_sto + align_up(st_ptr.size() * 4) > step_ws_bytes) return BOS_ERR_WORKSPACE;
  char* dtab = static_cast<char*>(step_ws);
  bos_stepper::Half* hf = ctx ? &ctx->half[par] : nullptr;
  const char* htab = tab.data();
  if (hf) {
    // the tables go through pinned memory so that the upload does not wait
    // for the step in flight (this half's previous step has completed)
    if (!grow_pinned(reinterpret_cast<void**>(&hf->tab), &hf->tab_cap, tab.size()) ||
        !grow_pinned(reinterpret_cast<void**>(&hf->st), &hf->st_cap, st_ptr.size() * 4 + 4))
      return BOS_ERR_HIP;
    if (!tab.empty()) std::memcpy(hf->tab, tab.data(), tab.size());
    htab = hf->tab;
    if (!hf->ev && hipEventCreateWithFlags(&hf->ev, hipEventDisableTiming) != hipSuccess) return BOS_ERR_HIP;
  }
  if (!tab.empty() && hipMemcpyAsync(dtab, htab, tab.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return BOS_ERR_HIP;
  hipError_t e = hipSuccess;
  for (const Round& rd : rounds) {
    if (e == hipSuccess && rd.nfill)
      e = launch_fill_status_batched(reinterpret_cast<const FillSeg*>(dtab + rd.o_fill), rd.nfill, s);
    for (uint32_t i : rd.whole) {
      if (e != hipSuccess) break;
      e = enqueue_routing(plans[i], jobs[i].in, start_buf(i), jobs[i].seed, jobs[i].attempt, 1,
                          static_cast<char*>(jobs[i].ws), s, -1, split_last(plans[i]));
    }
    for (const auto& kv : rd.route) {
      if (e != hipSuccess) break;
      const int m = int(kv.first / 256u);
      const uint32_t lz = (kv.first / 16u) % 16u;
      const RouteGroup& g = kv.second;
      if (g.args.size() == 1)  // one job: the persistent kernel of the single-sort path
        e = launch_route(R, g.args[0], (m & 1) != 0, (m & 2) != 0, g.items0, num_cus(), s, (m & 4) != 0);
      else
        e = launch_route_batched(R, lz, (m & 1) != 0, (m & 2) != 0, reinterpret_cast<const PassArgs*>(dtab + g.o_args),
                                 reinterpret_cast<const uint32_t*>(dtab + g.o_starts), uint32_t(g.args.size()),
                                 g.blocks, g.threads, g.lds, s, (m & 4) != 0);
    }
    if (e == hipSuccess && rd.nstrip)
      e = launch_strip_batched(R, reinterpret_cast<const StripSeg*>(dtab + rd.o_strip), rd.nstrip, rd.sblocks, s);
    for (int ti = 0; ti < 5; ++ti)
      if (e == hipSuccess && rd.ntile[ti])
        e = launch_sort_batched(R, 0, kTiles[ti], reinterpret_cast<const SortSeg*>(dtab + rd.o_tile[ti]), rd.ntile[ti],
                                rd.tiles[ti], s);
    if (e == hipSuccess && rd.nmerge) {
      e = launch_sort_batched(R, 1, 0, reinterpret_cast<const SortSeg*>(dtab + rd.o_merge), rd.nmerge, rd.mtiles, s);
      if (e == hipSuccess)
        e = launch_sort_batched(R, 2, 0, reinterpret_cast<const SortSeg*>(dtab + rd.o_merge), rd.nmerge, rd.mtiles, s);
    }
    if (e == hipSuccess && rd.nm4)
      e = launch_merge4_batched(R, reinterpret_cast<const M4Seg*>(dtab + rd.o_m4), rd.nm4, rd.m4, s);
  }
  uint32_t* st_host_ptr = nullptr;
  std::vector<uint32_t> st_host(ctx ? 0 : st_ptr.size(), 0);
  if (e == hipSuccess && !st_ptr.empty()) {
    uint32_t* d_out = reinterpret_cast<uint32_t*>(dtab + o_sto);
    st_host_ptr = hf ? hf->st : st_host.data();
    e = launch_batch_status(reinterpret_cast<unsigned long long* const*>(dtab + o_stp),
                            reinterpret_cast<unsigned long long* const*>(dtab + o_erp), d_out, uint32_t(st_ptr.size()),
                            s);
    if (e == hipSuccess) e = hipMemcpyAsync(st_host_ptr, d_out, st_ptr.size() * 4, hipMemcpyDeviceToHost, s);
  }
  auto overflowed = [&](bos_job& j) {
    if (j.attempt < q.max_retries) {
      ++j.attempt;
      j.phase = 0;
      j.status = BOS_OK;
      j.reserved = 0;
    } else {
      j.phase = BOS_PHASE_DONE;
      j.status = BOS_ERR_OVERFLOW;
    }
  };
  if (!ctx) {
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return BOS_ERR_HIP;
    for (uint32_t i = 0; i < count; ++i) {
      if (jobs[i].phase == BOS_PHASE_DONE) continue;
      jobs[i].phase = phase[i];
      if (phase[i] == BOS_PHASE_DONE) jobs[i].status = BOS_OK;
    }
    for (size_t t = 0; t < st_job.size(); ++t)
      if (st_host[t] != 0) overflowed(jobs[st_job[t]]);
    for (size_t t = 0; t < finished.size(); ++t) {
      bos_job& j = jobs[finished[t]];
      if (j.phase == BOS_PHASE_DONE && j.status == BOS_OK && st_host[st_job.size() + t] != 0)
        j.status = BOS_ERR_INTERNAL;  // a four-way tile failed its bound checks
    }
    return BOS_OK;
  }
  // Pipelined: this step stays in flight; the previous one is waited for and
  // its routing checks and completions are applied.  Jobs are found by their
  // workspace, so the caller may reorder, drop finished or add jobs between
  // calls.
  const bool enqueued = !rounds.empty();
  if (e == hipSuccess && enqueued) e = hipEventRecord(hf->ev, s);
  if (e != hipSuccess) return BOS_ERR_HIP;
  for (uint32_t i = 0; i < count; ++i)
    if (jobs[i].phase != BOS_PHASE_DONE) jobs[i].phase = phase[i];
  bos_stepper::Half& prev = ctx->half[par ^ 1u];
  if (ctx->pending) {
    if (hipEventSynchronize(prev.ev) != hipSuccess) return BOS_ERR_HIP;
    std::unordered_map<void*, uint32_t> at;
    at.reserve(count * 2);
    for (uint32_t i = 0; i < count; ++i) at[jobs[i].ws] = i;
    for (const bos_stepper::Routed& r : prev.routed) {
      auto it = at.find(r.ws);
      if (it == at.end()) continue;
      bos_job& j = jobs[it->second];
      if (j.phase == BOS_PHASE_DONE || j.attempt != r.attempt) continue;
      if (prev.st[r.slot] != 0)
        overflowed(j);
      else
        j.reserved = 1;  // this attempt's routing checked
    }
    for (const bos_stepper::Finished& f : prev.finished) {
      auto it = at.find(f.ws);
      if (it == at.end()) continue;
      bos_job& j = jobs[it->second];
      if (j.phase == BOS_PHASE_DONE || j.attempt != f.attempt || j.reserved != 1) continue;
      j.phase = BOS_PHASE_DONE;
      j.status = prev.st[f.slot] != 0 ? BOS_ERR_INTERNAL : BOS_OK;
    }
    prev.routed.clear();
    prev.finished.clear();
  }
  hf->routed.clear();
  hf->finished.clear();
  for (size_t t = 0; t < st_job.size(); ++t)
    hf->routed.push_back({jobs[st_job[t]].ws, jobs[st_job[t]].attempt, uint32_t(t)});
  for (size_t t = 0; t < finished.size(); ++t)
    hf->finished.push_back({jobs[finished[t]].ws, jobs[finished[t]].attempt, uint32_t(st_job.size() + t)});
  ctx->pending = enqueued;
  ++ctx->calls;
  return BOS_OK;
}

}  // namespace

extern "C" {

bos_status bos_sort_step(bos_job* jobs, uint32_t count, bos_rec rec, const bos_params* p, void* step_ws,
                         size_t step_ws_bytes, void* stream) {
  return step_impl(jobs, count, rec, p, step_ws, step_ws_bytes, stream, nullptr);
}

bos_stepper* bos_stepper_create(void) {
  if (!has_gpu()) return nullptr;
  bos_stepper* st = new (std::nothrow) bos_stepper();
  if (st && hipGetDevice(&st->device) != hipSuccess) st->device = -1;
  return st;
}

void bos_stepper_destroy(bos_stepper* st) {
  if (!st) return;
  for (bos_stepper::Half& h : st->half) {
    if (h.ev) {
      (void)hipEventSynchronize(h.ev);
      (void)hipEventDestroy(h.ev);
    }
    if (h.tab) (void)hipHostFree(h.tab);
    if (h.st) (void)hipHostFree(h.st);
  }
  delete st;
}

bos_status bos_sort_step_async(bos_stepper* st, bos_job* jobs, uint32_t count, bos_rec rec, const bos_params* p,
                               void* step_ws, size_t step_ws_bytes, void* stream) {
  if (!st) return BOS_ERR_INVALID_ARG;
  return step_impl(jobs, count, rec, p, step_ws, step_ws_bytes, stream, st);
}

size_t bos_bitonic_workspace_bytes(uint64_t n, bos_rec rec) {
  if (rec != 8 && rec != 16) return 0;
  uint64_t N = bitonic_tile(int(rec));
  while (N < n) N <<= 1;
  return align_up(size_t(N) * rec);
}

bos_status bos_bitonic_sort(const void* in, void* out, uint64_t n, bos_rec rec, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  if (rec != 8 && rec != 16) return BOS_ERR_INVALID_ARG;
  if (n > kMaxN) return BOS_ERR_INVALID_ARG;
  if (n == 0) return BOS_OK;
  if (!in || !out) return BOS_ERR_INVALID_ARG;
  if (!ws || ws_bytes < bos_bitonic_workspace_bytes(n, rec)) return BOS_ERR_WORKSPACE;
  uint64_t N = bitonic_tile(int(rec));
  while (N < n) N <<= 1;
  return hip_status(launch_bitonic(int(rec), in, out, n, ws, N, static_cast<hipStream_t>(stream)));
}

bos_status bos_set_tuning(const bos_tune_entry* entries, uint32_t count) {
  if (count && !entries) return BOS_ERR_INVALID_ARG;
  for (uint32_t i = 0; i < count; ++i) {
    const bos_tune_entry& e = entries[i];
    const bool zok = e.z == 0 || (e.z >= 8 && e.z <= 2048 && (e.z & (e.z - 1)) == 0);
    if ((e.rec != 8 && e.rec != 16) || e.log2n > 40 || !zok || e.k > 12 ||
        (e.tile && !sort_tile_ok(int(e.rec), e.tile)))
      return BOS_ERR_INVALID_ARG;
  }
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.assign(entries, entries + count);
    ++g_tune_gen;
  }
  bos_release_cache();  // captured batches were planned with the old table
  return BOS_OK;
}

uint32_t bos_get_tuning(bos_tune_entry* out, uint32_t cap) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const uint32_t cnt = uint32_t(g_tune.size());
  for (uint32_t i = 0; i < cnt && i < cap && out; ++i) out[i] = g_tune[i];
  return cnt;
}

void bos_release_cache(void) {
  std::lock_guard<std::mutex> lock(g_graph_mu);
  for (auto& kv : g_graphs) release_entry(kv.second);
  g_graphs.clear();
}

void bos_profile_enable(int on) {
  g_prof_on = on != 0;
  if (!g_prof_on) g_prof_pending = false;
}

uint32_t bos_profile_read(bos_launch_time* out, uint32_t cap) {
  const uint32_t cnt = uint32_t(g_prof.size());
  for (uint32_t i = 0; i < cnt; ++i) {
    ProfRec& r = g_prof[i];
    float ms = 0.f;
    (void)hipEventSynchronize(r.stop);
    (void)hipEventElapsedTime(&ms, r.start, r.stop);
    if (out && i < cap) {
      out[i].kind = r.kind;
      out[i].index = r.index;
      out[i].ms = ms;
      out[i].reserved = 0;
      out[i].bytes = r.bytes;
    }
    g_event_pool.push_back(r.start);
    g_event_pool.push_back(r.stop);
  }
  g_prof.clear();
  return cnt;
}

const char* bos_status_string(bos_status s) {
  switch (s) {
    case BOS_OK: return "ok";
    case BOS_ERR_INVALID_ARG: return "invalid argument";
    case BOS_ERR_OVERFLOW: return "bucket overflow in every attempt";
    case BOS_ERR_WORKSPACE: return "workspace missing or too small";
    case BOS_ERR_HIP: return "HIP runtime error";
    case BOS_ERR_INSECURE_Z: return "Z below the security floor";
    case BOS_ERR_UNSUPPORTED: return "unsupported (no GPU or parameters)";
    case BOS_ERR_INTERNAL: return "internal consistency check failed (merge tile bounds)";
  }
  return "unknown status";
}

bos_status bos_debug_labels(uint64_t n, uint32_t levels, uint64_t seed, uint32_t attempt, uint32_t* labels_dev,
                            void* stream) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  if (levels > 31 || (n && !labels_dev)) return BOS_ERR_INVALID_ARG;
  return hip_status(launch_labels(labels_dev, n, levels, seed, attempt, static_cast<hipStream_t>(stream)));
}

bos_status bos_debug_levels(const void* in, uint64_t n, bos_rec rec, const bos_params* p, uint32_t attempt,
                            void* ws, size_t ws_bytes, void* stream, void* recs_host, uint32_t* tags_host,
                            uint32_t* levels_host, int32_t* ovf_level, int64_t* ovf_pair) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  const bos_params q = resolve(p);
  Plan pl;
  bos_status st = make_plan(n, int(rec), q, true, &pl);
  if (st != BOS_OK) return st;
  if (!ws || ws_bytes < pl.total) return BOS_ERR_WORKSPACE;
  if (!recs_host || !tags_host || !levels_host || !ovf_level || !ovf_pair || (n && !in)) return BOS_ERR_INVALID_ARG;
  char* w = static_cast<char*>(ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t slots = size_t(pl.B) * pl.Z;
  // boundary 0: level-0 arrays are never materialized by the fused first pass;
  // report them as not available (zero records, all-dummy tags)
  std::memset(recs_host, 0, slots * pl.rec);
  std::memset(tags_host, 0xFF, slots * 4);
  levels_host[0] = 0;
  uint64_t stv = kNoOverflow;
  // run passes 0..P-2 one at a time (the last pass strips instead of writing slots)
  for (uint32_t t = 0; t + 1 < pl.P; ++t) {
    if (enqueue_routing(pl, in, nullptr, q.seed, attempt, 0, w, s, int(t)) != hipSuccess) return BOS_ERR_HIP;
    char* rh = static_cast<char*>(recs_host) + (t + 1) * slots * pl.rec;
    uint32_t* th = tags_host + (t + 1) * slots;
    if (hipMemcpyAsync(rh, w + pl.off_rec[t & 1], slots * pl.rec, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(th, w + pl.off_tag[t & 1], slots * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&stv, w + pl.off_status, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return BOS_ERR_HIP;
    levels_host[t + 1] = pl.lev0[t] + pl.klev[t];
  }
  *ovf_level = stv == kNoOverflow ? -1 : int32_t(stv >> 32);
  *ovf_pair = stv == kNoOverflow ? -1 : int64_t(stv & 0xFFFFFFFFull);
  return stv == kNoOverflow ? BOS_OK : BOS_ERR_OVERFLOW;
}

}  // extern "C"

namespace {
bos_status sort_batched_sequential(const bos_instance* inst, uint32_t count, bos_rec rec, bos_params q, void* ws,
                                   size_t ws_bytes, hipStream_t s, uint32_t* d_status, bos_report* rep) {
  bos_status worst = BOS_OK;
  uint64_t bytes = 0;
  uint32_t attempts = 0;
  std::vector<uint32_t> host_status(count, BOS_OK);
  for (uint32_t i = 0; i < count; ++i) {
    q.seed = inst[i].seed;
    bos_report r;
    const bos_status st = bos_sort(inst[i].in, inst[i].out, inst[i].n, rec, &q, ws, ws_bytes, s, &r);
    host_status[i] = st;
    if (st != BOS_OK && worst == BOS_OK) worst = st;
    bytes += r.algorithmic_bytes;
    attempts += r.attempts;
  }
  if (d_status && count) {
    if (hipMemcpyAsync(d_status, host_status.data(), count * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return BOS_ERR_HIP;
  }
  if (rep) {
    rep->attempts = attempts;
    rep->algorithmic_bytes = bytes;
    rep->buckets = count;
  }
  return worst;
}
}  // namespace

// ---- out-of-core bucket ORP and sort (Section 4.3) --------------------------
//
// The records, the output and the two slot arrays of Algorithm 3.1 stay in host
// memory; the device holds the small per-run arrays (overflow word, bin loads,
// block counts) and staging buffers.  Every routing pass streams the slot
// arrays through the device once: a chunk of the pass's blocks is a range of
// consecutive block indices, whose input is one contiguous range of buckets
// when the chunk covers whole groups of 2^(i+k) buckets and 2^k contiguous
// segments otherwise, and whose output is one contiguous range of buckets
// (the consecutive-bucket structure of Section 4.3).  Chunks alternate between
// two staging sets and run as a pipeline over three streams (input copies,
// kernels, output copies; OocPipe), so that the next chunk's input copy runs
// while this chunk's output copy does: the host link carries both directions
// at once.  The per-bin finish (bos_orp) or strip (bos_sort) streams the bins
// the same way; the sort's comparison phase is a two-pass external sort: runs
// sorted on the device, then output segments cut by sample splitters, each
// gathered from the runs, sorted on the device and written once.
namespace {

constexpr uint64_t kMaxNHost = 1ull << 36;
constexpr int kOocDevices = 64;

struct OocStreams {
  hipStream_t st[3] = {nullptr, nullptr, nullptr};  // input copies, kernels, output copies
  hipEvent_t ev = nullptr;
  hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_k[2] = {nullptr, nullptr}, ev_out[2] = {nullptr, nullptr};
};
std::mutex g_ooc_mu;
OocStreams g_ooc[kOocDevices];

// Host workspace: slot arrays 0 and 1 (records, then the two tag arrays side
// by side: after routing they hold the sort's runs, 2 B Z 4 >= n R bytes).
struct HostLayout {
  size_t off_rec[2], off_tag[2], total;
};
HostLayout host_layout(const Plan& pl) {
  HostLayout h;
  const size_t slots = size_t(pl.B) * pl.Z;
  h.off_rec[0] = 0;
  h.off_rec[1] = align_up(slots * pl.rec);
  h.off_tag[0] = h.off_rec[1] + align_up(slots * pl.rec);
  h.off_tag[1] = h.off_tag[0] + align_up(slots * 4);
  h.total = h.off_tag[1] + align_up(slots * 4);
  return h;
}

// Device workspace: status word, ticket and block counts; bin loads; chunk
// offsets of the block scan and the finish's tie flag; the external sort's
// error word; then the staging area.
struct DevLayout {
  size_t off_status, off_loads, off_coff, off_err, off_stage, stage;
};
constexpr size_t kOocMinStage = size_t(16) << 20;
DevLayout dev_layout(const Plan& pl, size_t dws_bytes) {
  DevLayout d;
  d.off_status = 0;
  d.off_loads = align_up(16 + size_t(pl.nblocks_last) * 8);
  d.off_coff = d.off_loads + align_up(size_t(pl.B) * 4);
  d.off_err = d.off_coff + align_up((size_t(pl.nblocks_last) / kScanChunk + 2) * 8);
  d.off_stage = d.off_err + align_up(8);  // the OR of the external sort's error words
  d.stage = dws_bytes > d.off_stage ? dws_bytes - d.off_stage : 0;
  return d;
}

bos_status ooc_streams(OocStreams** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kOocDevices) return BOS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_ooc_mu);
  OocStreams& o = g_ooc[dev];
  if (!o.st[0]) {
    // default priority (no priority variants)
    for (int i = 0; i < 3; ++i)
      if (hipStreamCreateWithFlags(&o.st[i], hipStreamNonBlocking) != hipSuccess) return BOS_ERR_HIP;
    if (hipEventCreateWithFlags(&o.ev, hipEventDisableTiming) != hipSuccess) return BOS_ERR_HIP;
    for (int b = 0; b < 2; ++b)
      if (hipEventCreateWithFlags(&o.ev_in[b], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&o.ev_k[b], hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&o.ev_out[b], hipEventDisableTiming) != hipSuccess)
        return BOS_ERR_HIP;
  }
  *out = &o;
  return BOS_OK;
}

uint64_t pow2_floor(uint64_t x) {
  uint64_t p = 1;
  while (p * 2 <= x) p *= 2;
  return x ? p : 0;
}
uint32_t log2u(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

hipError_t h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
  return bytes ? hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
}
hipError_t d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
  return bytes ? hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s) : hipSuccess;
}
hipError_t sync3(OocStreams* o) {
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = hipStreamSynchronize(o->st[i]);
  return e;
}

// One chunk of a pipelined loop over staging set b = chunk mod 2: its input
// copies go on in() (which first waits until the set's previous output copy
// has left), its kernels on kernels() (after the input copies), its output
// copies on out() (after the kernels), and done() marks the set free again.
// Every loop ends with sync3.
struct OocPipe {
  OocStreams* o;
  int b = 0;
  hipError_t start(uint64_t chunk, hipStream_t* s) {
    b = int(chunk & 1u);
    *s = o->st[0];
    return chunk >= 2 ? hipStreamWaitEvent(o->st[0], o->ev_out[b], 0) : hipSuccess;
  }
  hipError_t kernels(hipStream_t* s) {
    *s = o->st[1];
    hipError_t e = hipEventRecord(o->ev_in[b], o->st[0]);
    return e == hipSuccess ? hipStreamWaitEvent(o->st[1], o->ev_in[b], 0) : e;
  }
  hipError_t out(hipStream_t* s) {
    *s = o->st[2];
    hipError_t e = hipEventRecord(o->ev_k[b], o->st[1]);
    return e == hipSuccess ? hipStreamWaitEvent(o->st[2], o->ev_k[b], 0) : e;
  }
  hipError_t done() { return hipEventRecord(o->ev_out[b], o->st[2]); }
};

// One attempt's routing passes, chunk by chunk (the last in split form: bins
// compacted into host slot array (P - 1) & 1, loads and block counts on the
// device).
hipError_t ooc_route(const Plan& pl, const bos_params& q, uint32_t attempt, const char* in, char* hws,
                     const HostLayout& hl, char* dws, const DevLayout& dl, OocStreams* o) {
  const int R = pl.rec;
  unsigned long long* status = reinterpret_cast<unsigned long long*>(dws + dl.off_status);
  hipError_t e = launch_fill_u64(status, 2 + pl.nblocks_last, 0, o->st[0]);
  if (e == hipSuccess) e = launch_fill_u64(status, 1, kNoOverflow, o->st[0]);
  if (e == hipSuccess) e = hipStreamSynchronize(o->st[0]);
  if (e != hipSuccess) return e;
  // staging: two sets of input records, input tags, output records, output tags
  const uint64_t cap = pow2_floor(dl.stage / (4 * size_t(R + 4)));  // slots per buffer
  for (uint32_t t = 0; t < pl.P; ++t) {
    const uint32_t i0 = pl.lev0[t], k = pl.klev[t];
    const bool first = t == 0, last = t + 1 == pl.P;
    const uint64_t items = pl.B >> k, blk_slots = uint64_t(pl.Z) << k;
    const uint64_t cb = std::min<uint64_t>(items, cap / blk_slots);
    const char* hin_rec = hws + hl.off_rec[(t + 1) & 1];
    const char* hin_tag = hws + hl.off_tag[(t + 1) & 1];
    char* hout_rec = hws + hl.off_rec[t & 1];
    char* hout_tag = hws + hl.off_tag[t & 1];
    uint32_t c = 0;
    OocPipe pipe{o};
    for (uint64_t it0 = 0; it0 < items; it0 += cb, ++c) {
      const int b = int(c & 1u);
      hipStream_t s = nullptr;
      e = pipe.start(c, &s);
      if (e != hipSuccess) return e;
      char* set = dws + dl.off_stage + size_t(b) * 2 * cap * (R + 4);
      char* d_in_rec = set;
      uint32_t* d_in_tag = reinterpret_cast<uint32_t*>(set + cap * R);
      char* d_out_rec = set + cap * (R + 4);
      uint32_t* d_out_tag = reinterpret_cast<uint32_t*>(set + cap * (R + 4) + cap * R);
      PassArgs a;
      std::memset(&a, 0, sizeof(a));
      if (first) {
        // groups [it0 2^k, (it0 + cb) 2^k) hold X[x_lo, x_hi)
        const uint64_t j_lo = it0 << k, j_hi = (it0 + cb) << k;
        const uint64_t x_lo = (j_lo * pl.n) >> pl.L, x_hi = (j_hi * pl.n) >> pl.L;
        e = h2d(d_in_rec, in + x_lo * R, (x_hi - x_lo) * R, s);
        a.x_in = d_in_rec;
        a.x_off = x_lo;
      } else {
        const uint64_t g = 1ull << i0, h0 = it0 >> i0;
        a.staged = 1;
        a.in_h0 = h0;
        if (cb >= g) {  // whole groups: one contiguous range of buckets
          const uint64_t slot0 = (h0 << (i0 + k)) << pl.lz, ns = cb * blk_slots;
          e = h2d(d_in_rec, hin_rec + slot0 * R, ns * R, s);
          if (e == hipSuccess) e = h2d(d_in_tag, hin_tag + slot0 * 4, ns * 4, s);
          a.in_r0 = 0;
          a.in_lseg = i0;
        } else {  // inside one group: 2^k segments of cb buckets
          const uint64_t r0 = it0 & (g - 1), seg = cb << pl.lz;
          for (uint64_t m = 0; m < (1ull << k) && e == hipSuccess; ++m) {
            const uint64_t slot0 = ((h0 << (i0 + k)) + (m << i0) + r0) << pl.lz;
            e = h2d(d_in_rec + m * seg * R, hin_rec + slot0 * R, seg * R, s);
            if (e == hipSuccess) e = h2d(d_in_tag + m * seg, hin_tag + slot0 * 4, seg * 4, s);
          }
          a.in_r0 = r0;
          a.in_lseg = log2u(cb);
        }
        a.rec_in = d_in_rec;
        a.tag_in = d_in_tag;
      }
      if (e != hipSuccess) return e;
      const uint64_t out_slot0 = (it0 << k) << pl.lz, ns_out = cb * blk_slots;
      a.rec_out = d_out_rec;
      a.tag_out = d_out_tag;
      a.out_slot0 = out_slot0;
      a.status = status;
      a.ticket = reinterpret_cast<uint32_t*>(status + 1);
      a.scan = status + 2;
      a.n = pl.n;
      a.buckets = pl.B;
      a.seed = q.seed;
      a.z = pl.Z;
      a.lz = pl.lz;
      a.levels = pl.L;
      a.level0 = i0;
      a.klev = k;
      a.attempt = attempt;
      a.fin = 1;
      a.item_off = uint32_t(it0);
      if (last) a.loads = reinterpret_cast<uint32_t*>(dws + dl.off_loads);
      const uint32_t kind = first ? BOS_K_ROUTE_FIRST : last ? BOS_K_ROUTE_LAST : BOS_K_ROUTE_MID;
      const uint64_t slot_bytes = ns_out * (uint64_t(R) + 4);
      e = pipe.kernels(&s);
      if (e != hipSuccess) return e;
      prof_begin(kind, t, slot_bytes * 2, s);
      e = launch_route(R, a, first, last, uint32_t(cb), num_cus(), s, last);
      prof_end(s);
      if (e == hipSuccess) e = pipe.out(&s);
      if (e == hipSuccess) e = d2h(hout_rec + out_slot0 * R, d_out_rec, ns_out * R, s);
      if (e == hipSuccess && !last) e = d2h(hout_tag + out_slot0 * 4, d_out_tag, ns_out * 4, s);
      if (e == hipSuccess) e = pipe.done();
      if (e != hipSuccess) return e;
    }
    e = sync3(o);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Output offset of every routing block (exclusive scan of the block counts),
// read back to the host.
hipError_t ooc_block_offsets(const Plan& pl, char* dws, const DevLayout& dl, hipStream_t s,
                             std::vector<uint64_t>* boff) {
  unsigned long long* scan = reinterpret_cast<unsigned long long*>(dws + dl.off_status) + 2;
  unsigned long long* coff = reinterpret_cast<unsigned long long*>(dws + dl.off_coff);
  const uint32_t nb = pl.nblocks_last, nch = (nb + kScanChunk - 1) / kScanChunk;
  hipError_t e = launch_block_scan(scan, coff, nb, s);
  std::vector<uint64_t> sc(nb), co(nch);
  if (e == hipSuccess) e = d2h(sc.data(), scan, size_t(nb) * 8, s);
  if (e == hipSuccess) e = d2h(co.data(), coff, size_t(nch) * 8, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  boff->resize(size_t(nb) + 1);
  for (uint32_t b = 0; b < nb; ++b) (*boff)[b] = sc[b] + co[b / kScanChunk];
  (*boff)[nb] = pl.n;
  return hipSuccess;
}

// bos_orp's per-bin finish, or bos_sort's strip (into `dst`, host), over
// chunks of whole routing blocks.
hipError_t ooc_finish(const Plan& pl, const bos_params& q, uint32_t attempt, bool sort, char* dst, char* hws,
                      const HostLayout& hl, char* dws, const DevLayout& dl, OocStreams* o,
                      const std::vector<uint64_t>& boff) {
  const int R = pl.rec;
  const uint32_t klast = pl.klev[pl.P - 1];
  const char* binned = hws + hl.off_rec[(pl.P - 1) & 1];
  unsigned long long* scan = reinterpret_cast<unsigned long long*>(dws + dl.off_status) + 2;
  unsigned long long* coff = reinterpret_cast<unsigned long long*>(dws + dl.off_coff);
  unsigned long long* tie = coff + pl.nblocks_last / kScanChunk + 1;
  const uint32_t* loads = reinterpret_cast<const uint32_t*>(dws + dl.off_loads);
  hipError_t e = hipSuccess;
  if (!sort) {
    e = launch_fill_u64(tie, 1, (q.flags & BOS_EXACT_FINISH) ? 1ull : 0ull, o->st[0]);
    if (e == hipSuccess) e = hipStreamSynchronize(o->st[0]);
    if (e != hipSuccess) return e;
  }
  // two sets of (bin slots, output records)
  const uint64_t cap = pow2_floor(dl.stage / (4 * size_t(R)));
  const uint64_t bslots = uint64_t(pl.Z) << klast;  // slots per routing block
  const uint64_t cblk = std::min<uint64_t>(pl.nblocks_last, cap / bslots);
  uint32_t c = 0;
  OocPipe pipe{o};
  for (uint64_t b0 = 0; b0 < pl.nblocks_last; b0 += cblk, ++c) {
    const uint64_t b1 = std::min<uint64_t>(b0 + cblk, pl.nblocks_last);
    const int sb = int(c & 1u);
    hipStream_t s = nullptr;
    e = pipe.start(c, &s);
    if (e != hipSuccess) return e;
    char* d_bin = dws + dl.off_stage + size_t(sb) * 2 * cap * R;
    char* d_out = d_bin + cap * R;
    const uint64_t slot0 = b0 * bslots, out0 = boff[b0], out1 = boff[b1];
    e = h2d(d_bin, binned + slot0 * R, (b1 - b0) * bslots * R, s);
    if (e == hipSuccess) e = pipe.kernels(&s);
    if (e != hipSuccess) return e;
    if (sort) {
      prof_begin(BOS_K_STRIP, c, 2 * (out1 - out0) * R, s);
      e = launch_strip_staged(R, d_bin, loads, scan, coff, d_out, pl.n, klast, pl.lz, pl.tile, b0, uint32_t(b1 - b0),
                              slot0, out0, s);
    } else {
      FinishArgs f;
      std::memset(&f, 0, sizeof(f));
      f.binned = d_bin;
      f.loads = loads;
      f.boff = scan;
      f.coff = coff;
      f.out = d_out;
      f.n = pl.n;
      f.nbins = pl.B;
      f.seed = q.seed;
      f.klev = klast;
      f.attempt = attempt;
      f.tie = tie;
      f.gb_lo = b0 << klast;
      f.gb_hi = b1 << klast;
      f.bin_slot0 = slot0;
      f.out0 = out0;
      prof_begin(BOS_K_ORP_FINISH, c, 2 * (out1 - out0) * R, s);
      e = launch_orp_finish(R, pl.lz, f, num_cus(), s);
    }
    prof_end(s);
    if (e == hipSuccess) e = pipe.out(&s);
    if (e == hipSuccess) e = d2h(dst + out0 * R, d_out, (out1 - out0) * R, s);
    if (e == hipSuccess) e = pipe.done();
    if (e != hipSuccess) return e;
  }
  return sync3(o);
}

// Unsigned lexicographic (key, payload) order of two host records.
bool host_rec_less(const char* a, const char* b, int R) {
  if (R == 8) {
    uint32_t ka, kb, pa, pb;
    std::memcpy(&ka, a, 4);
    std::memcpy(&kb, b, 4);
    if (ka != kb) return ka < kb;
    std::memcpy(&pa, a + 4, 4);
    std::memcpy(&pb, b + 4, 4);
    return pa < pb;
  }
  uint64_t ka, kb, pa, pb;
  std::memcpy(&ka, a, 8);
  std::memcpy(&kb, b, 8);
  if (ka != kb) return ka < kb;
  std::memcpy(&pa, a + 8, 8);
  std::memcpy(&pb, b + 8, 8);
  return pa < pb;
}

// Comparison phase of the out-of-core sort (Section 3.3 applied to host
// arrays): the permuted records in `a` (host, n records) are sorted into
// `out` (host).  Runs of rl records (a multiple of the tile, so their tile
// sorts cover the tiles the strip prepared) are sorted on the device in
// place; then every q-th record of each run is a sample, the samples are
// ordered by (record, run, position), every t-th opens an output segment, and
// each run is cut at each splitter by binary search (a total order, so equal
// records split consistently).  A segment holds at most t q + m (q - 1) <= rl
// records; its run slices are gathered, sorted on the device and written to
// their place in `out`.  Every access depends on comparisons of the permuted
// records only.
bos_status ooc_comparison_sort(const Plan& pl, char* a, char* out, char* dws, const DevLayout& dl, OocStreams* o) {
  const int R = pl.rec;
  const uint64_t n = pl.n;
  // two sets of (buffer, buffer, merge splits) of rl records
  uint64_t rl = pow2_floor(dl.stage / 2 / (2 * size_t(R)));
  while (rl >= pl.tile && 2 * (align_up(2 * rl * R) + align_up(comparison_sort_split_bytes(rl, R))) > dl.stage)
    rl /= 2;
  if (rl < pl.tile || rl < 2) return BOS_ERR_WORKSPACE;
  const size_t set_bytes = align_up(2 * rl * R) + align_up(comparison_sort_split_bytes(rl, R));
  unsigned long long* err = reinterpret_cast<unsigned long long*>(dws + dl.off_err);
  auto sort_on_device = [&](int sb, uint64_t len, hipStream_t s, void** result) -> hipError_t {
    char* set = dws + dl.off_stage + size_t(sb) * set_bytes;
    uint64_t* split = reinterpret_cast<uint64_t*>(set + align_up(2 * rl * R));
    *result = set;
    if (len <= 1) return hipSuccess;
    hipError_t e = launch_comparison_sort(R, set, set + rl * R, len, pl.tile, split, s, result, true);
    if (e == hipSuccess) e = launch_or_u64(err, comparison_sort_err_word(split, len, R), s);
    return e;
  };
  hipError_t e = launch_fill_u64(err, 1, 0ull, o->st[0]);
  if (e == hipSuccess) e = hipStreamSynchronize(o->st[0]);
  if (e != hipSuccess) return BOS_ERR_HIP;
  const uint64_t m = (n + rl - 1) / rl;
  char* dst_runs = m == 1 ? out : a;  // a single run goes straight to out
  OocPipe pipe{o};
  for (uint64_t r = 0; r < m; ++r) {
    const int sb = int(r & 1u);
    hipStream_t s = nullptr;
    const uint64_t len = std::min(rl, n - r * rl);
    char* set = dws + dl.off_stage + size_t(sb) * set_bytes;
    void* result = nullptr;
    e = pipe.start(r, &s);
    if (e == hipSuccess) e = h2d(set, a + r * rl * R, len * R, s);
    if (e == hipSuccess) e = pipe.kernels(&s);
    if (e == hipSuccess) e = sort_on_device(sb, len, s, &result);
    if (e == hipSuccess) e = pipe.out(&s);
    if (e == hipSuccess) e = d2h(dst_runs + r * rl * R, result, len * R, s);
    if (e == hipSuccess) e = pipe.done();
    if (e != hipSuccess) return BOS_ERR_HIP;
  }
  if (sync3(o) != hipSuccess) return BOS_ERR_HIP;
  if (m > 1) {
    // samples every q records of every run, q the largest power of two with m q <= rl / 2
    uint64_t q = pow2_floor(rl / (2 * m));
    if (q == 0) return BOS_ERR_WORKSPACE;
    struct Smp {
      const char* p;
      uint64_t run, pos;
    };
    std::vector<Smp> smp;
    for (uint64_t r = 0; r < m; ++r) {
      const uint64_t len = std::min(rl, n - r * rl);
      for (uint64_t i = 0; i < len; i += q) smp.push_back(Smp{a + (r * rl + i) * R, r, i});
    }
    std::sort(smp.begin(), smp.end(), [&](const Smp& x, const Smp& y) {
      if (host_rec_less(x.p, y.p, R)) return true;
      if (host_rec_less(y.p, x.p, R)) return false;
      return x.run != y.run ? x.run < y.run : x.pos < y.pos;
    });
    const uint64_t t = (rl - m * q) / q;
    // cut[j * m + r]: first position of run r in segment j
    std::vector<uint64_t> cut;
    for (uint64_t r = 0; r < m; ++r) cut.push_back(0);
    for (uint64_t si = t; si < smp.size(); si += t) {
      const Smp& sp = smp[si];
      for (uint64_t r = 0; r < m; ++r) {
        const char* run = a + r * rl * R;
        const uint64_t len = std::min(rl, n - r * rl);
        uint64_t pos;
        if (r == sp.run) {
          pos = sp.pos;
        } else {
          // records before (sp, run, pos) in the order (record, run, position)
          uint64_t lo = 0, hi = len;
          while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            const char* x = run + mid * R;
            const bool before = r < sp.run ? !host_rec_less(sp.p, x, R) : host_rec_less(x, sp.p, R);
            if (before)
              lo = mid + 1;
            else
              hi = mid;
          }
          pos = lo;
        }
        cut.push_back(pos);
      }
    }
    for (uint64_t r = 0; r < m; ++r) cut.push_back(std::min(rl, n - r * rl));
    const uint64_t nseg = cut.size() / m - 1;
    uint64_t base = 0;
    OocPipe spipe{o};
    for (uint64_t j = 0; j < nseg; ++j) {
      const int sb = int(j & 1u);
      hipStream_t s = nullptr;
      char* set = dws + dl.off_stage + size_t(sb) * set_bytes;
      uint64_t len = 0;
      e = spipe.start(j, &s);
      for (uint64_t r = 0; r < m && e == hipSuccess; ++r) {
        const uint64_t c0 = cut[j * m + r], c1 = cut[(j + 1) * m + r];
        if (c1 < c0 || len + (c1 - c0) > rl) return BOS_ERR_INTERNAL;  // the segment bound above
        e = h2d(set + len * R, a + (r * rl + c0) * R, (c1 - c0) * R, s);
        len += c1 - c0;
      }
      void* result = nullptr;
      if (e == hipSuccess) e = spipe.kernels(&s);
      if (e == hipSuccess) e = sort_on_device(sb, len, s, &result);
      if (e == hipSuccess) e = spipe.out(&s);
      if (e == hipSuccess) e = d2h(out + base * R, result, len * R, s);
      if (e == hipSuccess) e = spipe.done();
      if (e != hipSuccess) return BOS_ERR_HIP;
      base += len;
    }
    if (base != n) return BOS_ERR_INTERNAL;
    if (sync3(o) != hipSuccess) return BOS_ERR_HIP;
  }
  unsigned long long eh = 0;
  if (d2h(&eh, err, 8, o->st[0]) != hipSuccess || hipStreamSynchronize(o->st[0]) != hipSuccess) return BOS_ERR_HIP;
  return eh ? BOS_ERR_INTERNAL : BOS_OK;
}

bos_status ooc_impl(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* hws,
                    size_t hws_bytes, void* dws, size_t dws_bytes, void* stream, bos_report* rep, bool sort) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  bos_params q = resolve(p);
  q.flags |= BOS_SYNC;
  Plan pl;
  bos_status st = make_plan(n, int(rec), q, true, &pl, kMaxNHost);
  if (st != BOS_OK) return st;
  if (n == 0) {
    fill_report(rep, pl, 0, kNoOverflow, 0);
    return BOS_OK;
  }
  if (!in || !out || in == out) return BOS_ERR_INVALID_ARG;
  if (!split_last(pl)) return BOS_ERR_UNSUPPORTED;  // one routing pass: the in-core calls cover it
  for (uint32_t t = 0; t < pl.P; ++t)
    if (!use_route_kernel(pl, t)) return BOS_ERR_UNSUPPORTED;
  const HostLayout hl = host_layout(pl);
  if (!hws || hws_bytes < hl.total) return BOS_ERR_WORKSPACE;
  const DevLayout dl = dev_layout(pl, dws_bytes);
  const uint64_t blk_max = uint64_t(pl.Z) << pl.k;
  if (!dws || dl.stage < kOocMinStage || dl.stage < 4 * blk_max * (uint64_t(pl.rec) + 4)) return BOS_ERR_WORKSPACE;
  OocStreams* o = nullptr;
  st = ooc_streams(&o);
  if (st != BOS_OK) return st;
  // order after the caller's stream
  hipStream_t cs = static_cast<hipStream_t>(stream);
  if (hipEventRecord(o->ev, cs) != hipSuccess || hipStreamWaitEvent(o->st[0], o->ev, 0) != hipSuccess ||
      hipStreamWaitEvent(o->st[1], o->ev, 0) != hipSuccess || hipStreamWaitEvent(o->st[2], o->ev, 0) != hipSuccess)
    return BOS_ERR_HIP;
  char* h = static_cast<char*>(hws);
  char* d = static_cast<char*>(dws);
  uint32_t attempts = 0;
  uint64_t ovf = kNoOverflow, last_ovf = kNoOverflow;
  bool ok = false;
  uint32_t att = q.attempt;
  for (; att <= std::max(q.max_retries, q.attempt); ++att) {
    if (ooc_route(pl, q, att, static_cast<const char*>(in), h, hl, d, dl, o) != hipSuccess) return BOS_ERR_HIP;
    attempts = att + 1;
    uint64_t sw = 0;
    if (d2h(&sw, d + dl.off_status, 8, o->st[0]) != hipSuccess || hipStreamSynchronize(o->st[0]) != hipSuccess)
      return BOS_ERR_HIP;
    if (sw == kNoOverflow) {
      ok = true;
      ovf = last_ovf;
      break;
    }
    last_ovf = sw;
  }
  if (!ok) {
    fill_report(rep, pl, attempts, last_ovf, 0);
    return BOS_ERR_OVERFLOW;
  }
  std::vector<uint64_t> boff;
  if (ooc_block_offsets(pl, d, dl, o->st[0], &boff) != hipSuccess) return BOS_ERR_HIP;
  if (!sort) {
    if (ooc_finish(pl, q, att, false, static_cast<char*>(out), h, hl, d, dl, o, boff) != hipSuccess)
      return BOS_ERR_HIP;
    fill_report(rep, pl, attempts, ovf, 0);
    return BOS_OK;
  }
  // strip into the tag arrays (dead after routing), then the comparison phase
  char* a = h + hl.off_tag[0];
  if (ooc_finish(pl, q, att, true, a, h, hl, d, dl, o, boff) != hipSuccess) return BOS_ERR_HIP;
  st = ooc_comparison_sort(pl, a, static_cast<char*>(out), d, dl, o);
  fill_report(rep, pl, attempts, ovf, 6 * n * uint64_t(pl.rec));
  return st;
}

}  // namespace

extern "C" {

size_t bos_host_workspace_bytes(uint64_t n, bos_rec rec, const bos_params* p) {
  if (!has_gpu()) return 0;
  Plan pl;
  bos_params q = resolve(p);
  q.min_security_bits = 0;
  if (make_plan(n, int(rec), q, true, &pl, kMaxNHost) != BOS_OK) return 0;
  return host_layout(pl).total;
}

size_t bos_host_device_bytes(uint64_t n, bos_rec rec, const bos_params* p) {
  if (!has_gpu()) return 0;
  Plan pl;
  bos_params q = resolve(p);
  q.min_security_bits = 0;
  if (make_plan(n, int(rec), q, true, &pl, kMaxNHost) != BOS_OK) return 0;
  const DevLayout dl = dev_layout(pl, 0);
  const uint64_t blk_max = uint64_t(pl.Z) << pl.k;
  return dl.off_stage + std::max<size_t>(kOocMinStage, 4 * blk_max * (size_t(pl.rec) + 4));
}

bos_status bos_orp_host(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* host_ws,
                        size_t host_ws_bytes, void* dev_ws, size_t dev_ws_bytes, void* stream, bos_report* rep) {
  return ooc_impl(in, out, n, rec, p, host_ws, host_ws_bytes, dev_ws, dev_ws_bytes, stream, rep, false);
}

bos_status bos_sort_host(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* host_ws,
                         size_t host_ws_bytes, void* dev_ws, size_t dev_ws_bytes, void* stream, bos_report* rep) {
  return ooc_impl(in, out, n, rec, p, host_ws, host_ws_bytes, dev_ws, dev_ws_bytes, stream, rep, true);
}

}  // extern "C"
