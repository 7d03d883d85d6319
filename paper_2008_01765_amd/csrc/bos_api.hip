// bos_api.hip — planner, launch sequencing and the C ABI of libbos (include/bos.h).
//
// Planner (Algorithm 3.1): B = smallest power of two >= 2n/Z, L = log2 B; the
// L levels are cut into passes of at most k levels (k fused levels = 2^k
// buckets per block, bounded by LDS); the workspace holds two slot arrays
// (records + 4-byte tags, ping-pong), the overflow status word and the
// look-back words of the strip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "bos.h"
#include "bos_common.h"
#include "bos_prof.h"

namespace bos {
hipError_t launch_fill_u64(unsigned long long* p, uint64_t count, unsigned long long v, hipStream_t s);
hipError_t launch_labels(uint32_t* out, uint64_t n, uint32_t L, uint64_t seed, uint32_t attempt, hipStream_t s);
hipError_t launch_pass(int rec, const PassArgs& a, bool first, bool last, uint32_t nblocks, hipStream_t s);
hipError_t launch_route(int rec, const PassArgs& a, bool first, bool last, uint32_t nitems, uint32_t grid,
                        hipStream_t s);
hipError_t launch_comparison_sort(int rec, void* buf0, void* buf1, uint64_t n, uint32_t ts, uint64_t* split,
                                  hipStream_t s, void** result);
uint32_t comparison_sort_passes(uint64_t n, uint32_t ts);
size_t comparison_sort_split_bytes(uint64_t n);
hipError_t launch_bitonic(int rec, const void* in, void* out, uint64_t n, void* ws, uint64_t N, uint32_t ts,
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
constexpr uint32_t kBitonicTile = 8192;
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
  uint64_t n = 0, B = 1;
  int rec = 8;
  uint32_t Z = 512, lz = 9, L = 0, P = 1, k = 0, tile = kDefaultTile;
  uint32_t klev[kMaxPasses] = {0}, lev0[kMaxPasses] = {0};
  size_t off_rec[2] = {0, 0}, off_tag[2] = {0, 0}, off_status = 0, off_scan = 0, off_split = 0, total = 0;
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
  if (q.z == 0) q.z = 512;
  return q;
}

// Largest k such that a block of 2^k buckets fits in LDS and in 512 threads.
uint32_t max_klev(int rec, uint32_t z, bool last_shuffle) {
  uint32_t best = 0;
  for (uint32_t k = 1; k <= 12; ++k) {
    const uint64_t m = uint64_t(z) << k;
    if (m / 16 > uint64_t(kMaxThreads)) break;
    if (pass_lds_bytes(rec, z, k, last_shuffle) > lds_max()) break;
    best = k;
  }
  return best;
}

bos_status make_plan(uint64_t n, int rec, const bos_params& q, bool shuffle_last, Plan* pl) {
  if (rec != 8 && rec != 16) return BOS_ERR_INVALID_ARG;
  if (n > kMaxN) return BOS_ERR_INVALID_ARG;
  const uint32_t Z = q.z;
  if (Z < 8 || Z > 2048 || (Z & (Z - 1))) return BOS_ERR_INVALID_ARG;
  pl->n = n;
  pl->rec = rec;
  pl->Z = Z;
  pl->generic = (q.flags & BOS_GENERIC_ROUTING) != 0;
  pl->lz = 0;
  while ((1u << pl->lz) < Z) ++pl->lz;
  uint64_t B = 1;
  uint32_t L = 0;
  while (B * Z < 2 * n) {
    B *= 2;
    ++L;
  }
  if (L > 31) return BOS_ERR_INVALID_ARG;
  pl->B = B;
  pl->L = L;
  // Lemma 3.2: overflow probability <= B log2 B e^(-Z/6)
  if (q.min_security_bits && L > 0) {
    const double log2eps = double(L) + std::log2(double(L)) - double(Z) / (6.0 * std::log(2.0));
    if (log2eps > -double(q.min_security_bits)) return BOS_ERR_INSECURE_Z;
  }
  const uint32_t kmid = max_klev(rec, Z, false), klast = max_klev(rec, Z, shuffle_last);
  if (kmid == 0 || klast == 0) return BOS_ERR_UNSUPPORTED;
  uint32_t k = q.k ? std::min(q.k, kmid) : std::min(4u, kmid);
  pl->k = k;
  pl->tile = q.tile ? q.tile : kDefaultTile;
  if (pl->tile != kDefaultTile) return BOS_ERR_INVALID_ARG;  // the tile sort is built for 4096
  if (L == 0) {
    pl->P = 1;
    pl->klev[0] = 0;
    pl->lev0[0] = 0;
  } else {
    uint32_t P = (L + k - 1) / k;
    for (;; ++P) {
      if (P > kMaxPasses) return BOS_ERR_UNSUPPORTED;
      const uint32_t base = L / P, extra = L % P;
      // passes 0..extra-1 get base+1 levels, the rest base; the last gets base
      // (or base+1 if P == extra, impossible since extra < P)
      const uint32_t last_lv = base;
      if (base + (extra ? 1 : 0) <= k && last_lv <= klast && last_lv >= 1) {
        uint32_t lv = 0;
        for (uint32_t t = 0; t < P; ++t) {
          pl->klev[t] = base + (t < extra ? 1 : 0);
          pl->lev0[t] = lv;
          lv += pl->klev[t];
        }
        pl->P = P;
        break;
      }
      if (base == 0) return BOS_ERR_UNSUPPORTED;
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
  off = align_up(off + comparison_sort_split_bytes(n));
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

// Enqueue one attempt of the routing phase; `out` receives the stripped bins.
hipError_t enqueue_routing(const Plan& pl, const void* in, void* out, uint64_t seed, uint32_t attempt,
                           uint32_t fin, char* ws, hipStream_t s, int stop_after = -1) {
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
    a.fin = fin;
    const uint64_t slot_bytes = pl.B * pl.Z * (uint64_t(pl.rec) + 4), rec_bytes = pl.n * pl.rec;
    const uint32_t kind = first && last ? BOS_K_ROUTE_SINGLE
                          : first       ? BOS_K_ROUTE_FIRST
                          : last        ? BOS_K_ROUTE_LAST
                                        : BOS_K_ROUTE_MID;
    const uint64_t bytes = (first ? rec_bytes : slot_bytes) + (last ? rec_bytes : slot_bytes);
    prof_begin(kind, t, bytes, s);
    const uint32_t nitems = uint32_t(pl.B >> pl.klev[t]);
    if (use_route_kernel(pl, t))
      e = launch_route(pl.rec, a, first, last, nitems, num_cus(), s);
    else
      e = launch_pass(pl.rec, a, first, last, nitems, s);
    prof_end(s);
    if (e != hipSuccess) return e;
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
                       hipStream_t s, uint32_t* attempts_out, uint64_t* ovf_out) {
  uint64_t last_ovf = kNoOverflow;
  const uint32_t tries = (q.flags & BOS_SYNC) ? q.max_retries + 1 : 1;
  for (uint32_t att = 0; att < tries; ++att) {
    hipError_t e = enqueue_routing(pl, in, out, q.seed, att, fin, ws, s);
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
  st = run_routing(pl, q, in, out, 0, static_cast<char*>(ws), static_cast<hipStream_t>(stream), &attempts, &ovf);
  fill_report(rep, pl, attempts, ovf, 0);
  return st;
}

bos_status bos_sort(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* ws,
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
  // The comparison sort ping-pongs between `out` and slot array 0 (free once
  // the routing phase is over); the routing output goes where the sort must
  // start so that the result lands in `out`.
  const uint32_t passes = comparison_sort_passes(n, pl.tile);
  // the last routing pass reads slot array P & 1; the other one is free
  void* tmp = w + pl.off_rec[(pl.P + 1) & 1];
  void* start = (passes % 2 == 0) ? out : tmp;
  void* other = (passes % 2 == 0) ? tmp : out;
  uint32_t attempts = 0;
  uint64_t ovf = kNoOverflow;
  st = run_routing(pl, q, in, start, 1, w, s, &attempts, &ovf);
  if (st != BOS_OK) {
    fill_report(rep, pl, attempts, ovf, 0);
    return st;
  }
  void* result = nullptr;
  hipError_t e = launch_comparison_sort(pl.rec, start, other, n, pl.tile,
                                        reinterpret_cast<uint64_t*>(w + pl.off_split), s, &result);
  if (e != hipSuccess) return BOS_ERR_HIP;
  if (result != out) {
    e = hipMemcpyAsync(out, result, n * pl.rec, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return BOS_ERR_HIP;
  }
  if (q.flags & BOS_SYNC) {
    if (hipStreamSynchronize(s) != hipSuccess) return BOS_ERR_HIP;
  }
  fill_report(rep, pl, attempts, ovf, uint64_t(2 + 2 * passes) * n * pl.rec);
  return BOS_OK;
}

size_t bos_batched_workspace_bytes(const uint64_t* n, uint32_t count, bos_rec rec, const bos_params* p) {
  size_t mx = 0;
  for (uint32_t i = 0; i < count; ++i) mx = std::max(mx, bos_workspace_bytes(n[i], rec, p));
  return mx;
}

bos_status bos_sort_batched(const bos_instance* inst, uint32_t count, bos_rec rec, const bos_params* p,
                            void* ws, size_t ws_bytes, void* stream, uint32_t* d_status, bos_report* rep) {
  if (!has_gpu()) return BOS_ERR_UNSUPPORTED;
  if (count && !inst) return BOS_ERR_INVALID_ARG;
  bos_params q = resolve(p);
  bos_status worst = BOS_OK;
  uint64_t bytes = 0;
  uint32_t attempts = 0;
  std::vector<uint32_t> host_status(count, BOS_OK);
  for (uint32_t i = 0; i < count; ++i) {
    q.seed = inst[i].seed;
    bos_report r;
    const bos_status st = bos_sort(inst[i].in, inst[i].out, inst[i].n, rec, &q, ws, ws_bytes, stream, &r);
    host_status[i] = st;
    if (st != BOS_OK && worst == BOS_OK) worst = st;
    bytes += r.algorithmic_bytes;
    attempts += r.attempts;
  }
  if (d_status && count) {
    if (hipMemcpyAsync(d_status, host_status.data(), count * 4, hipMemcpyHostToDevice,
                       static_cast<hipStream_t>(stream)) != hipSuccess ||
        hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess)
      return BOS_ERR_HIP;
  }
  if (rep) {
    std::memset(rep, 0, sizeof(*rep));
    rep->attempts = attempts;
    rep->z = q.z;
    rep->algorithmic_bytes = bytes;
    rep->first_overflow_level = -1;
    rep->first_overflow_pair = -1;
  }
  return worst;
}

size_t bos_bitonic_workspace_bytes(uint64_t n, bos_rec rec) {
  if (rec != 8 && rec != 16) return 0;
  uint64_t N = kBitonicTile;
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
  uint64_t N = kBitonicTile;
  while (N < n) N <<= 1;
  return hip_status(launch_bitonic(int(rec), in, out, n, ws, N, kBitonicTile, static_cast<hipStream_t>(stream)));
}

void bos_release_cache(void) {}

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
