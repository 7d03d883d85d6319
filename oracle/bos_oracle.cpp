/*
 * bos_oracle.cpp — plain single-threaded CPU oracle for bucket ORP and bucket
 * oblivious sort (Asharov et al., SOSA 2020).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  Shares no code
 * with the GPU library.
 *
 * The code follows the paper in its own order:
 *   plan            Algorithm 3.1 (choice of Z and B), Section 3.1
 *   labels          Algorithm 3.1 (every element draws its destination bin uniformly)
 *   placement       Algorithm 3.1 (B even groups, padded with dummies to Z)
 *   butterfly       Algorithm 3.1 (levels i, pairs j, MergeSplit, overflow abort)
 *   ORP finish      Section 3.2 (delete dummies, permute each bin, concatenate)
 *   sort            Section 3.3 (ORP, then a non-oblivious comparison sort)
 *   access counts   Section 3.4 / Section 2 (one block read or write = 1 access)
 *
 * Readings taken where the paper leaves a choice open:
 *   - B = 1 when 2n <= Z (no levels); groups are the balanced floor split
 *     [floor(jn/B), floor((j+1)n/B)).
 *   - Level i routes by the label bit that is i+1 places from the top, that is
 *     bit L-1-i of the L-bit label, so the final bin index equals the label.
 *   - MergeSplit appends real elements in scan order (A0's slots, then A1's),
 *     so its outputs are stable; the paper defines them as sets.
 *   - Overflow means strictly more than Z real elements in an output bucket.
 *     After an overflow the attempt is abandoned and the next attempt draws
 *     fresh labels (overflow depends on the labels only, never on the data).
 *   - Labels and per-bin permutation keys come from Philox4x64-10; see
 *     bos_oracle_label and bos_oracle_shuffle_key.
 *   - The random permutation of each bin: the bin's real elements are put in record
 *     order (key, payload), the p-th of them receives the 64-bit random key
 *     r(b*Z + p), and they are sorted by (r, p).  This is a uniformly random
 *     ordering of the bin (up to 64-bit key ties, broken by p) that does not
 *     depend on the order in which the butterfly delivered the elements.
 */
#include "bos_oracle.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

namespace {

struct Rec {
  uint64_t key;
  uint64_t payload;
};

bool rec_less(const Rec& a, const Rec& b) {
  if (a.key != b.key) return a.key < b.key;
  return a.payload < b.payload;
}

Rec load_rec(const uint8_t* base, uint32_t rec, uint64_t idx) {
  Rec r{0, 0};
  const uint8_t* p = base + idx * rec;
  const uint32_t half = rec / 2;
  std::memcpy(&r.key, p, half);        // little-endian host
  std::memcpy(&r.payload, p + half, half);
  return r;
}

void store_rec(uint8_t* base, uint32_t rec, uint64_t idx, const Rec& r) {
  uint8_t* p = base + idx * rec;
  const uint32_t half = rec / 2;
  std::memcpy(p, &r.key, half);
  std::memcpy(p + half, &r.payload, half);
}

/* One slot of a bucket: a real element (record + label) or a dummy. */
struct Slot {
  bool real;
  uint32_t label;
  Rec r;
};

const Slot kDummy = {false, 0u, {0, 0}};

/* splitmix64 output function (Steele, Lea, Flood 2014), used only to hash the
 * access sequence into a digest. */
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Records the server-memory access sequence (Section 2: op, addr). */
struct Tracer {
  uint64_t* buf = nullptr;
  uint64_t cap = 0;
  uint64_t len = 0;
  uint64_t count = 0;
  uint64_t digest = 0x6A09E667F3BCC909ull;
  void access(bool write, uint32_t arr, uint64_t idx) {
    const uint64_t code = (write ? (1ull << 63) : 0ull) | (uint64_t(arr & 0x7F) << 56) |
                          (idx & ((1ull << 56) - 1));
    if (buf && len < cap) buf[len] = code;
    ++len;
    ++count;
    digest = mix64(digest ^ code);
  }
  void read(uint32_t arr, uint64_t idx) { access(false, arr, idx); }
  void write(uint32_t arr, uint64_t idx) { access(true, arr, idx); }
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

/* The planned B and L, with the optional test override of B applied. */
int plan_with_override(uint64_t n, const bos_oracle_cfg* cfg, uint64_t* B, uint32_t* L) {
  if (bos_oracle_plan(n, cfg->z, B, L) != BOS_ORACLE_OK) return BOS_ORACLE_INVALID;
  if (cfg->b_override) {
    uint64_t b = cfg->b_override;
    if ((b & (b - 1)) != 0 || b < *B) return BOS_ORACLE_INVALID;
    uint32_t l = 0;
    while ((1ull << l) < b) ++l;
    if (l > 31) return BOS_ORACLE_INVALID;
    *B = b;
    *L = l;
  }
  return BOS_ORACLE_OK;
}

/* Labels of one attempt: the caller's override for attempt 0, else Philox. */
void draw_labels(uint64_t n, uint32_t L, uint64_t B, const bos_oracle_cfg* cfg, uint32_t attempt,
                 std::vector<uint32_t>& lab) {
  lab.resize(n);
  for (uint64_t i = 0; i < n; ++i) {
    if (attempt == 0 && cfg->label_override)
      lab[i] = cfg->label_override[i] & uint32_t(B - 1);
    else
      lab[i] = bos_oracle_label(cfg->seed, attempt, i, L);
  }
}

/* Algorithm 3.1, initial placement: group j = X[floor(jn/B), floor((j+1)n/B))
 * goes into A^(0)_j in input order and is padded with dummies to Z slots. */
void place_groups(const uint8_t* X, uint64_t n, uint32_t rec, uint64_t B, uint32_t Z,
                  const std::vector<uint32_t>& lab, std::vector<Slot>& A, Tracer& tr) {
  A.assign(B * Z, kDummy);
  for (uint64_t j = 0; j < B; ++j) {
    const uint64_t lo = j * n / B, hi = (j + 1) * n / B;
    for (uint64_t t = lo; t < hi; ++t) {
      tr.read(BOS_ORACLE_ARR_X, t);
      A[j * Z + (t - lo)] = Slot{true, lab[t], load_rec(X, rec, t)};
    }
    for (uint32_t s = 0; s < Z; ++s) tr.write(BOS_ORACLE_ARR_LEVEL0, j * Z + s);
  }
}

/* Algorithm 3.1, level i: for j = 0..B/2-1, MergeSplit the pair of buckets at
 * distance 2^i starting at j' + j (j' = floor(j / 2^i) * 2^i) of A^(i) into
 * buckets 2j and 2j+1 of A^(i+1).  Returns false on overflow and reports the
 * pair. */
bool butterfly_level(const std::vector<Slot>& A, std::vector<Slot>& Anext, uint64_t B, uint32_t Z,
                     uint32_t L, uint32_t i, Tracer& tr, int64_t* ovf_pair) {
  Anext.assign(B * Z, kDummy);
  const uint32_t in_arr = BOS_ORACLE_ARR_LEVEL0 + i, out_arr = in_arr + 1;
  std::vector<Slot> out0, out1;
  out0.reserve(2 * Z);
  out1.reserve(2 * Z);
  for (uint64_t j = 0; j < B / 2; ++j) {
    const uint64_t jp = (j >> i) << i;
    const uint64_t b0 = jp + j, b1 = jp + j + (1ull << i);
    out0.clear();
    out1.clear();
    // MergeSplit(A0, A1, i): read both input buckets; each real element goes to
    // A'_0 or A'_1 by the (i+1)-st most significant label bit.
    for (uint64_t b : {b0, b1}) {
      for (uint32_t s = 0; s < Z; ++s) {
        tr.read(in_arr, b * Z + s);
        const Slot& x = A[b * Z + s];
        if (!x.real) continue;
        const uint32_t bit = (x.label >> (L - 1 - i)) & 1u;
        (bit ? out1 : out0).push_back(x);
      }
    }
    if (out0.size() > Z || out1.size() > Z) {
      *ovf_pair = int64_t(j);
      return false;
    }
    for (size_t t = 0; t < out0.size(); ++t) Anext[(2 * j) * Z + t] = out0[t];
    for (size_t t = 0; t < out1.size(); ++t) Anext[(2 * j + 1) * Z + t] = out1[t];
    for (uint32_t s = 0; s < Z; ++s) tr.write(out_arr, (2 * j) * Z + s);
    for (uint32_t s = 0; s < Z; ++s) tr.write(out_arr, (2 * j + 1) * Z + s);
  }
  return true;
}

/* Section 3.2: delete the dummies of every final bin, permute each bin at
 * random, concatenate bins 0..B-1 into Y. */
void finish_orp(const std::vector<Slot>& A, uint64_t B, uint32_t Z, uint32_t L, uint64_t seed,
                uint32_t attempt, std::vector<Rec>& Y, Tracer& tr) {
  const uint32_t arr = BOS_ORACLE_ARR_LEVEL0 + L;
  uint64_t off = 0;
  std::vector<Rec> bin;
  std::vector<std::pair<uint64_t, uint64_t>> keyed;  // (r, p)
  for (uint64_t b = 0; b < B; ++b) {
    bin.clear();
    for (uint32_t s = 0; s < Z; ++s) {
      tr.read(arr, b * Z + s);
      if (A[b * Z + s].real) bin.push_back(A[b * Z + s].r);
    }
    // Random permutation of the bin: record order first, then sort by
    // (r(b*Z + p), p).
    std::sort(bin.begin(), bin.end(), rec_less);
    keyed.clear();
    for (uint64_t p = 0; p < bin.size(); ++p)
      keyed.emplace_back(bos_oracle_shuffle_key(seed, attempt, b * Z + p), p);
    std::sort(keyed.begin(), keyed.end());
    for (const auto& kp : keyed) {
      tr.write(BOS_ORACLE_ARR_Y, off);
      Y[off++] = bin[kp.second];
    }
  }
}

/* Runs Algorithm 3.1 followed by the Section 3.2 finish, retrying on overflow.
 * Leaves the permuted records in Y. */
int run_orp(const uint8_t* X, uint64_t n, uint32_t rec, const bos_oracle_cfg* cfg,
            std::vector<Rec>& Y, Tracer& tr, bos_oracle_report* rep) {
  uint64_t B;
  uint32_t L;
  if (plan_with_override(n, cfg, &B, &L) != BOS_ORACLE_OK) return BOS_ORACLE_INVALID;
  const uint32_t Z = cfg->z;
  rep->buckets = B;
  rep->levels = L;
  rep->attempts = 0;
  rep->first_overflow_level = -1;
  rep->first_overflow_pair = -1;
  Y.assign(n, Rec{0, 0});
  if (n == 0) return BOS_ORACLE_OK;

  std::vector<uint32_t> lab;
  std::vector<Slot> A, Anext;
  for (uint32_t attempt = 0; attempt <= cfg->max_retries; ++attempt) {
    rep->attempts = attempt + 1;
    const uint64_t count_before = tr.count;
    auto t0 = std::chrono::steady_clock::now();
    draw_labels(n, L, B, cfg, attempt, lab);
    rep->sec_labels += seconds_since(t0);

    t0 = std::chrono::steady_clock::now();
    place_groups(X, n, rec, B, Z, lab, A, tr);
    bool ok = true;
    for (uint32_t i = 0; i < L && ok; ++i) {
      int64_t pair = -1;
      ok = butterfly_level(A, Anext, B, Z, L, i, tr, &pair);
      if (!ok) {
        rep->first_overflow_level = int32_t(i);
        rep->first_overflow_pair = pair;
      } else {
        A.swap(Anext);
      }
    }
    rep->sec_route += seconds_since(t0);
    if (!ok) continue;

    t0 = std::chrono::steady_clock::now();
    finish_orp(A, B, Z, L, cfg->seed, attempt, Y, tr);
    rep->sec_finish += seconds_since(t0);
    rep->accesses_orp = tr.count - count_before;
    return BOS_ORACLE_OK;
  }
  return BOS_ORACLE_OVERFLOW;
}

/* Bottom-up merge sort by (key, payload) between buffers Y and T (arrays
 * BOS_ORACLE_ARR_Y / _T).  Each pass reads every element once, when it becomes
 * the head of its run, and writes it once.  Returns the buffer holding the
 * result. */
std::vector<Rec>* merge_sort(std::vector<Rec>& Y, std::vector<Rec>& T, Tracer& tr) {
  const uint64_t n = Y.size();
  std::vector<Rec>* src = &Y;
  std::vector<Rec>* dst = &T;
  uint32_t src_arr = BOS_ORACLE_ARR_Y, dst_arr = BOS_ORACLE_ARR_T;
  T.assign(n, Rec{0, 0});
  for (uint64_t w = 1; w < n; w *= 2) {
    for (uint64_t lo = 0; lo < n; lo += 2 * w) {
      const uint64_t mid = std::min(lo + w, n), hi = std::min(lo + 2 * w, n);
      uint64_t a = lo, b = mid;
      if (a < mid) tr.read(src_arr, a);
      if (b < hi) tr.read(src_arr, b);
      for (uint64_t k = lo; k < hi; ++k) {
        const bool take_left = a < mid && (b >= hi || !rec_less((*src)[b], (*src)[a]));
        tr.write(dst_arr, k);
        if (take_left) {
          (*dst)[k] = (*src)[a++];
          if (a < mid) tr.read(src_arr, a);
        } else {
          (*dst)[k] = (*src)[b++];
          if (b < hi) tr.read(src_arr, b);
        }
      }
    }
    std::swap(src, dst);
    std::swap(src_arr, dst_arr);
  }
  return src;
}

void clear_report(bos_oracle_report* rep) { std::memset(rep, 0, sizeof(*rep)); }

bool valid_rec(uint32_t rec) { return rec == 8 || rec == 16; }

}  // namespace

extern "C" {

int bos_oracle_plan(uint64_t n, uint32_t z, uint64_t* buckets, uint32_t* levels) {
  if (z < 2 || (z & 1u)) return BOS_ORACLE_INVALID;
  // B: smallest power of two >= 2n/Z (Algorithm 3.1); B = 1 when 2n <= Z.
  uint64_t B = 1;
  uint32_t L = 0;
  while (B * uint64_t(z) < 2 * n) {
    B *= 2;
    ++L;
    if (L > 31) return BOS_ORACLE_INVALID;
  }
  *buckets = B;
  *levels = L;
  return BOS_ORACLE_OK;
}

void bos_oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  // Philox4x64: two 64x64->128 multiplications per round, multipliers and
  // Weyl key increments as published by Salmon et al. (SC'11), ten rounds.
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    const unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    const uint64_t hi0 = uint64_t(p0 >> 64), lo0 = uint64_t(p0);
    const uint64_t hi1 = uint64_t(p1 >> 64), lo1 = uint64_t(p1);
    const uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

uint32_t bos_oracle_label(uint64_t seed, uint32_t attempt, uint64_t i, uint32_t levels) {
  // Element i takes 32-bit word (i mod 8) of the 256-bit Philox block with
  // counter (floor(i/8), attempt, 0, 0) and key (seed, 0); word 2w is the low
  // half of 64-bit output w.  The label is the top L bits of that word.
  if (levels == 0) return 0;
  const uint64_t ctr[4] = {i / 8, attempt, 0, 0};
  const uint64_t key[2] = {seed, 0};
  uint64_t w[4];
  bos_oracle_philox4x64_10(ctr, key, w);
  const uint32_t j = uint32_t(i % 8);
  const uint32_t word = uint32_t(w[j / 2] >> (32 * (j % 2)));
  return word >> (32 - levels);
}

uint64_t bos_oracle_shuffle_key(uint64_t seed, uint32_t attempt, uint64_t g) {
  // Key g is 64-bit output (g mod 4) of the Philox block with counter
  // (floor(g/4), attempt, 0, 0) and key (seed, 1).
  const uint64_t ctr[4] = {g / 4, attempt, 0, 0};
  const uint64_t key[2] = {seed, 1};
  uint64_t w[4];
  bos_oracle_philox4x64_10(ctr, key, w);
  return w[g % 4];
}

int bos_oracle_orp(const void* in, void* out, uint64_t n, uint32_t rec, const bos_oracle_cfg* cfg,
                   bos_oracle_report* rep) {
  if (!cfg || !rep || !valid_rec(rec) || (n && (!in || !out))) return BOS_ORACLE_INVALID;
  clear_report(rep);
  Tracer tr;
  tr.buf = cfg->trace;
  tr.cap = cfg->trace_cap;
  std::vector<Rec> Y;
  const int rc = run_orp(static_cast<const uint8_t*>(in), n, rec, cfg, Y, tr, rep);
  rep->digest_orp = tr.digest;
  rep->trace_len = tr.len;
  if (rc != BOS_ORACLE_OK) return rc;
  for (uint64_t t = 0; t < n; ++t) store_rec(static_cast<uint8_t*>(out), rec, t, Y[t]);
  return BOS_ORACLE_OK;
}

int bos_oracle_sort(const void* in, void* out, uint64_t n, uint32_t rec, const bos_oracle_cfg* cfg,
                    bos_oracle_report* rep) {
  if (!cfg || !rep || !valid_rec(rec) || (n && (!in || !out))) return BOS_ORACLE_INVALID;
  clear_report(rep);
  Tracer tr;
  tr.buf = cfg->trace;
  tr.cap = cfg->trace_cap;
  std::vector<Rec> Y, T;
  const int rc = run_orp(static_cast<const uint8_t*>(in), n, rec, cfg, Y, tr, rep);
  rep->digest_orp = tr.digest;
  if (rc != BOS_ORACLE_OK) {
    rep->trace_len = tr.len;
    return rc;
  }
  // Section 3.3: a non-oblivious comparison sort of the permuted array.
  Tracer sort_tr;
  sort_tr.buf = tr.buf ? tr.buf + std::min(tr.len, tr.cap) : nullptr;
  sort_tr.cap = tr.buf ? tr.cap - std::min(tr.len, tr.cap) : 0;
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<Rec>* res = merge_sort(Y, T, sort_tr);
  rep->sec_sort = seconds_since(t0);
  rep->accesses_sort = sort_tr.count;
  rep->digest_sort = sort_tr.digest;
  rep->trace_len = tr.len + sort_tr.len;
  for (uint64_t t = 0; t < n; ++t) store_rec(static_cast<uint8_t*>(out), rec, t, (*res)[t]);
  return BOS_ORACLE_OK;
}

int bos_oracle_levels(const void* in, uint64_t n, uint32_t rec, const bos_oracle_cfg* cfg,
                      uint32_t attempt, void* recs, uint32_t* tags, int32_t* ovf_level,
                      int64_t* ovf_pair) {
  if (!cfg || !valid_rec(rec) || !recs || !tags || !ovf_level || !ovf_pair || (n && !in))
    return BOS_ORACLE_INVALID;
  uint64_t B;
  uint32_t L;
  if (plan_with_override(n, cfg, &B, &L) != BOS_ORACLE_OK) return BOS_ORACLE_INVALID;
  const uint32_t Z = cfg->z;
  *ovf_level = -1;
  *ovf_pair = -1;
  Tracer tr;
  std::vector<uint32_t> lab;
  std::vector<Slot> A, Anext;
  draw_labels(n, L, B, cfg, attempt, lab);
  place_groups(static_cast<const uint8_t*>(in), n, rec, B, Z, lab, A, tr);
  auto dump = [&](uint32_t level) {
    uint8_t* rbase = static_cast<uint8_t*>(recs) + uint64_t(level) * B * Z * rec;
    uint32_t* tbase = tags + uint64_t(level) * B * Z;
    for (uint64_t s = 0; s < B * Z; ++s) {
      const Slot& x = A[s];
      store_rec(rbase, rec, s, x.real ? x.r : Rec{0, 0});
      tbase[s] = x.real ? x.label : 0xFFFFFFFFu;
    }
  };
  dump(0);
  for (uint32_t i = 0; i < L; ++i) {
    int64_t pair = -1;
    if (!butterfly_level(A, Anext, B, Z, L, i, tr, &pair)) {
      *ovf_level = int32_t(i);
      *ovf_pair = pair;
      return BOS_ORACLE_OVERFLOW;
    }
    A.swap(Anext);
    dump(i + 1);
  }
  return BOS_ORACLE_OK;
}

int bos_oracle_merge_sort(const void* in, void* out, uint64_t n, uint32_t rec) {
  if (!valid_rec(rec) || (n && (!in || !out))) return BOS_ORACLE_INVALID;
  std::vector<Rec> Y(n), T;
  for (uint64_t t = 0; t < n; ++t) Y[t] = load_rec(static_cast<const uint8_t*>(in), rec, t);
  Tracer tr;
  std::vector<Rec>* res = merge_sort(Y, T, tr);
  for (uint64_t t = 0; t < n; ++t) store_rec(static_cast<uint8_t*>(out), rec, t, (*res)[t]);
  return BOS_ORACLE_OK;
}

}  // extern "C"
