/*
 * bos.h — C ABI of libbos, bucket oblivious random permutation (ORP) and bucket
 * oblivious sort on AMD MI355X (gfx950).
 *
 * Method: Asharov, Chan, Nayak, Pass, Ren, Shi, "Bucket Oblivious Sort: An
 * Extremely Simple Oblivious Sort" (SOSA 2020).  The problem statement is that
 * of Section 1 and Section 2 (functionalities "oblivious sort" and "oblivious
 * permutation"): sort or permute n records held in untrusted memory so that the
 * sequence of memory addresses touched reveals nothing beyond n.  Here HBM and
 * LDS play the untrusted memory; every HBM and LDS address of the routing
 * phase is a function of (n, Z, levels per pass) only.  The strip of dummies
 * reveals the bin loads, as Lemma 3.3 allows, and the final comparison sort of
 * bos_sort reveals only what a comparison sort of a uniformly permuted array
 * reveals (Section 3.3).
 *
 * Records: little-endian array-of-structs {key, payload}, both unsigned, of
 * 4 + 4 bytes (BOS_REC_U32U32) or 8 + 8 bytes (BOS_REC_U64U64).  Record order is
 * unsigned lexicographic on (key, payload).
 *
 * Ownership: the caller owns every buffer.  `in`, `out` and `ws` are device
 * pointers (hipMalloc'd or torch CUDA tensors), at least 16-byte aligned;
 * `in` and `out` must not overlap each other or `ws`.  The library allocates no
 * device memory on these calls; it keeps only small host-side caches (captured
 * graphs of the batched path), released by bos_release_cache().
 *
 * Streams: `stream` is a hipStream_t (NULL = legacy default stream).  Work is
 * stream-ordered.  With BOS_SYNC (the default when params is NULL) the call
 * synchronizes `stream` after each attempt to read the overflow status and
 * retries on overflow; without it the call enqueues one attempt and returns,
 * leaving the status on the device.
 *
 * Errors: every entry point returns a bos_status; no exception crosses the ABI.
 * On any status other than BOS_OK the content of `out` is unspecified.
 */
#ifndef BOS_H
#define BOS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BOS_OK = 0,
  BOS_ERR_INVALID_ARG = 1, /* bad record type, null pointer, Z not supported, n too large */
  BOS_ERR_OVERFLOW = 2,    /* a bucket overflowed in every attempt (Algorithm 3.1 abort) */
  BOS_ERR_WORKSPACE = 3,   /* ws NULL or smaller than bos_workspace_bytes() */
  BOS_ERR_HIP = 4,         /* a HIP runtime call failed */
  BOS_ERR_INSECURE_Z = 5,  /* log2 of the Lemma 3.2 failure bound exceeds -min_security_bits */
  BOS_ERR_UNSUPPORTED = 6, /* no GPU, or a parameter combination the kernels do not cover */
  BOS_ERR_INTERNAL = 7     /* a consistency check of the comparison sort failed (a merge
                              tile whose bounds break the splitters' guarantee was
                              skipped); reported by bos_sort under BOS_SYNC */
} bos_status;

typedef enum { BOS_REC_U32U32 = 8, BOS_REC_U64U64 = 16 } bos_rec;

/* flags */
#define BOS_SYNC 1u        /* synchronize and retry on overflow inside the call */
#define BOS_GENERIC_ROUTING 2u /* test hook: route with the generic (non-specialised)
                                  kernel; same results, slower */
#define BOS_STRICT 8u          /* strict client (Section 4.1): one butterfly level per
                                  pass, so a workgroup holds one MergeSplit's 2Z slots
                                  (the paper's client storage) and keeps no LDS state
                                  from one level to the next; the per-bin finish works
                                  on one bin's Z slots.  For a threat model in which
                                  the working set of a fused block is observable.
                                  Slower (L passes instead of L/3); same outputs.  k
                                  must be 0 or 1 (else BOS_ERR_INVALID_ARG). */
#define BOS_EXACT_FINISH 4u    /* test hook: run bos_orp's per-bin finish through its
                                  exact-comparator launch (otherwise taken only when two
                                  random keys of a bin tie); same results, slower */

typedef struct {
  uint64_t seed;              /* Philox key: labels and per-bin permutation keys */
  uint32_t z;                 /* bucket capacity Z (Algorithm 3.1): a power of two;
                                 the kernels take Z in [8, 2048] (2, 4 and larger
                                 powers: BOS_ERR_UNSUPPORTED; Z = 2 or 4 fails
                                 Lemma 3.2's bound at every n > 1 anyway); 0 =
                                 the tuning table's, else 512 (the paper's
                                 choice) */
  uint32_t k;                 /* butterfly levels fused per pass; 0 = the tuning
                                 table's, else the planner's choice (3), either
                                 capped at what fits.  An explicit k whose block
                                 of 2^k buckets does not fit in LDS (64 KiB..160
                                 KiB by Z and record size) or in one workgroup
                                 is rejected with BOS_ERR_UNSUPPORTED; k > 12
                                 with BOS_ERR_INVALID_ARG */
  uint32_t tile;              /* records per tile of the final sort: 1024, 2048,
                                 4096, 8192 or (8-byte records) 16384; 0 = the
                                 tuning table's, else 4096 */
  uint32_t max_retries;       /* extra attempts after an overflow (default 3) */
  uint32_t min_security_bits; /* reject Z when log2(B log2 B e^(-Z/6)) > -bits;
                                 0 disables the check (default 80) */
  uint32_t flags;             /* BOS_SYNC */
  uint32_t attempt;           /* bos_orp / bos_sort: index of the first attempt
                                 (Philox counter word of the labels, Algorithm
                                 3.1's retry).  With BOS_SYNC the call runs
                                 attempts attempt .. max(attempt, max_retries);
                                 without, attempt alone.  Default 0.  An
                                 asynchronous caller that finds the status word
                                 (bos_status_offset) set re-issues the call with
                                 attempt + 1 and gets what a BOS_SYNC call would
                                 have produced.  Ignored by the batched and step
                                 entry points (their jobs carry their own). */
} bos_params;

typedef struct {
  uint32_t attempts;              /* index of the last attempt run, plus one
                                     (1 = the first attempt did not overflow) */
  uint32_t z, k, tile;            /* parameters used */
  uint32_t levels;                /* L = log2 B */
  uint32_t passes;                /* HBM passes of the routing phase */
  int32_t first_overflow_level;   /* first overflowing MergeSplit (level i, pair j)
                                     of the last failed attempt; -1 if none */
  int32_t reserved;
  int64_t first_overflow_pair;
  uint64_t buckets;               /* B */
  uint64_t algorithmic_bytes;     /* HBM bytes the method must move in the last attempt */
} bos_report;

typedef struct {
  const void* in;   /* device, n records */
  void* out;        /* device, n records */
  uint64_t n;
  uint64_t seed;
} bos_instance;

/* Fill *p with the defaults listed above. */
void bos_default_params(bos_params* p);

/* Device workspace (bytes) that bos_orp / bos_sort need for n records.
 * Returns 0 when the arguments are invalid. */
size_t bos_workspace_bytes(uint64_t n, bos_rec rec, const bos_params* p);

/* Byte offset, within the workspace of a bos_orp or bos_sort call with these
 * arguments (n, rec, z, k and tile as resolved by the planner), of the call's
 * overflow status word: 8 bytes, device memory, written in stream order by the
 * attempt's routing passes.  Once the stream has passed an asynchronous call
 * (no BOS_SYNC) it holds 0xFFFFFFFFFFFFFFFF if the attempt did not overflow,
 * else (level << 32) | pair of the first overflowing MergeSplit (Algorithm
 * 3.1's abort); the output is then unspecified and the caller re-issues the
 * call with bos_params.attempt + 1.  Returns SIZE_MAX for invalid arguments or
 * without a GPU. */
size_t bos_status_offset(uint64_t n, bos_rec rec, const bos_params* p);

/* Bucket ORP (Algorithm 3.1 followed by Section 3.2): out = in permuted by a
 * uniformly random permutation drawn from `seed`.  The output is a deterministic
 * function of (in, n, seed, Z) and does not depend on k or tile.  n may be 0. */
bos_status bos_orp(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p,
                   void* ws, size_t ws_bytes, void* stream, bos_report* rep /* host, nullable */);

/* Bucket oblivious sort (Section 3.3): the ORP's bin assignment (each bin
 * compacted obliviously; a bin that straddles a tile of the first sort phase is
 * sorted obliviously, every other bin is ordered by the oblivious tile sort),
 * then a non-oblivious comparison (merge) sort whose passes merge four runs
 * at a time once runs span a merge tile.  out = in sorted by (key, payload);
 * the output does not depend on seed, Z, k or tile. */
bos_status bos_sort(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p,
                    void* ws, size_t ws_bytes, void* stream, bos_report* rep);

/* bos_sort without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a 64 MiB array inside the library,
 * one per GPU, held until the process ends; the call allocates nothing.
 * Limit: the plan's workspace (bos_workspace_bytes) must fit in 64 MiB, which
 * holds n <= 2^20 records of 8 bytes or n <= 2^19 of 16 bytes at Z = 512;
 * larger n returns BOS_ERR_WORKSPACE before anything is launched.  Every call
 * on one GPU uses that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller.  The
 * array keeps the last call's contents; the call clears what it needs.
 * Arguments, output and errors otherwise as bos_sort. */
bos_status bos_sort_noalloc(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p,
                            void* stream, bos_report* rep);

/* Workspace for bos_sort_batched over `count` instances of the given sizes. */
size_t bos_batched_workspace_bytes(const uint64_t* n, uint32_t count, bos_rec rec,
                                   const bos_params* p);

/* Many independent bucket oblivious sorts (Section 3.3) of uneven sizes in one
 * pass-major launch sequence, captured once into a hipGraph per batch shape and
 * replayed afterwards.  inst: host array of `count` descriptors (device in/out
 * pointers, n, seed).  d_status: device array of `count` uint32 receiving
 * BOS_OK or BOS_ERR_OVERFLOW per instance of the last attempt.  With BOS_SYNC
 * the call retries overflowing instances (one at a time) and returns the worst
 * status; rep (nullable) receives totals.  Without BOS_SYNC the call enqueues
 * the first attempt of every instance and returns without waiting for the
 * device (the per-instance tables are uploaded from pinned host memory that
 * the library keeps per batch shape); d_status then holds each instance's
 * outcome once `stream` has passed the call, and an instance that overflowed
 * is redone by a BOS_SYNC call (or bos_sort with attempt 1) on it alone. */
bos_status bos_sort_batched(const bos_instance* inst, uint32_t count, bos_rec rec,
                            const bos_params* p, void* ws, size_t ws_bytes, void* stream,
                            uint32_t* d_status, bos_report* rep);

/* ---- continuous batching ------------------------------------------------ */

#define BOS_PHASE_DONE 0xFFFFFFFFu

/* One sort request driven by bos_sort_step. */
typedef struct {
  const void* in;     /* device, n records */
  void* out;          /* device, n records */
  uint64_t n;
  uint64_t seed;
  void* ws;           /* device workspace of this job: bos_workspace_bytes(n) bytes */
  size_t ws_bytes;
  uint32_t phase;     /* in/out: 0 for a new job, BOS_PHASE_DONE once finished */
  uint32_t attempt;   /* in/out: routing attempt, 0 for a new job */
  uint32_t status;    /* out: BOS_OK, or BOS_ERR_OVERFLOW once every attempt overflowed */
  uint32_t reserved;
} bos_job;

/* Device bytes of the step tables bos_sort_step needs for `count` jobs. */
size_t bos_step_workspace_bytes(uint32_t count);

/* Continuous batching of bucket oblivious sorts (Section 3.3): run one step
 * of every unfinished job and return.  A job's phases are its routing passes
 * (Algorithm 3.1; the last pass also compacts each bin and strips the dummies),
 * the tile sort and the merge passes of the comparison sort: phase values
 * 0..P-1, P, P+1.. (P = routing passes of the job's plan).  Array order is
 * priority: a step runs at least one phase of the first unfinished job and
 * hands a work budget of about twice that phase (at most 2^23 records'
 * worth) to the jobs after it, in order, each running as many phases as fit
 * (possibly none); jobs in the same
 * phase kind share launches, so requests admitted between steps run alongside
 * those already on the device.  The overflow check (Algorithm 3.1's abort) happens at the
 * end of the step in which a job's routing finished: an overflowed job goes
 * back to phase 0 with attempt + 1, or ends with BOS_ERR_OVERFLOW once
 * max_retries is used up.  Each finished job's output equals bos_sort's for
 * the same input, parameters and seed, and so does its attempt count.
 * jobs: host array, updated in place (phase, attempt, status).
 * step_ws: device, bos_step_workspace_bytes(count) bytes.  Synchronizes
 * `stream` before returning.  Errors: INVALID_ARG (aliasing in/out, a phase
 * beyond the job's last), WORKSPACE (a job's ws or step_ws too small),
 * INSECURE_Z, HIP. */
bos_status bos_sort_step(bos_job* jobs, uint32_t count, bos_rec rec, const bos_params* p, void* step_ws,
                         size_t step_ws_bytes, void* stream);

/* Pipelined continuous batching.  A stepper (host object, one per request
 * loop) lets each call enqueue its step and then wait for the PREVIOUS call's
 * step, so the device runs one step while the host plans the next; the
 * schedule, outputs and attempt counts are those of bos_sort_step.
 *   - A job whose phases have all been enqueued shows phase P + 1 + M (M =
 *     merge passes of its plan) until the call after its last step; it turns
 *     BOS_PHASE_DONE once that step has completed and the overflow check of
 *     its routing (run at the end of the step where the routing finished) has
 *     passed.  An overflowed job goes back to phase 0 with attempt + 1, as in
 *     bos_sort_step; phases already enqueued for the overflowed attempt still
 *     run and their writes are redone.
 *   - Jobs are matched across calls by their ws pointer: between calls the
 *     caller may reorder the array, drop jobs that are BOS_PHASE_DONE and add
 *     new ones (phase 0, attempt 0, reserved 0); it must not change a
 *     resident job's fields.  `reserved` carries the library's state.
 *   - Call until every job is BOS_PHASE_DONE (a call with nothing left to
 *     enqueue only collects the previous step).  A job that ends with
 *     BOS_ERR_OVERFLOW may still be read by the step in flight: reuse its
 *     buffers only in stream order.
 * step_ws: device, 2 x bos_step_workspace_bytes(count) bytes (the two steps
 * in flight use one half each; it may be a different buffer on each call).
 * The stepper holds two pinned host buffers and two events; it is not
 * thread-safe.  Errors as bos_sort_step; INVALID_ARG for a null stepper. */
typedef struct bos_stepper bos_stepper;
bos_stepper* bos_stepper_create(void); /* NULL without a GPU or on allocation failure */
void bos_stepper_destroy(bos_stepper* st); /* waits for a step in flight and drops its results */
bos_status bos_sort_step_async(bos_stepper* st, bos_job* jobs, uint32_t count, bos_rec rec, const bos_params* p,
                               void* step_ws, size_t step_ws_bytes, void* stream);

/* Oblivious bitonic sort (Batcher) of the same records by (key, payload): the
 * GPU baseline the bucket sort is measured against.  ws: bos_bitonic_workspace_bytes. */
size_t bos_bitonic_workspace_bytes(uint64_t n, bos_rec rec);
bos_status bos_bitonic_sort(const void* in, void* out, uint64_t n, bos_rec rec, void* ws,
                            size_t ws_bytes, void* stream);

/* ---- out-of-core (Section 4.3) --------------------------------------------- */

/* Bucket ORP (bos_orp_host) and bucket oblivious sort (bos_sort_host) of n
 * records held in HOST memory, for n beyond what the device holds (n <= 2^36).
 * Same results as bos_orp / bos_sort with the same arguments: bos_orp_host's
 * output is the one bos_orp gives for (input, seed, Z), bos_sort_host's is the
 * sorted input.
 *
 * The slot arrays of Algorithm 3.1 live in host memory (host_ws).  Every
 * routing pass streams them through the device once, in chunks of
 * consecutive routing blocks: a chunk reads one contiguous range of buckets
 * when it covers whole groups of 2^(i+k) buckets (2^k contiguous segments
 * otherwise) and writes one contiguous range, the consecutive-bucket
 * structure Section 4.3 builds its locality on.  The per-bin finish (ORP) or
 * the strip (sort) streams the bins once more; the sort's comparison phase
 * then sorts device-sized runs and merges them by sample splitters (one
 * further read and write of the records).  Host-memory addresses, like device
 * addresses, depend on (n, Z, k) in the routing phase, on the bin loads in the
 * strip, and on comparisons of the permuted records in the comparison phase.
 *
 * in, out: host, n records each (not overlapping).  host_ws: host,
 * bos_host_workspace_bytes(n, rec, p) bytes.  dev_ws: device, at least
 * bos_host_device_bytes(n, rec, p) bytes; a larger one gives larger chunks.
 * Host buffers allocated with hipHostMalloc (pinned) are copied at full DMA
 * rate and let copies overlap kernels; pageable memory works, slower.
 * The call orders itself after `stream`, runs on three internal streams of
 * the current device (input copies, kernels, output copies, pipelined over
 * two staging halves of dev_ws) and returns when `out` is written (overflow
 * retries as with BOS_SYNC, whatever params->flags says).  The internal
 * streams are shared by every out-of-core call on a device: such calls that
 * overlap (two host threads) must be serialised by the caller.  Errors: INVALID_ARG (as bos_sort,
 * n > 2^36), WORKSPACE (a workspace too small), UNSUPPORTED (a plan of one
 * routing pass, or Z = 8: use the in-core calls), OVERFLOW, INSECURE_Z, HIP,
 * INTERNAL (a consistency check of the comparison phase failed). */
size_t bos_host_workspace_bytes(uint64_t n, bos_rec rec, const bos_params* p);
size_t bos_host_device_bytes(uint64_t n, bos_rec rec, const bos_params* p);
bos_status bos_orp_host(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* host_ws,
                        size_t host_ws_bytes, void* dev_ws, size_t dev_ws_bytes, void* stream, bos_report* rep);
bos_status bos_sort_host(const void* in, void* out, uint64_t n, bos_rec rec, const bos_params* p, void* host_ws,
                         size_t host_ws_bytes, void* dev_ws, size_t dev_ws_bytes, void* stream, bos_report* rep);

/* ---- tuning table --------------------------------------------------------- */

/* One autotuner result: for records of `rec` bytes and n in size class
 * `log2n` (the smallest c with 2^c >= n), use bucket capacity z, k levels per
 * pass and comparison-sort tile `tile` (as in bos_params).  A zero field
 * leaves the library default (Z = 512, k = 3, tile = 4096). */
typedef struct {
  uint32_t rec;
  uint32_t log2n;
  uint32_t z;
  uint32_t k;
  uint32_t tile;
  uint32_t reserved;
} bos_tune_entry;

/* Replace the process-wide tuning table (count 0 clears it).  Wherever a
 * caller's bos_params leaves z, k or tile at 0, the plan of an n-record
 * instance takes them from the entry of the same record size whose size class
 * is nearest to n's; a tuned z that falls short of min_security_bits at that
 * n is doubled until it meets it (Lemma 3.2).  With z = 0, bos_orp's output
 * therefore depends on the table: pass an explicit z for a fixed result
 * (bos_sort's output never depends on it).  Drops cached batch graphs.
 * Errors: INVALID_ARG (record size, z, k or tile out of range). */
bos_status bos_set_tuning(const bos_tune_entry* entries, uint32_t count);

/* Copy up to `cap` entries of the table into `out`; returns the entry count. */
uint32_t bos_get_tuning(bos_tune_entry* out, uint32_t cap);

/* Drop cached graphs and plans. */
void bos_release_cache(void);

/* Static text for a status code. */
const char* bos_status_string(bos_status s);

/* ---- test and measurement hooks (not part of the method) ---------------- */

/* Run one attempt of the routing phase only (Algorithm 3.1) and copy the slot
 * arrays at every pass boundary to host memory: recs_host[(P+1) * B * Z * rec],
 * tags_host[(P+1) * B * Z] (tag = label or 0xFFFFFFFF for a dummy), and the
 * level index of every boundary to levels_host[P+1].  Bucket contents are
 * sets: the order of slots inside a bucket is the network's, not the paper's.
 * Synchronizes `stream`.  Returns BOS_ERR_OVERFLOW with *ovf_level / *ovf_pair
 * set when the attempt overflows. */
bos_status bos_debug_levels(const void* in, uint64_t n, bos_rec rec, const bos_params* p,
                            uint32_t attempt, void* ws, size_t ws_bytes, void* stream,
                            void* recs_host, uint32_t* tags_host, uint32_t* levels_host,
                            int32_t* ovf_level, int64_t* ovf_pair);

/* Labels of attempt `attempt` for elements 0..n-1 computed by the device
 * generator, written to labels_dev (device, n uint32). */
bos_status bos_debug_labels(uint64_t n, uint32_t levels, uint64_t seed, uint32_t attempt,
                            uint32_t* labels_dev, void* stream);

/* Per-launch timing.  When enabled, every kernel launch of bos_orp, bos_sort,
 * bos_sort_batched and bos_bitonic_sort is bracketed by two HIP events on the
 * launch's stream.  bos_profile_read() waits for the recorded events, copies
 * up to `cap` records (oldest first) and clears the log; it returns the number
 * of records that were logged.  Not thread-safe; meant for benchmarks. */
typedef enum {
  BOS_K_ROUTE_FIRST = 1,  /* first routing pass: input read, labels, levels */
  BOS_K_ROUTE_MID = 2,    /* middle routing pass: slot arrays in and out */
  BOS_K_ROUTE_LAST = 3,   /* last routing pass: levels, per-bin finish, strip */
  BOS_K_ROUTE_SINGLE = 4, /* first and last pass at once (L <= k) */
  BOS_K_SORT_TILE = 5,    /* comparison sort: tile sort */
  BOS_K_SORT_MERGE = 6,   /* comparison sort: one merge pass (two-way, or four-way with its splitters) */
  BOS_K_BITONIC_TILE = 7, /* bitonic baseline: local phases */
  BOS_K_BITONIC_GLOBAL = 8,
  BOS_K_BITONIC_TAIL = 9,
  BOS_K_OTHER = 10,
  BOS_K_STRIP = 11,       /* scan of the bin loads and strip after a split last pass */
  BOS_K_ORP_FINISH = 12   /* bos_orp after a split last pass: scan of the bin loads, then
                             each bin sorted, permuted by its random keys and stripped */
} bos_kernel_kind;
typedef struct {
  uint32_t kind;     /* bos_kernel_kind */
  uint32_t index;    /* pass index within its phase */
  float ms;          /* elapsed time between the two events */
  uint32_t reserved;
  uint64_t bytes;    /* algorithmic HBM bytes of the launch */
} bos_launch_time;
void bos_profile_enable(int on);
uint32_t bos_profile_read(bos_launch_time* out, uint32_t cap);

/* Address digests (the test build libbos_trace.so, compiled with
 * BOS_TRACE_DIGEST): bind two device buffers of `slots` uint64 words (a power
 * of two; the caller zeroes them).  From then on every HBM and LDS access of
 * the routing passes, the per-bin finish and the strip folds (array, index)
 * into route_buf[g], and every access of the comparison sort into
 * sort_buf[g], g = the accessing thread's global index in its launch modulo
 * `slots`, in program order; equal buffers after two runs mean equal access
 * sequences (Definition 2.1).  The plain library returns BOS_ERR_UNSUPPORTED.
 * Null buffers switch the folding off. */
bos_status bos_trace_bind(void* route_buf, void* sort_buf, uint64_t slots);

/* Number of passes and levels per pass the planner picks (passes_out[0] =
 * P, passes_out[1 + t] = levels of pass t, up to 32 passes). */
bos_status bos_plan(uint64_t n, bos_rec rec, const bos_params* p, uint64_t* buckets,
                    uint32_t* levels, uint32_t* passes_out);

#ifdef __cplusplus
}
#endif
#endif
