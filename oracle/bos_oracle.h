/*
 * bos_oracle.h — plain single-threaded CPU oracle for bucket oblivious random
 * permutation (ORP) and bucket oblivious sort (Asharov, Chan, Nayak, Pass, Ren,
 * Shi, "Bucket Oblivious Sort: An Extremely Simple Oblivious Sort", SOSA 2020).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the product path never calls it.
 *
 * Every function follows the paper step by step (Algorithm 3.1, Sections 3.2,
 * 3.3, 3.4 and 4.1); nothing is blocked, fused or reordered.  Where the paper
 * leaves a choice open, the reading taken is stated next to the code.
 *
 * Records are little-endian {key, payload} pairs of two unsigned integers of
 * rec/2 bytes each (rec = 8 or 16).  Record order is unsigned lexicographic on
 * (key, payload).
 */
#ifndef BOS_ORACLE_H
#define BOS_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define BOS_ORACLE_OK 0
#define BOS_ORACLE_INVALID 1
#define BOS_ORACLE_OVERFLOW 2

typedef struct {
  uint64_t seed;               /* Philox key word 0 */
  uint32_t z;                  /* bucket capacity Z: even, >= 2 */
  uint32_t max_retries;        /* attempts allowed = max_retries + 1 */
  uint64_t b_override;         /* 0, or a power of two >= the planned B (test hook) */
  const uint32_t* label_override; /* NULL, or n labels (< B) used by attempt 0 (test hook) */
  uint64_t* trace;             /* NULL, or a buffer receiving one code per memory access */
  uint64_t trace_cap;          /* entries available in trace */
} bos_oracle_cfg;

typedef struct {
  uint64_t buckets;            /* B */
  uint32_t levels;             /* log2 B */
  uint32_t attempts;           /* attempts run, including the successful one */
  int32_t first_overflow_level;  /* level i of the first overflowing MergeSplit of
                                    the last failed attempt, -1 if none failed */
  int32_t pad_;
  int64_t first_overflow_pair; /* its pair index j, -1 if none failed */
  uint64_t accesses_orp;       /* server-memory accesses of the successful ORP attempt */
  uint64_t accesses_sort;      /* server-memory accesses of the merge sort */
  uint64_t digest_orp;         /* hash of the access sequence of all ORP attempts */
  uint64_t digest_sort;        /* hash of the access sequence of the merge sort */
  uint64_t trace_len;          /* accesses recorded (all attempts, then the sort) */
  double sec_labels, sec_route, sec_finish, sec_sort;
} bos_oracle_report;

/* Access encoding used by trace/digest: bit 63 = write, bits 56..62 = array id,
 * bits 0..55 = element index within the array.  Array ids: 0 = input X,
 * 1 + i = level array A^(i), 100 = ORP output / sort buffer Y, 101 = sort
 * buffer T.  Level-array index = bucket * Z + slot. */
#define BOS_ORACLE_ARR_X 0u
#define BOS_ORACLE_ARR_LEVEL0 1u
#define BOS_ORACLE_ARR_Y 100u
#define BOS_ORACLE_ARR_T 101u

/* Section 3.1 / 3.2: number of buckets B (smallest power of two >= 2n/Z, 1 when
 * 2n <= Z) and levels log2 B.  Returns BOS_ORACLE_INVALID for odd Z, Z < 2 or
 * more than 31 levels. */
int bos_oracle_plan(uint64_t n, uint32_t z, uint64_t* buckets, uint32_t* levels);

/* Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void bos_oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Uniform random bin label of element i in attempt a (Algorithm 3.1). */
uint32_t bos_oracle_label(uint64_t seed, uint32_t attempt, uint64_t i, uint32_t levels);

/* 64-bit random key number g of attempt a, used to permute each final bin
 * (Section 3.2, Section 4.1). */
uint64_t bos_oracle_shuffle_key(uint64_t seed, uint32_t attempt, uint64_t g);

/* Bucket ORP (Section 3.2): out[0..n) = a random permutation of in[0..n). */
int bos_oracle_orp(const void* in, void* out, uint64_t n, uint32_t rec,
                   const bos_oracle_cfg* cfg, bos_oracle_report* rep);

/* Bucket oblivious sort (Section 3.3): ORP, then a bottom-up merge sort. */
int bos_oracle_sort(const void* in, void* out, uint64_t n, uint32_t rec,
                    const bos_oracle_cfg* cfg, bos_oracle_report* rep);

/* Oblivious random bin assignment of one attempt (Algorithm 3.1), dumping every
 * level array: recs[(L+1)*B*Z*rec] and tags[(L+1)*B*Z] (tag = label, or
 * 0xFFFFFFFF for a dummy whose record bytes are zero).  Levels after an
 * overflow are left untouched.  *ovf_level / *ovf_pair receive the first
 * overflowing MergeSplit or -1. */
int bos_oracle_levels(const void* in, uint64_t n, uint32_t rec, const bos_oracle_cfg* cfg,
                      uint32_t attempt, void* recs, uint32_t* tags,
                      int32_t* ovf_level, int64_t* ovf_pair);

/* Plain bottom-up merge sort by (key, payload), the non-oblivious comparison
 * sort of Section 3.3, exposed on its own. */
int bos_oracle_merge_sort(const void* in, void* out, uint64_t n, uint32_t rec);

#ifdef __cplusplus
}
#endif
#endif
