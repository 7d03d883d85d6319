"""Pins of the CPU oracle to the paper (no GPU needed).

Each test checks the oracle against something other than itself: a library
routine (numpy's Philox, numpy's sort), a published known-answer vector, a
closed form implied by Algorithm 3.1 and Figure 1, the simulator of Lemma 3.3,
the access counts of Section 3.4, or a statistical property (Lemma 3.2 and the
uniformity part of Lemma 3.3).
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import closed_forms as cf
from paper_2008_01765_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _recs(n, rec, seed=42, key_bits=None):
    return inputs.records(n, rec, seed, key_bits=key_bits)


# ----------------------------------------------------------------- Philox ---

def test_philox_known_answers(oracle_lib):
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle_lib.philox4x64_10(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("seed,attempt", [(1, 0), (123456789, 2), (2**64 - 1, 7)])
def test_philox_matches_numpy(oracle_lib, seed, attempt):
    blocks = cf.philox_blocks(seed, 0, attempt, 1000, 8)
    for t in range(8):
        assert oracle_lib.philox4x64_10([1000 + t, attempt, 0, 0], [seed, 0]) == \
            [int(x) for x in blocks[t]]


@pytest.mark.parametrize("L", [1, 5, 8, 20, 31])
def test_labels_match_numpy_philox(oracle_lib, L):
    n = 1000
    want = cf.labels(99, 3, n, L)
    got = np.array([oracle_lib.label(99, 3, i, L) for i in range(n)], dtype=np.uint32)
    np.testing.assert_array_equal(got, want)
    assert got.max() < (1 << L)


def test_label_zero_levels(oracle_lib):
    assert all(oracle_lib.label(5, 0, i, 0) == 0 for i in range(20))


def test_shuffle_keys_match_numpy_philox(oracle_lib):
    want = cf.shuffle_keys(77, 1, 13, 50)
    got = [oracle_lib.shuffle_key(77, 1, 13 + t) for t in range(50)]
    assert got == [int(x) for x in want]


def test_labels_uniform_chi2():
    # Algorithm 3.1: each label is uniform on [0, B-1].
    L, n = 6, 1 << 16
    lab = cf.labels(2024, 0, n, L)
    obs = np.bincount(lab, minlength=1 << L)
    p = stats.chisquare(obs).pvalue
    assert p > 1e-4


# ------------------------------------------------------------------- plan ---

@pytest.mark.parametrize("n", [0, 1, 2, 3, 7, 255, 256, 257, 1000, 1 << 16, (1 << 16) + 1, 10**6])
@pytest.mark.parametrize("z", [2, 4, 8, 16, 512, 1024, 6])
def test_plan_is_smallest_power_of_two(oracle_lib, n, z):
    B, L = oracle_lib.plan(n, z)
    assert cf.is_pow2(B) and B == 1 << L
    assert B * z >= 2 * n                       # B >= 2n/Z
    assert B == 1 or (B // 2) * z < 2 * n       # smallest such power of two


def test_plan_rejects_odd_z(oracle_lib):
    with pytest.raises(ValueError):
        oracle_lib.plan(100, 7)


def test_plan_headline_sizes(oracle_lib):
    # The sizes the paper quotes (n = 2^30, Z = 512) and the workloads' sizes.
    assert oracle_lib.plan(1 << 30, 512) == (1 << 22, 22)
    assert oracle_lib.plan(1 << 16, 512) == (256, 8)
    assert oracle_lib.plan(1 << 24, 512) == (1 << 16, 16)
    assert oracle_lib.plan(1 << 28, 256) == (1 << 21, 21)


# -------------------------------------------------- level contents (Alg 3.1) ---

CASES = [  # n, rec, Z
    (1 << 12, 8, 64), (1000, 16, 32), (777, 8, 16), (64, 8, 8), (5, 8, 4), (33, 16, 2),
    (1 << 14, 8, 512),
]


@pytest.mark.parametrize("n,rec,z", CASES)
def test_levels_match_closed_form(oracle_lib, n, rec, z):
    recs = _recs(n, rec)
    B, L = oracle_lib.plan(n, z)
    for seed in range(6):
        res = oracle_lib.levels(recs, seed, z)
        lab = cf.labels(seed, 0, n, L)
        ovf = cf.first_overflow(n, lab, B, L, z)
        assert res["overflow"] == ovf
        last = L if ovf[0] < 0 else ovf[0]
        for i in range(last + 1):
            R, T, over = cf.expected_level(recs, lab, B, L, z, i)
            assert not over
            np.testing.assert_array_equal(res["recs"][i], R)
            np.testing.assert_array_equal(res["tags"][i], T)


def test_final_bin_is_label(oracle_lib):
    n, z = 3000, 64
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    res = oracle_lib.levels(recs, 5, z)
    assert res["rc"] == 0
    tags = res["tags"][L]
    for b in range(B):
        real = tags[b] != 0xFFFFFFFF
        assert np.all(tags[b][real] == b)
        # reals precede dummies in every final bin (Section 3.2)
        k = int(real.sum())
        assert real[:k].all() and not real[k:].any()


def test_level_arrays_carry_every_element(oracle_lib):
    n, z = 2048, 32
    recs = _recs(n, 16)
    B, L = oracle_lib.plan(n, z)
    res = oracle_lib.levels(recs, 11, z)
    if res["rc"] != 0:
        pytest.skip("this seed overflows")
    for i in range(L + 1):
        real = res["tags"][i] != 0xFFFFFFFF
        assert int(real.sum()) == n
        got = res["recs"][i][real]
        np.testing.assert_array_equal(cf.sorted_records(got), cf.sorted_records(recs))


# --------------------------------------------------------------- overflow ---

def test_forced_overflow_all_zero_labels(oracle_lib):
    # n = B*Z/2 with all labels 0: level 0 fills bucket 2j with Z reals, level 1
    # merges buckets 0 and 2 -> 2Z reals for output 0: first overflow (1, 0).
    for z, B in [(8, 4), (16, 8), (64, 16)]:
        n = B * z // 2
        recs = _recs(n, 8)
        lab = np.zeros(n, dtype=np.uint32)
        res = oracle_lib.levels(recs, 0, z, labels=lab)
        assert res["rc"] == 2 and res["overflow"] == (1, 0)
        assert cf.first_overflow(n, lab, B, B.bit_length() - 1, z) == (1, 0)


def test_level_zero_never_overflows(oracle_lib):
    # Level-0 MergeSplits see at most Z/2 + Z/2 reals.
    n, z = 512, 8
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    for seed in range(50):
        res = oracle_lib.levels(recs, seed, z)
        assert res["overflow"][0] != 0


def test_no_overflow_when_n_le_z(oracle_lib):
    for n in range(0, 9):
        recs = _recs(n, 8)
        for seed in range(20):
            r = oracle_lib.orp(recs, seed, z=16, max_retries=0, b_override=8)
            assert r["rc"] == 0


def test_overflow_predicate_many_seeds(oracle_lib):
    n, z = 1 << 11, 16
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    seen_overflow = 0
    for seed in range(40):
        res = oracle_lib.levels(recs, seed, z)
        lab = cf.labels(seed, 0, n, L)
        ovf = cf.first_overflow(n, lab, B, L, z)
        assert res["overflow"] == ovf
        assert (res["rc"] == 2) == (ovf[0] >= 0)
        seen_overflow += ovf[0] >= 0
    assert seen_overflow > 0  # Z = 16 at n = 2^11 overflows often


def test_retry_uses_next_attempt_labels(oracle_lib):
    n, z = 1 << 12, 32  # about one attempt in eight overflows
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    retried = 0
    for seed in range(60):
        r = oracle_lib.orp(recs, seed, z=z, max_retries=50)
        assert r["rc"] == 0
        a = r["report"]["attempts"]
        retried += a > 1
        # every failed attempt really overflows, the accepted one does not
        for att in range(a - 1):
            assert cf.first_overflow(n, cf.labels(seed, att, n, L), B, L, z)[0] >= 0
        lab = cf.labels(seed, a - 1, n, L)
        assert cf.first_overflow(n, lab, B, L, z) == (-1, -1)
        if a > 1:
            prev = cf.first_overflow(n, cf.labels(seed, a - 2, n, L), B, L, z)
            assert (r["report"]["first_overflow_level"], r["report"]["first_overflow_pair"]) == prev
        np.testing.assert_array_equal(r["out"], cf.expected_orp(recs, seed, a - 1, lab, B, z))
    assert retried > 0


def test_overflow_after_last_retry(oracle_lib):
    n, z = 1 << 12, 4
    recs = _recs(n, 8)
    r = oracle_lib.orp(recs, 3, z=z, max_retries=2)
    assert r["rc"] == 2 and r["out"] is None
    assert r["report"]["attempts"] == 3


def test_overflow_rate_within_lemma_3_2(oracle_lib):
    # Lemma 3.2: P[overflow] <= B log B e^{-Z/6}.  At n = 2^10, Z = 64 the bound
    # is ~3.7e-3; over 400 seeds the count must stay within a binomial bound.
    n, z = 1 << 10, 64
    B, L = oracle_lib.plan(n, z)
    eps = B * L * math.exp(-z / 6)
    trials = 400
    fails = 0
    for seed in range(trials):
        lab = cf.labels(seed, 0, n, L)
        fails += cf.first_overflow(n, lab, B, L, z)[0] >= 0
    assert stats.binom.sf(fails - 1, trials, eps) > 1e-6


# -------------------------------------------------------------------- ORP ---

@pytest.mark.parametrize("n,rec,z", CASES + [(0, 8, 512), (1, 16, 512), (256, 8, 512), (257, 8, 512)])
def test_orp_output_closed_form(oracle_lib, n, rec, z):
    recs = _recs(n, rec)
    B, L = oracle_lib.plan(n, z)
    r = oracle_lib.orp(recs, 9, z=z, max_retries=40)
    assert r["rc"] == 0
    a = r["report"]["attempts"] - 1
    lab = cf.labels(9, a, n, L)
    np.testing.assert_array_equal(r["out"], cf.expected_orp(recs, 9, a, lab, B, z))
    # a permutation of the input (Section 2, permutation functionality)
    np.testing.assert_array_equal(cf.sorted_records(r["out"]), cf.sorted_records(recs))


def test_orp_duplicates(oracle_lib):
    n, z = 5000, 64
    recs = _recs(n, 16, key_bits=3)
    recs[:, 1] = recs[:, 1] % 7  # many byte-identical records
    B, L = oracle_lib.plan(n, z)
    r = oracle_lib.orp(recs, 4, z=z, max_retries=40)
    a = r["report"]["attempts"] - 1
    lab = cf.labels(4, a, n, L)
    np.testing.assert_array_equal(r["out"], cf.expected_orp(recs, 4, a, lab, B, z))


def test_orp_uniform_permutation(oracle_lib):
    # Lemma 3.3: with no overflow possible (n <= Z) and B = 4 bins, the output
    # permutation is uniform over all n! orders.
    n = 4
    recs = np.stack([np.arange(n), np.arange(n)], axis=1).astype(np.uint32)
    perms = {}
    trials = 24000
    for seed in range(trials):
        out = oracle_lib.orp(recs, seed, z=8, max_retries=0, b_override=4)["out"]
        key = tuple(out[:, 1])
        perms[key] = perms.get(key, 0) + 1
    assert len(perms) == math.factorial(n)
    p = stats.chisquare(np.array(list(perms.values()))).pvalue
    assert p > 1e-4


def test_orp_single_bin_shuffle_uniform(oracle_lib):
    # Section 3.2 with no butterfly level (B = 1, L = 0, as 2n <= Z): the
    # output is the per-bin random permutation alone, so this pins the per-bin
    # shuffle apart from the routing.  Over seeds, every one of the 5! orders
    # of five distinct records must be equally likely.  The records enter out
    # of record order so that a shuffle that kept (or sorted) the input order
    # fails.
    n = 5
    recs = np.array([[30, 0], [10, 1], [40, 2], [0, 3], [20, 4]], dtype=np.uint32)
    assert oracle_lib.plan(n, 16) == (1, 0)
    perms = {}
    trials = 30000
    for seed in range(trials):
        out = oracle_lib.orp(recs, seed, z=16, max_retries=0)["out"]
        key = tuple(int(v) for v in out[:, 1])
        perms[key] = perms.get(key, 0) + 1
    assert len(perms) == math.factorial(n)
    assert all(sorted(p) == list(range(n)) for p in perms)
    p = stats.chisquare(np.array(list(perms.values()))).pvalue
    assert p > 1e-4
    # each record lands in each position with probability 1/n
    pos = np.zeros((n, n))
    for k, c in perms.items():
        for t, rid in enumerate(k):
            pos[rid, t] += c
    assert stats.chisquare(pos.reshape(-1)).pvalue > 1e-4


@pytest.mark.parametrize("n,rec,z,kb", [(1 << 12, 8, 64, None), (5000, 16, 32, 4), (3001, 8, 16, 6),
                                        (1, 8, 512, None), (300, 16, 512, None)])
def test_vectorised_orp_closed_form(oracle_lib, n, rec, z, kb):
    # The library-sort form of the ORP closed form (used at sizes where the
    # per-bin loop is too slow) equals the per-bin loop and the oracle.
    recs = _recs(n, rec, key_bits=kb)
    if kb is not None:
        recs[:, 1] = recs[:, 1] % 5  # byte-identical records too
    B, L = oracle_lib.plan(n, z)
    r = oracle_lib.orp(recs, 11, z=z, max_retries=40)
    a = r["report"]["attempts"] - 1
    lab = cf.labels(11, a, n, L)
    want = cf.expected_orp(recs, 11, a, lab, B, z)
    np.testing.assert_array_equal(cf.expected_orp_vec(recs, 11, a, lab, B, z), want)
    np.testing.assert_array_equal(r["out"], want)


def test_loads_multinomial(oracle_lib):
    # Lemma 3.3's simulator draws the loads by throwing n balls into B bins.
    n, z = 1 << 12, 64
    B, L = oracle_lib.plan(n, z)
    tot = np.zeros(B)
    for seed in range(20):
        tot += cf.loads(cf.labels(seed, 0, n, L), B)
    assert stats.chisquare(tot).pvalue > 1e-4


# ------------------------------------------------------------------- sort ---

@pytest.mark.parametrize("n,rec,z,kb", [(1 << 12, 8, 64, None), (3001, 16, 32, 20), (0, 8, 8, None),
                                        (1, 8, 8, None), (2, 16, 4, 3), (4096, 8, 512, 4)])
def test_sort_matches_library_sort(oracle_lib, n, rec, z, kb):
    recs = _recs(n, rec, key_bits=kb)
    r = oracle_lib.sort(recs, 3, z=z, max_retries=40)
    assert r["rc"] == 0
    np.testing.assert_array_equal(r["out"], cf.sorted_records(recs))


def test_merge_sort_matches_library(oracle_lib):
    for n in [0, 1, 2, 3, 17, 1000]:
        recs = _recs(n, 16, key_bits=5)
        np.testing.assert_array_equal(oracle_lib.merge_sort(recs), cf.sorted_records(recs))


def test_sort_output_independent_of_seed_and_z(oracle_lib):
    recs = _recs(2000, 8, key_bits=10)
    outs = [oracle_lib.sort(recs, s, z=z, max_retries=40)["out"] for s in (1, 2) for z in (16, 64)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


# -------------------------------------------------------- access counting ---

@pytest.mark.parametrize("n,z", [(1 << 10, 64), (1 << 12, 64), (1 << 14, 512), (1000, 128), (1, 8),
                                 (64, 8)])
def test_access_counts(oracle_lib, n, z):
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    r = oracle_lib.sort(recs, 1, z=z, max_retries=40)
    assert r["rc"] == 0
    rep = r["report"]
    # Section 3.4: each of the L+1 level arrays (B*Z slots) is written once and
    # read once, plus the input read and the output write.
    assert rep["accesses_orp"] == 2 * n + 2 * B * z * (L + 1)
    # bottom-up merge sort: ceil(log2 n) passes, each reading and writing n.
    assert rep["accesses_sort"] == 2 * n * math.ceil(math.log2(n)) if n > 1 else rep["accesses_sort"] == 0
    if B * z == 2 * n and z >= 8:
        assert rep["accesses_orp"] <= 4 * n * math.log2(n)
        assert rep["accesses_orp"] + rep["accesses_sort"] <= 6 * n * math.log2(n)


# ------------------------------------------------------------------ trace ---

@pytest.mark.parametrize("n,z", [(1 << 9, 16), (700, 32), (64, 64)])
def test_trace_equals_simulator(oracle_lib, n, z):
    recs = _recs(n, 8)
    B, L = oracle_lib.plan(n, z)
    cap = 4 * n + 4 * B * z * (L + 2)
    for seed in range(4):
        r = oracle_lib.orp(recs, seed, z=z, max_retries=0, trace_cap=cap)
        if r["rc"] != 0:
            continue
        w, a, i = oracle_lib.decode_trace(r["trace"])
        lab = cf.labels(seed, 0, n, L)
        sw, sa, si = cf.sim_orp_trace(n, z, B, L, cf.loads(lab, B))
        np.testing.assert_array_equal(w, sw)
        np.testing.assert_array_equal(a, sa)
        np.testing.assert_array_equal(i, si)


def test_orp_trace_independent_of_data(oracle_lib):
    n, z = 5000, 32
    d1 = oracle_lib.orp(_recs(n, 16, 42), 8, z=z, max_retries=40)["report"]
    d2 = oracle_lib.orp(_recs(n, 16, 43, key_bits=4), 8, z=z, max_retries=40)["report"]
    assert d1["digest_orp"] == d2["digest_orp"]
    assert d1["attempts"] == d2["attempts"]


def test_sort_trace_depends_only_on_order_type(oracle_lib):
    n, z = 3000, 32
    a = _recs(n, 8, 42, key_bits=16)
    b = a.copy()
    b[:, 0] = 2 * a[:, 0] + 1  # same order type
    ra = oracle_lib.sort(a, 6, z=z, max_retries=40)["report"]
    rb = oracle_lib.sort(b, 6, z=z, max_retries=40)["report"]
    assert ra["digest_orp"] == rb["digest_orp"]
    assert ra["digest_sort"] == rb["digest_sort"]


@pytest.mark.slow
def test_orp_trace_identical_for_two_key_sets_at_full_size(oracle_lib):
    # The duplicate-heavy workload at full size (n = 2^24, 16-byte records,
    # keys uniform on [0, 2^20)) with data seeds 42 and 43 and one ORP seed:
    # the access sequences of the ORP phase are identical (Section 3.2's
    # obliviousness, counted by the oracle's trace digest), and so are the
    # attempt counts.
    from paper_2008_01765_amd import inputs
    ra = oracle_lib.orp(inputs.workload_dup(42), 1)["report"]
    rb = oracle_lib.orp(inputs.workload_dup(43), 1)["report"]
    assert ra["digest_orp"] == rb["digest_orp"]
    assert ra["attempts"] == rb["attempts"]
