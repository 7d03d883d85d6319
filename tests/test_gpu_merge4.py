"""Four-way merge passes of the comparison sort (Section 3.3's non-oblivious
sort; the sort's output is the records in (key, payload) order, so the
expected value is that order itself, plus the oracle on a ragged case).

The sizes put the four-way passes at every case of their tiling: an odd
number of merge levels (one two-way pass first), runs shorter than a merge
tile (two-way passes first), a partial last group with short and empty runs,
whole records repeated (ties across all four runs), and a large ragged n.
"""
import numpy as np
import pytest

import closed_forms as cf
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos  # noqa: E402

CASES = [
    # n, rec, tile
    (1 << 15, 8, 4096),            # three levels: one two-way, one four-way pass
    (1 << 16, 8, 1024),            # runs of 1024 and 2048 first, then two four-way passes
    (4096 * 9 + 1, 8, 4096),       # last group: one record in its first run
    (4096 * 12 + 777, 8, 4096),    # last group: runs 0..1 full, run 2 partial, run 3 empty
    (100000, 16, 2048),
    ((1 << 17) + 5, 16, 8192),
    (3 * (1 << 18) + 4321, 8, 4096),
    ((1 << 22) + 12345, 8, 4096),
    ((1 << 21) + 999, 16, 8192),
]


@pytest.mark.parametrize("n,rec,tile", CASES)
def test_sort_four_way_passes(n, rec, tile):
    a = inputs.records(n, rec, 7)
    out = bos.to_numpy(bos.sort(bos.from_numpy(a), seed=3, tile=tile, min_security_bits=0))
    np.testing.assert_array_equal(out, cf.sorted_records(a))


@pytest.mark.parametrize("n", [4096 * 24 + 513, (1 << 21) + 3])
@pytest.mark.parametrize("rec", [8, 16])
@pytest.mark.parametrize("distinct", [1, 3, 1000])
def test_sort_four_way_repeated_records(n, rec, distinct):
    # whole records repeated (key and payload), so ties cross every run; the
    # larger n reaches runs wide enough for the workgroup-wide sample ranks,
    # with windows of repeated samples larger than the LDS holds
    g = np.random.default_rng(distinct)
    dt = np.uint32 if rec == 8 else np.uint64
    v = g.integers(0, distinct, n)
    a = np.stack([v % 7, v], axis=1).astype(dt)
    out = bos.to_numpy(bos.sort(bos.from_numpy(a), seed=1, tile=4096, min_security_bits=0))
    np.testing.assert_array_equal(out, cf.sorted_records(a))


def test_sort_four_way_matches_oracle():
    import oracle
    oracle.build(force=False)
    a = inputs.records(4096 * 20 + 17, 8, 11, key_bits=14)
    out = bos.to_numpy(bos.sort(bos.from_numpy(a), seed=9, z=256, tile=4096, min_security_bits=0))
    want = oracle.sort(a, 9, z=256)
    np.testing.assert_array_equal(out, want["out"])
