"""Batched bucket oblivious sort (bos_sort_batched) on the GPU.

Every instance of a batch must come out byte-identical to the same instance
sorted alone (bos_sort) and to the oracle; the captured graph is replayed with
new inputs, with eager GPU work between replays.
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


def _batch(sizes, rec, data_seed):
    return [inputs.records(int(n), rec, data_seed + i, key_bits=(20 if rec == 16 else None))
            for i, n in enumerate(sizes)]


SIZES = [1024, 3000, 0, 1, 257, 4096, 70000, 12345, 2048, 100, 1 << 15, 5]


@pytest.mark.parametrize("rec,z", [(8, 512), (16, 512), (16, 256), (8, 1024)])
def test_batched_equals_alone_and_oracle(rec, z):
    hosts = _batch(SIZES, rec, 100)
    seeds = [1000 + i for i in range(len(hosts))]
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], seeds, z=z, min_security_bits=0)
    for h, o, s in zip(hosts, outs, seeds):
        got = bos.to_numpy(o)
        np.testing.assert_array_equal(got, cf.sorted_records(h))
        alone = bos.to_numpy(bos.sort(bos.from_numpy(h), seed=s, z=z, min_security_bits=0))
        np.testing.assert_array_equal(got, alone)


@pytest.mark.parametrize("rec,tile", [(8, 1024), (16, 2048), (8, 4096)])
def test_batched_four_way_passes(rec, tile):
    # Merge phases that start with a four-way pass (even level counts), that
    # start with a two-way pass (odd counts: the four-way samples are then
    # gathered), that never reach a merge tile, with runs wide enough for the
    # workgroup-wide rank kernel, ragged tails, and instances with no merge
    # pass: every instance equals the same instance sorted alone and numpy's
    # sort.
    sizes = [1 << 18, 300000, 5000, 70001, 4 * tile + 3, 1, 0, tile, 1 << 16, 2 * tile + 1]
    hosts = _batch(sizes, rec, 77)
    seeds = [300 + i for i in range(len(hosts))]
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], seeds, tile=tile)
    for h, o, s in zip(hosts, outs, seeds):
        got = bos.to_numpy(o)
        np.testing.assert_array_equal(got, cf.sorted_records(h))
        if len(h):
            alone = bos.to_numpy(bos.sort(bos.from_numpy(h), seed=s, tile=tile))
            np.testing.assert_array_equal(got, alone)


def test_graph_replays_with_new_inputs():
    sizes = [5000, 20000, 777, 1 << 14]
    for rnd in range(3):
        hosts = _batch(sizes, 16, 7 + 31 * rnd)
        ts = [bos.from_numpy(h) for h in hosts]
        # eager work on the same stream between replays
        junk = torch.randn(1 << 20, device="cuda")
        junk = (junk * 2).sum()
        torch.cuda.synchronize()
        outs = bos.sort_batched(ts, [rnd * 10 + i for i in range(len(ts))])
        for h, o in zip(hosts, outs):
            np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))


def test_batched_overflow_retries_match_alone(ora_lib=None):
    # Z = 32 overflows often at these sizes: overflowing instances continue
    # alone from attempt 1, exactly as bos_sort would.
    import oracle
    oracle.build(force=False)
    sizes = [1 << 14, 9000, 1 << 13, 6000]
    hosts = _batch(sizes, 8, 5)
    seeds = [11, 12, 13, 14]
    outs, rep = bos.sort_batched([bos.from_numpy(h) for h in hosts], seeds, z=32, max_retries=30,
                                 min_security_bits=0, report=True)
    retried = 0
    for h, o, s in zip(hosts, outs, seeds):
        want = oracle.sort(h, s, z=32, max_retries=30)
        assert want["rc"] == 0
        retried += want["report"]["attempts"] > 1
        np.testing.assert_array_equal(bos.to_numpy(o), want["out"])
    assert retried > 0
    assert rep["attempts"] >= len(sizes) + retried


def test_sequential_fallback_for_other_z():
    hosts = _batch([3000, 100, 9000], 8, 3)
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], [1, 2, 3], z=64, min_security_bits=0)
    for h, o in zip(hosts, outs):
        np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))


def test_batched_workload_shape():
    # a slice of the batched workload: 256 instances, log-uniform sizes in
    # [2^10, 2^16], 16-byte records
    sizes = inputs.batched_sizes(count=256, lo_log2=10, hi_log2=16, cap=1 << 22, seed=4242)
    hosts = [inputs.records(int(n), 16, 4242 + i) for i, n in enumerate(sizes)]
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], [1000 + i for i in range(len(hosts))])
    for h, o in zip(hosts, outs):
        np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))


def test_batched_workload_full_size():
    # The batched configuration the benchmark times: 4096 instances of 16-byte
    # records (uniform u64 key, payload = index), sizes log-uniform in
    # [2^10, 2^20] rescaled to a total <= 2^28, Z, k and tile from the stored
    # tuning table.  Every instance comes out sorted by (key, payload) and as a
    # permutation of its input (an order-independent checksum per instance);
    # 8 sampled instances are compared whole with numpy's sort.
    from paper_2008_01765_amd import autotune

    previous = bos.get_tuning()
    autotune.install()
    try:
        sizes = inputs.batched_sizes(4096, 10, 20, 1 << 28, seed=4242)
        total = int(sizes.sum())
        host = inputs.records(total, 16, 43)
        master = bos.from_numpy(host)
        offs = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        ins = [master[int(o):int(o) + int(n)] for o, n in zip(offs, sizes)]
        outm = torch.empty_like(master)
        outs = [outm[int(o):int(o) + int(n)] for o, n in zip(offs, sizes)]
        bos.sort_batched(ins, list(range(len(ins))), outs=outs)
        got = bos.to_numpy(outm)
        del ins, outs, master, outm
    finally:
        bos.set_tuning(previous)
        bos.release_workspaces()
    k, p = got[:, 0], got[:, 1]
    ok = (k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (p[1:] >= p[:-1]))
    ok[offs[1:] - 1] = True  # instance boundaries
    assert bool(np.all(ok))

    def mix(a):
        with np.errstate(over="ignore"):
            z = a[:, 0] * np.uint64(0x9E3779B97F4A7C15) ^ (a[:, 1] + np.uint64(0x632BE59BD9B4E019))
            z ^= z >> np.uint64(29)
            z *= np.uint64(0xBF58476D1CE4E5B9)
            return z ^ (z >> np.uint64(32))

    np.testing.assert_array_equal(np.add.reduceat(mix(got), offs), np.add.reduceat(mix(host), offs))
    for i in np.random.default_rng(8).choice(len(sizes), 8, replace=False):
        o, n = int(offs[i]), int(sizes[i])
        np.testing.assert_array_equal(got[o:o + n], cf.sorted_records(host[o:o + n]))
