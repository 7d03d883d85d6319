"""Data-independent access patterns on the GPU (Definition 2.1), measured.

libbos_trace.so is libbos built with BOS_TRACE_DIGEST: every HBM and LDS
access of the routing passes, the per-bin finish and the strip folds (array,
index) into a 64-bit slot of its thread, in program order, in one device
buffer; every access of the comparison sort does the same in a second buffer
(bos_trace_bind).  Equal buffers after two runs mean that every thread of every
launch touched the same arrays at the same indices in the same order.

On the duplicate-heavy workload (n = 2^24 records of 16 bytes, keys uniform on
[0, 2^20), Z = 512, one ORP seed) with two different key sets:
  * bos_orp: routing + finish digests identical;
  * bos_sort: routing + strip digests identical; the comparison sort's digests
    identical for inputs of the same order type (key' = 2 key + 1), as the
    composition argument of Section 3.3 has it, and different otherwise;
  * a different ORP seed changes the routing digest (the loads differ), so the
    digest does see the addresses.
The same checks run on the other workloads: the small one (2^16 records of 8
bytes), the headline one at full size (2^28 records of 8 bytes, Z = 512, with a
trace buffer of one slot per thread of the largest launch), the sweep's other
(Z, k) shapes at 2^20 records, and a batch of uneven instances through the
batched engine (16-byte records, per-instance seeds): its routing digest is
identical for two key sets, its comparison-sort digest for inputs of the same
order type.
Covered: the register-resident routing kernels (every Z in [16, 2048]), the
split last pass, the per-bin finish and the strip, the tile sort and the
merge passes, and their table-driven forms in the batched engine.  Not
covered: the generic routing kernel (Z = 8) and the fused single-pass plans,
whose last pass takes blocks in ticket order.
"""
import numpy as np
import pytest

from gpu_util import torch_is_sorted
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos  # noqa: E402

SLOTS = 1 << 22


class _Tracer:
    """Runs calls of the traced library with two zeroed digest buffers of
    `slots` slots bound (one slot per thread of the largest launch keeps the
    digest deterministic: no two threads of a launch share a slot)."""

    def __init__(self, L, slots):
        self.L = L
        self.bufs = [torch.zeros(slots, dtype=torch.int64, device="cuda") for _ in range(2)]
        assert L.bos_trace_bind(self.bufs[0].data_ptr(), self.bufs[1].data_ptr(), slots) == bos.OK

    def __call__(self, fn, t, **kw):
        for b in self.bufs:
            b.zero_()
        torch.cuda.synchronize()
        out = fn(t, **kw)
        torch.cuda.synchronize()
        return out, self.bufs[0].clone(), self.bufs[1].clone()

    def close(self):
        self.L.bos_trace_bind(None, None, 0)
        self.bufs = None
        torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def trace_lib():
    with bos.using_library(bos.TRACE_LIB_PATH) as L:
        yield L


@pytest.fixture
def traced(trace_lib):
    tr = _Tracer(trace_lib, SLOTS)
    yield tr
    tr.close()


def _dup(seed):
    return inputs.records(1 << 24, 16, seed, key_bits=20)


def test_plain_library_has_no_digests():
    assert bos.lib().bos_trace_bind(None, None, 0) == bos.UNSUPPORTED


def test_orp_digest_independent_of_data(traced):
    a, b = _dup(42), _dup(43)
    oa, ra, _ = traced(bos.orp, bos.from_numpy(a), seed=1, z=512)
    ob, rb, _ = traced(bos.orp, bos.from_numpy(b), seed=1, z=512)
    # the buffer saw the accesses (persistent launches: one slot per thread of
    # the largest grid, about 1.3e5 here)
    assert int(torch.count_nonzero(ra)) > 10000
    assert torch.equal(ra, rb)
    assert not torch.equal(oa, ob)
    # the traced build computes the same permutation as the plain one
    assert torch.equal(oa, bos.orp(bos.from_numpy(a), seed=1, z=512))
    _, rc, _ = traced(bos.orp, bos.from_numpy(a), seed=2, z=512)
    assert not torch.equal(ra, rc)  # other labels, other loads: other strip offsets


def test_sort_digests(traced):
    a, b = _dup(42), _dup(43)
    c = a.copy()
    c[:, 0] = 2 * c[:, 0] + 1  # same order type as a (keys < 2^20: no wrap)
    oa, ra, sa = traced(bos.sort, bos.from_numpy(a), seed=1, z=512)
    ob, rb, sb = traced(bos.sort, bos.from_numpy(b), seed=1, z=512)
    oc, rc, sc = traced(bos.sort, bos.from_numpy(c), seed=1, z=512)
    for o in (oa, ob, oc):
        assert torch_is_sorted(o)
    assert int(torch.count_nonzero(sa)) > 0
    # routing, per-bin compaction and strip: independent of the data
    assert torch.equal(ra, rb) and torch.equal(ra, rc)
    # comparison sort: a function of the order type only
    assert torch.equal(sa, sc)
    assert not torch.equal(sa, sb)


def _same_order_type(a):
    """Records of the same relative order as a (key' = 2 key + 1, no wrap for
    keys below 2^31)."""
    c = a.copy()
    c[:, 0] = 2 * c[:, 0] + 1
    return c


def _check_orp_and_sort(tr, a, b, **kw):
    """Routing, finish and strip digests of bos_orp and bos_sort identical for
    the key sets a and b; comparison-sort digests identical for a and an input
    of a's order type and different for b."""
    oa, ra, _ = tr(bos.orp, bos.from_numpy(a), **kw)
    ob, rb, _ = tr(bos.orp, bos.from_numpy(b), **kw)
    assert int(torch.count_nonzero(ra)) > 0
    assert torch.equal(ra, rb)
    assert not torch.equal(oa, ob)
    del oa, ob
    c = _same_order_type(a)
    sa_out, ra, sa = tr(bos.sort, bos.from_numpy(a), **kw)
    assert torch_is_sorted(sa_out)
    del sa_out
    _, rb, sb = tr(bos.sort, bos.from_numpy(b), **kw)
    _, rc, sc = tr(bos.sort, bos.from_numpy(c), **kw)
    assert int(torch.count_nonzero(sa)) > 0
    assert torch.equal(ra, rb) and torch.equal(ra, rc)
    assert torch.equal(sa, sc)
    assert not torch.equal(sa, sb)


def test_small_workload_digests(traced):
    # 2^16 records of 8 bytes (uniform u32 keys below 2^31, so the order-type
    # copy does not wrap), Z = 512
    a = inputs.records(1 << 16, 8, 42)
    b = inputs.records(1 << 16, 8, 43)
    a[:, 0] >>= 1
    b[:, 0] >>= 1
    _check_orp_and_sort(traced, a, b, seed=1, z=512)


@pytest.mark.parametrize("z,k", [(256, 2), (256, 4), (512, 2), (512, 4), (1024, 2), (1024, 3)])
def test_sweep_shapes_digests(traced, z, k):
    # the headline sweep's (Z, k) shapes at 2^20 records of 8 bytes
    a = inputs.records(1 << 20, 8, 42)
    b = inputs.records(1 << 20, 8, 43)
    a[:, 0] >>= 1
    b[:, 0] >>= 1
    _check_orp_and_sort(traced, a, b, seed=1, z=z, k=k, min_security_bits=0)


def test_headline_workload_digests(trace_lib):
    # n = 2^28 records of 8 bytes, Z = 512, default k: the largest launch (tile
    # sort, merge tiles) has n / 16 = 2^24 threads, one slot each
    n = 1 << 28
    tr = _Tracer(trace_lib, n >> 4)
    try:
        a = inputs.records(n, 8, 42)
        b = inputs.records(n, 8, 43)
        a[:, 0] >>= 1
        b[:, 0] >>= 1
        _check_orp_and_sort(tr, a, b, seed=1, z=512)
    finally:
        tr.close()


def test_batched_digests(trace_lib):
    # uneven instances of 16-byte records through the batched engine (one
    # captured graph per batch shape); a plain sort first binds the digest
    # buffers in every kernel file the batch launches from, outside capture
    tr = _Tracer(trace_lib, SLOTS)
    try:
        tr(bos.sort, bos.from_numpy(inputs.records(1 << 18, 16, 5, key_bits=20)), seed=1, z=512)
        sizes = [1 << 10, 3000, 1 << 14, 70001, 1 << 17, 5000, 1 << 12, 123457]
        seeds = [500 + i for i in range(len(sizes))]

        def batch(data_seed, order_type=False):
            hs = [inputs.records(m, 16, data_seed + i, key_bits=20) for i, m in enumerate(sizes)]
            if order_type:
                hs = [_same_order_type(h) for h in hs]
            return [bos.from_numpy(h) for h in hs]

        def run(ts):
            return bos.sort_batched(ts, seeds, z=512)

        oa, ra, sa = tr(run, batch(42))
        ob, rb, sb = tr(run, batch(43))
        oc, rc, sc = tr(run, batch(42, order_type=True))
        for o in oa + ob + oc:
            assert torch_is_sorted(o)
        assert int(torch.count_nonzero(ra)) > 0 and int(torch.count_nonzero(sa)) > 0
        assert torch.equal(ra, rb) and torch.equal(ra, rc)
        assert torch.equal(sa, sc)
        assert not torch.equal(sa, sb)
    finally:
        tr.close()
