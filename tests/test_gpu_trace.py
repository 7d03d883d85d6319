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
Covered: the register-resident routing kernels (every Z in [16, 2048]), the
split last pass, the per-bin finish and the strip, the tile sort and the
merge passes.  Not covered: the generic routing kernel (Z = 8) and the fused
single-pass plans, whose last pass takes blocks in ticket order.
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


@pytest.fixture(scope="module")
def traced():
    bufs = [torch.zeros(SLOTS, dtype=torch.int64, device="cuda") for _ in range(2)]
    with bos.using_library(bos.TRACE_LIB_PATH) as L:
        assert L.bos_trace_bind(bufs[0].data_ptr(), bufs[1].data_ptr(), SLOTS) == bos.OK

        def run(fn, t, **kw):
            for b in bufs:
                b.zero_()
            torch.cuda.synchronize()
            out = fn(t, **kw)
            torch.cuda.synchronize()
            return out, bufs[0].clone(), bufs[1].clone()

        yield run
        L.bos_trace_bind(None, None, 0)


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
