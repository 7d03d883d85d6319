"""Asynchronous use of the C ABI (calls without BOS_SYNC).

* bos_orp / bos_sort enqueue one attempt and leave its overflow status word on
  the device at bos_status_offset; the caller reads it and re-issues the call
  with bos_params.attempt + 1 until the word says no overflow.  The word must
  equal the first overflowing MergeSplit of the closed form (Algorithm 3.1's
  abort), and the final output must equal what the synchronous call (which
  retries inside) produces.
* bos_sort_batched without BOS_SYNC returns while the device still works on
  the stream, and d_status then holds every instance's outcome.
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


def _overflowing_seed(n, z, rec):
    import oracle
    oracle.build(force=False)
    B, L = oracle.plan(n, z)
    for seed in range(200):
        first = cf.first_overflow(n, cf.labels(seed, 0, n, L), B, L, z)
        second = cf.first_overflow(n, cf.labels(seed, 1, n, L), B, L, z)
        if first[0] >= 0 and second[0] < 0:
            return seed, first
    raise AssertionError("no seed overflowing exactly once")


@pytest.mark.parametrize("fn,rec", [("orp", 8), ("orp", 16), ("sort", 8), ("sort", 16)])
def test_async_status_word_and_reissue(fn, rec):
    n, z = 1 << 12, 32
    seed, first = _overflowing_seed(n, z, rec)
    a = inputs.records(n, rec, 42)
    x = bos.from_numpy(a)
    call = bos.orp if fn == "orp" else bos.sort
    want = bos.to_numpy(call(x, seed=seed, z=z, k=2, max_retries=5, min_security_bits=0))
    # attempt 0: overflows; the word names the closed form's first MergeSplit
    out = torch.empty_like(x)
    call(x, seed=seed, z=z, k=2, min_security_bits=0, out=out, sync=False, attempt=0)
    assert bos.status_word(x, z=z, k=2, min_security_bits=0) == first
    # attempt 1: no overflow, and the output is the synchronous call's
    _, rep = call(x, seed=seed, z=z, k=2, min_security_bits=0, out=out, sync=False, attempt=1, report=True)
    assert rep["attempts"] == 2
    assert bos.status_word(x, z=z, k=2, min_security_bits=0) is None
    np.testing.assert_array_equal(bos.to_numpy(out), want)


def test_sync_call_starts_at_the_given_attempt():
    n, z = 1 << 12, 32
    seed, _ = _overflowing_seed(n, z, 8)
    x = bos.from_numpy(inputs.records(n, 8, 42))
    o0, r0 = bos.orp(x, seed=seed, z=z, max_retries=5, min_security_bits=0, report=True)
    o1, r1 = bos.orp(x, seed=seed, z=z, max_retries=5, min_security_bits=0, report=True, attempt=1)
    assert r0["attempts"] == 2 and r1["attempts"] == 2
    assert torch.equal(o0, o1)


def _sleep_stream(ms):
    """Occupies the current stream for about `ms` milliseconds."""
    try:
        torch.cuda._sleep(int(ms * 2.0e6))  # cycles at roughly 2 GHz
    except (AttributeError, RuntimeError):
        big = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        for _ in range(max(1, int(ms))):
            big.add_(1)


def test_batched_async_returns_before_the_device():
    sizes = [1 << 10, 3000, 1 << 14, 77777, 1 << 16, 5, 0, 1 << 12] * 4
    hosts = [inputs.records(nn, 16, 500 + i) for i, nn in enumerate(sizes)]
    ts = [bos.from_numpy(h) if len(h) else torch.zeros((0, 2), dtype=torch.int64, device="cuda") for h in hosts]
    seeds = list(range(len(ts)))
    # first call captures the graph
    bos.sort_batched(ts, seeds, z=512)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    _sleep_stream(200)
    (outs, dstat) = bos.sort_batched(ts, seeds, z=512, sync=False, status=True)
    pending = not stream.query()
    torch.cuda.synchronize()
    assert pending, "the call waited for the device"
    assert int(dstat.abs().sum().item()) == 0
    for h, o in zip(hosts, outs):
        if len(h):
            np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))
    # and the synchronous form still agrees
    outs2 = bos.sort_batched(ts, seeds, z=512)
    for o, o2 in zip(outs, outs2):
        assert torch.equal(o, o2)
