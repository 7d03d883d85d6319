"""Out-of-core bucket ORP and sort (Section 4.3) on the GPU, through the C ABI.

bos_orp_host / bos_sort_host keep the records and slot arrays in host memory
and stream them through a bounded device workspace.  With the smallest device
workspace the routing passes run in many chunks, including chunks inside one
group of buckets (2^k input segments each), and the sort's comparison phase
merges several device-sized runs.  Their outputs must equal the in-core calls
(themselves bit-exact against the oracle) and, at a small size, the oracle.
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


def _host(a):
    t = bos.pinned_empty(a.shape, torch.int32 if a.dtype == np.uint32 else torch.int64)
    t.numpy()[:] = a.view(np.int32 if a.dtype == np.uint32 else np.int64)
    return t


def _np(t, rec):
    return t.numpy().view(np.uint32 if rec == 8 else np.uint64)


# n = 2^22 at Z = 512 and k = 3 has 5 routing passes; with the smallest device
# workspace a chunk holds 64 blocks, so the passes from level 9 on read 2^3
# segments per chunk, and the sort merges 16 runs.
@pytest.mark.parametrize("n,rec", [((1 << 22) - 777, 8), ((1 << 20) + 12345, 16)])
def test_orp_host_equals_orp(n, rec):
    a = inputs.records(n, rec, 61, key_bits=(20 if rec == 16 else None))
    got = _np(bos.orp_host(_host(a), seed=5, z=512), rec)
    want = bos.to_numpy(bos.orp(bos.from_numpy(a), seed=5, z=512))
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,rec", [((1 << 22) - 777, 8), ((1 << 20) + 12345, 16)])
def test_sort_host_sorts(n, rec):
    a = inputs.records(n, rec, 62, key_bits=(20 if rec == 16 else None))
    got, rep = bos.sort_host(_host(a), seed=7, z=512, report=True)
    np.testing.assert_array_equal(_np(got, rec), cf.sorted_records(a))
    assert rep["attempts"] == 1


def test_host_calls_match_oracle():
    import oracle
    oracle.build(force=False)
    a = inputs.records((1 << 17) + 5, 16, 63, key_bits=12)
    want = oracle.orp(a, 9, z=512)["out"]
    np.testing.assert_array_equal(_np(bos.orp_host(_host(a), seed=9, z=512), 16), want)
    want = oracle.sort(a, 9, z=512)["out"]
    np.testing.assert_array_equal(_np(bos.sort_host(_host(a), seed=9, z=512), 16), want)


def test_sort_host_repeated_records():
    # half the records byte-identical, the rest from four values: the
    # splitters order equal records by (run, position), so segments stay
    # within a device run
    n = (1 << 21) + 3
    a = inputs.records(n, 8, 64)
    a[: n // 2] = np.array([7, 7], dtype=np.uint32)
    a[n // 2:, 0] %= 4
    a[n // 2:, 1] %= 2
    got = _np(bos.sort_host(_host(a), seed=3, z=512), 8)
    np.testing.assert_array_equal(got, cf.sorted_records(a))


def test_one_chunk_per_pass():
    # a device workspace that holds every pass in one chunk and the whole sort in one run
    n = (1 << 18) + 99
    a = inputs.records(n, 8, 65)
    big = 1 << 30
    np.testing.assert_array_equal(_np(bos.orp_host(_host(a), seed=2, z=512, dev_ws_bytes=big), 8),
                                  bos.to_numpy(bos.orp(bos.from_numpy(a), seed=2, z=512)))
    np.testing.assert_array_equal(_np(bos.sort_host(_host(a), seed=2, z=512, dev_ws_bytes=big), 8),
                                  cf.sorted_records(a))


@pytest.mark.parametrize("k", [1, 2, 4])
def test_other_levels_per_pass(k):
    n = (1 << 20) - 3
    a = inputs.records(n, 8, 66)
    np.testing.assert_array_equal(_np(bos.orp_host(_host(a), seed=4, z=256, k=k, min_security_bits=0), 8),
                                  bos.to_numpy(bos.orp(bos.from_numpy(a), seed=4, z=256, k=k,
                                                       min_security_bits=0)))


def test_overflow_retries_match_in_core():
    # Z = 32 overflows often at this size; both paths run the same attempts
    # with the same labels
    n = 1 << 14
    a = inputs.records(n, 8, 67)
    retried = 0
    for seed in range(11, 17):
        got, rep = bos.orp_host(_host(a), seed=seed, z=32, max_retries=30, min_security_bits=0, report=True)
        want, wrep = bos.orp(bos.from_numpy(a), seed=seed, z=32, max_retries=30, min_security_bits=0, report=True)
        assert rep["attempts"] == wrep["attempts"]
        retried += rep["attempts"] > 1
        np.testing.assert_array_equal(_np(got, 8), bos.to_numpy(want))
    assert retried > 0


def test_errors():
    a = inputs.records(1000, 8, 68)
    # one routing pass: the in-core calls cover it
    with pytest.raises(bos.BosError) as e:
        bos.orp_host(_host(a), seed=1, z=512)
    assert e.value.status == bos.UNSUPPORTED
    # a device workspace below the minimum
    import ctypes as C
    b = inputs.records(1 << 20, 8, 69)
    t = _host(b)
    out = bos.pinned_empty(t.shape, t.dtype)
    p = bos.params(1, 512, 0, 0)
    hb = bos.lib().bos_host_workspace_bytes(t.shape[0], 8, C.byref(p))
    db = bos.lib().bos_host_device_bytes(t.shape[0], 8, C.byref(p))
    hws = bos.pinned_empty((hb,), torch.uint8)
    dws = torch.empty(db, dtype=torch.uint8, device="cuda")
    st = bos.lib().bos_orp_host(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), t.shape[0], 8, C.byref(p),
                                C.c_void_p(hws.data_ptr()), hb, C.c_void_p(dws.data_ptr()), db - 4096, None, None)
    assert st == bos.WORKSPACE
    st = bos.lib().bos_orp_host(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), t.shape[0], 8, C.byref(p),
                                C.c_void_p(hws.data_ptr()), hb - 1, C.c_void_p(dws.data_ptr()), db, None, None)
    assert st == bos.WORKSPACE
    st = bos.lib().bos_orp_host(C.c_void_p(t.data_ptr()), C.c_void_p(out.data_ptr()), t.shape[0], 8, C.byref(p),
                                C.c_void_p(hws.data_ptr()), hb, C.c_void_p(dws.data_ptr()), db, None, None)
    assert st == bos.OK
    np.testing.assert_array_equal(_np(out, 8), bos.to_numpy(bos.orp(bos.from_numpy(b), seed=1, z=512)))
