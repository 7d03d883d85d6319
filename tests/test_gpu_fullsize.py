"""Full-size parity of the GPU path (libbos through its C ABI).

* The duplicate-heavy workload (n = 2^24 records of 16 bytes, keys uniform on
  [0, 2^20), Z = 512): bos_orp and bos_sort compared whole, record by record,
  with the CPU oracle.
* The headline workload (n = 2^28 records of 8 bytes, uniform u32 key, payload
  = index) at every point of the sweep Z in {256, 512, 1024} x k in {2, 3, 4}:
  bos_orp compared whole with the closed form of Section 3.2 (bin = label; a
  bin's records in record order, then ordered by their per-bin keys), computed
  by library sorts; bos_sort compared whole with torch's library sort of the
  input.  Z = 1024 with k = 4 needs 192 KiB of LDS per block and must be
  rejected as unsupported.
"""
import numpy as np
import pytest

import closed_forms as cf
from gpu_util import torch_is_sorted, torch_sorted_records
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos  # noqa: E402


@pytest.fixture(scope="module")
def ora():
    import oracle
    oracle.build(force=False)
    return oracle


def test_orp_whole_duplicate_heavy_workload(ora):
    a = inputs.workload_dup(43)
    want = ora.orp(a, 1, z=512)
    assert want["rc"] == 0
    out, rep = bos.orp(bos.from_numpy(a), seed=1, z=512, report=True)
    assert rep["attempts"] == want["report"]["attempts"]
    assert (rep["buckets"], rep["levels"]) == (want["report"]["buckets"], want["report"]["levels"])
    np.testing.assert_array_equal(bos.to_numpy(out), want["out"])


def test_sort_whole_duplicate_heavy_workload(ora):
    a = inputs.workload_dup(42)
    want = ora.sort(a, 1, z=512)
    assert want["rc"] == 0
    out, rep = bos.sort(bos.from_numpy(a), seed=1, z=512, report=True)
    assert rep["attempts"] == want["report"]["attempts"]
    np.testing.assert_array_equal(bos.to_numpy(out), want["out"])


@pytest.fixture(scope="module")
def headline():
    n = 1 << 28
    a = inputs.records(n, 8, 42)
    x = bos.from_numpy(a)
    ref = torch_sorted_records(x)
    yield a, x, ref
    del x, ref
    bos.release_workspaces()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("z", [256, 512, 1024])
def test_headline_sweep_point_whole(headline, z):
    a, x, ref = headline
    n = a.shape[0]
    out = torch.empty_like(x)
    want = None
    for k in (2, 3, 4):
        if z == 1024 and k == 4:
            with pytest.raises(bos.BosError) as ei:
                bos.sort(x, seed=1, z=z, k=k, out=out, min_security_bits=0)
            assert ei.value.status == bos.UNSUPPORTED
            with pytest.raises(bos.BosError) as ei:
                bos.orp(x, seed=1, z=z, k=k, out=out, min_security_bits=0)
            assert ei.value.status == bos.UNSUPPORTED
            continue
        o, rep = bos.sort(x, seed=1, z=z, k=k, out=out, min_security_bits=0, report=True)
        assert rep["k"] == k and rep["z"] == z
        assert torch_is_sorted(o)
        assert torch.equal(o, ref), (z, k)
        o, rep = bos.orp(x, seed=1, z=z, k=k, out=out, min_security_bits=0, report=True)
        assert rep["k"] == k and rep["z"] == z
        if want is None:
            B, L = rep["buckets"], rep["levels"]
            att = rep["attempts"] - 1
            lab = cf.labels(1, att, n, L)
            want = torch.from_numpy(cf.expected_orp_vec(a, 1, att, lab, B, z, device="cuda").view(np.int32))
            want = want.to(x.device)
            del lab
        assert torch.equal(o, want), (z, k)
    del out, want
