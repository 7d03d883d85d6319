"""bos_sort_noalloc (the entry point that allocates nothing) through the C ABI:
its output equals bos_sort's, record for record, on two calls in a row (the
second with a smaller input, so the library's workspace holds the first
call's contents), for both record sizes; sizes beyond its 64 MiB workspace are
rejected before anything runs."""
import numpy as np
import pytest

from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def set_up_on_device():
    # The first call on a device looks up the array's device address, which
    # maps the library's code object holding it (once per device and
    # process); the calls measured below come after it.
    x = bos.from_numpy(inputs.records(64, 8, 1))
    bos.sort_noalloc(x, seed=1, z=512)
    torch.cuda.synchronize()


@pytest.mark.parametrize("rec,sizes", [(8, [1 << 20, 100003]), (16, [1 << 19, 5000])])
def test_noalloc_matches_bos_sort(rec, sizes):
    for n in sizes:
        a = inputs.records(n, rec, 42 + n, key_bits=(20 if rec == 16 else None))
        x = bos.from_numpy(a)
        want = bos.to_numpy(bos.sort(x, seed=3, z=512))
        out = torch.empty_like(x)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        got, rep = bos.sort_noalloc(x, seed=3, z=512, out=out, report=True)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # no device memory taken by the call
        assert got.data_ptr() == out.data_ptr()
        assert rep["attempts"] >= 1 and rep["z"] == 512
        np.testing.assert_array_equal(bos.to_numpy(got), want)


def test_noalloc_small_and_empty():
    for n in (0, 1, 3, 700):
        a = inputs.records(n, 8, 7)
        x = bos.from_numpy(a) if n else torch.zeros((0, 2), dtype=torch.int32, device="cuda")
        got = bos.sort_noalloc(x, seed=1, z=512)
        if n:
            np.testing.assert_array_equal(bos.to_numpy(got), bos.to_numpy(bos.sort(x, seed=1, z=512)))


def test_noalloc_rejects_sizes_beyond_its_workspace():
    x = torch.zeros((1 << 21, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(bos.BosError) as ei:
        bos.sort_noalloc(x, seed=1, z=512)
    assert ei.value.status == bos.WORKSPACE
