"""Tuning table (bos_set_tuning): plans that leave z, k or tile at 0 take
them from the table, per instance, in the single, batched and step paths;
results stay bit-exact against the oracle."""
import numpy as np
import pytest

import closed_forms as cf
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos, serving  # noqa: E402


@pytest.fixture
def table():
    yield
    bos.set_tuning([])


TABLE = [
    {"rec": 8, "log2n": 12, "z": 256, "k": 2, "tile": 1024},
    {"rec": 8, "log2n": 16, "z": 1024, "k": 3, "tile": 2048},
    {"rec": 8, "log2n": 20, "z": 512, "k": 4, "tile": 4096},
    {"rec": 16, "log2n": 14, "z": 512, "k": 2, "tile": 2048},
]


def test_table_round_trip_and_validation(table):
    bos.set_tuning(TABLE)
    assert bos.get_tuning() == TABLE
    for bad in ({"rec": 12, "log2n": 10, "z": 512}, {"rec": 8, "log2n": 10, "z": 500},
                {"rec": 8, "log2n": 10, "z": 512, "tile": 3000}, {"rec": 8, "log2n": 10, "k": 13}):
        with pytest.raises(bos.BosError):
            bos.set_tuning([bad])
    assert bos.get_tuning() == TABLE
    bos.set_tuning([])
    assert bos.get_tuning() == []


@pytest.mark.parametrize("n,want", [(4096, (256, 2, 1024)), (3000, (256, 2, 1024)), (1 << 16, (1024, 3, 2048)),
                                    (50000, (1024, 3, 2048)), (1 << 20, (512, 4, 4096)), (1 << 22, (512, 4, 4096))])
def test_single_sort_takes_nearest_class(table, n, want):
    import oracle
    oracle.build(force=False)
    bos.set_tuning(TABLE)
    h = inputs.records(n, 8, 17)
    out, rep = bos.sort(bos.from_numpy(h), seed=3, min_security_bits=0, report=True)
    assert (rep["z"], rep["k"], rep["tile"]) == want
    np.testing.assert_array_equal(bos.to_numpy(out), cf.sorted_records(h))
    # bos_orp with the tuned Z is the oracle's permutation at that Z
    if n <= 1 << 16:
        got = bos.to_numpy(bos.orp(bos.from_numpy(h), seed=3, min_security_bits=0))
        np.testing.assert_array_equal(got, oracle.orp(h, 3, z=want[0])["out"])


def test_security_floor_raises_tuned_z(table):
    # Z = 256 at n = 2^12 gives log2 eps ~ -54: at an 80-bit floor the plan
    # doubles it to 512
    bos.set_tuning(TABLE)
    h = inputs.records(4096, 8, 5)
    _, rep = bos.sort(bos.from_numpy(h), seed=1, report=True)
    assert rep["z"] == 512
    _, rep = bos.sort(bos.from_numpy(h), seed=1, min_security_bits=40, report=True)
    assert rep["z"] == 256


def test_explicit_parameters_override_table(table):
    bos.set_tuning(TABLE)
    h = inputs.records(1 << 16, 8, 9)
    _, rep = bos.sort(bos.from_numpy(h), seed=1, z=512, k=4, tile=4096, min_security_bits=0, report=True)
    assert (rep["z"], rep["k"], rep["tile"]) == (512, 4, 4096)


def test_batched_mixed_tuned_plans(table):
    # instances in different size classes get different Z, k and tile inside
    # one batch (routing launches grouped by Z, tile sorts by tile)
    bos.set_tuning(TABLE)
    sizes = [4096, 1 << 16, 3000, 70000, 1 << 20, 5, 0, 50000]
    hosts = [inputs.records(n, 8, 700 + i) for i, n in enumerate(sizes)]
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], [10 + i for i in range(len(hosts))],
                            min_security_bits=0)
    for h, o in zip(hosts, outs):
        np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))


def test_step_mixed_tuned_plans(table):
    bos.set_tuning(TABLE)
    sizes = [4096, 1 << 16, 3000, 70000, 1 << 20, 9000]
    hosts = [inputs.records(n, 8, 800 + i) for i, n in enumerate(sizes)]
    srv = serving.Server(hbm_budget_bytes=1 << 34, min_security_bits=0)
    futs = [srv.submit(bos.from_numpy(h), seed=i) for i, h in enumerate(hosts)]
    srv.run_until_idle()
    for h, f in zip(hosts, futs):
        np.testing.assert_array_equal(bos.to_numpy(f.result()), cf.sorted_records(h))


@pytest.mark.parametrize("rec", [8, 16])
@pytest.mark.parametrize("tile", [1024, 2048, 4096, 8192, 16384])
@pytest.mark.parametrize("n", [1, 1000, 1024, 1025, 2049, 4097, 8193, 10000, 16385, 1 << 15, 100003])
def test_tile_sizes(rec, tile, n):
    h = inputs.records(n, rec, 33 + n, key_bits=12)
    if rec == 16 and tile == 16384:
        # a 16384-record tile of 16-byte records does not fit a workgroup's LDS
        with pytest.raises(bos.BosError) as e:
            bos.sort(bos.from_numpy(h), seed=1, tile=tile, min_security_bits=0)
        assert e.value.status == bos.INVALID_ARG
        return
    out = bos.sort(bos.from_numpy(h), seed=1, tile=tile, min_security_bits=0)
    np.testing.assert_array_equal(bos.to_numpy(out), cf.sorted_records(h))


@pytest.mark.parametrize("tile", [8192, 16384])
def test_big_tiles_batched_and_step(table, tile):
    bos.set_tuning([{"rec": 8, "log2n": c, "z": 512, "k": 3, "tile": tile} for c in (12, 16, 20)])
    sizes = [5000, 1 << 16, 70000, 1 << 20, 3, 16385]
    hosts = [inputs.records(n, 8, 900 + i) for i, n in enumerate(sizes)]
    outs = bos.sort_batched([bos.from_numpy(h) for h in hosts], [1 + i for i in range(len(hosts))],
                            min_security_bits=0)
    for h, o in zip(hosts, outs):
        np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))
    srv = serving.Server(hbm_budget_bytes=1 << 34, min_security_bits=0)
    futs = [srv.submit(bos.from_numpy(h), seed=i) for i, h in enumerate(hosts)]
    srv.run_until_idle()
    for h, f in zip(hosts, futs):
        np.testing.assert_array_equal(bos.to_numpy(f.result()), cf.sorted_records(h))
