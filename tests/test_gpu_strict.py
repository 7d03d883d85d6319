"""Strict mode (BOS_STRICT, Section 4.1): one butterfly level per pass, so a
workgroup's working set is one MergeSplit's 2Z slots and no LDS state crosses
levels.  The plan must have L passes of one level; outputs equal the oracle's
(ORP) and the library sort (sort), exactly as without the flag."""
import numpy as np
import pytest

import closed_forms as cf
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos  # noqa: E402


@pytest.mark.parametrize("n,rec,z", [(1 << 16, 8, 512), (100000, 16, 256), (1 << 18, 8, 1024), (3000, 8, 64),
                                     (300, 16, 512), (1 << 20, 16, 512)])
def test_strict_plan_and_outputs(n, rec, z):
    import oracle
    oracle.build(force=False)
    pl = bos.plan(n, rec, z=z, min_security_bits=0, strict=True)
    assert pl["passes"] == ([1] * pl["levels"] if pl["levels"] else [0])
    a = inputs.records(n, rec, 42)
    x = bos.from_numpy(a)
    out, rep = bos.orp(x, seed=3, z=z, min_security_bits=0, strict=True, report=True)
    assert rep["k"] == 1 or pl["levels"] == 0
    assert rep["passes"] == max(1, pl["levels"])
    want = oracle.orp(a, 3, z=z)["out"]
    np.testing.assert_array_equal(bos.to_numpy(out), want)
    assert torch.equal(out, bos.orp(x, seed=3, z=z, min_security_bits=0))  # same permutation as k = 3
    s = bos.sort(x, seed=3, z=z, min_security_bits=0, strict=True)
    np.testing.assert_array_equal(bos.to_numpy(s), cf.sorted_records(a))


def test_strict_rejects_fused_levels():
    x = bos.from_numpy(inputs.records(1 << 12, 8, 1))
    with pytest.raises(bos.BosError) as ei:
        bos.orp(x, seed=1, z=64, k=2, min_security_bits=0, strict=True)
    assert ei.value.status == bos.INVALID_ARG
    bos.orp(x, seed=1, z=64, k=1, min_security_bits=0, strict=True)
