"""Device memory kept across contexts (vi_pool_trim): a context built from
blocks that held another context's data gives the same results as one built
from fresh allocations, and trimming returns the cache to the device."""
import numpy as np
import pytest
import torch

from paper_1503_05528_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vi():
    from paper_1503_05528_amd import vi as _vi
    _vi.lib()
    return _vi


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(vi, clip, **kw):
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), **kw)
    out = g.inpaint().cpu().numpy()
    nbytes = g.nbytes()
    g.close()
    return out, nbytes


def test_reused_blocks_give_identical_results(vi):
    print("[case] pool reuse", flush=True)
    a = synth.small(51, 72, 56, 12, levels=2, frac=0.05)
    b = synth.small(52, 90, 40, 10, levels=2, frac=0.04, kind="box")
    kw = dict(levels=2, seed=3)
    vi.pool_trim()
    ref_a, na = run(vi, a, **kw)  # fresh allocations
    ref_b, _ = run(vi, b, **kw)   # partly reuses a's blocks
    for _ in range(2):
        out_a, na2 = run(vi, a, **kw)
        out_b, _ = run(vi, b, **kw)
        assert np.array_equal(out_a, ref_a)
        assert np.array_equal(out_b, ref_b)
        assert na2 == na
    assert vi.pool_trim() > 0
    assert vi.pool_trim() == 0
    out_a, _ = run(vi, a, **kw)
    assert np.array_equal(out_a, ref_a)
