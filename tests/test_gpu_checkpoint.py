"""Checkpoint and resume through vi_get_state / vi_set_state: an inpainting
stopped after a level, saved to host memory, and resumed in a fresh context
gives the same video, bit for bit, as the uninterrupted run; the steps of
Alg. 4 driven one call at a time give the same video as vi_inpaint."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def finish(vi, g, start_level):
    """EM loops from start_level down to 0, then the final best-patch
    reconstruction; returns the RGB iterate of level 0."""
    for lvl in range(start_level, -1, -1):
        g.inpaint_level(lvl)
        if lvl > 0:
            g.transition(lvl - 1)
    g.reconstruct(0, vi.BEST, want_out=False)
    return host(g.get_state(0)[0])[..., :3]


@pytest.mark.parametrize("mode", [0, 1])
def test_resume_from_a_checkpoint(vi, mode):
    print(f"[case] checkpoint resume recon_mode={mode}", flush=True)
    clip = synth.small(61, 83, 66, 12, levels=3, frac=0.05)
    kw = dict(levels=3, seed=11, recon_mode=mode)
    video, mask = dev(clip.occluded_input()), dev(clip.mask)

    g = vi.Clip(video, mask, **kw)
    ref = host(g.inpaint())
    g.close()

    g = vi.Clip(video, mask, **kw)
    g.onion_init()
    stepped = finish(vi, g, 2)
    g.close()
    assert np.array_equal(stepped, ref)

    g = vi.Clip(video, mask, **kw)
    g.onion_init()
    g.inpaint_level(2)
    g.transition(1)
    saved = [host(t).copy() for t in g.get_state(1)]  # rgbt, cand, dist, nvox
    g.close()

    g = vi.Clip(video, mask, **kw)
    g.set_state(1, *saved)
    resumed = finish(vi, g, 1)
    g.close()
    assert np.array_equal(resumed, ref)
