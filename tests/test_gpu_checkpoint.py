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


def test_rejected_set_state_keeps_the_level(vi):
    # a match outside [-1, V) is refused before anything is written, so the
    # level keeps its searched state; a match inside the volume that is not
    # a source leaves the level incomplete, and the reconstruction refuses
    # it on the host (no kernel reads through that match)
    print("[case] rejected set_state", flush=True)
    clip = synth.small(62, 50, 40, 9, levels=1, frac=0.05)
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=1, seed=4, recon_mode=1)
    g.onion_init()
    g.nnf_search(0, 1)
    before = [host(t).copy() for t in g.get_state(0)]
    cand = before[1]
    tgt = np.flatnonzero(cand.ravel() >= 0)
    assert tgt.size > 0
    bad = cand.copy()
    bad.ravel()[tgt[tgt.size // 2]] = cand.size  # one past the last voxel
    with pytest.raises(vi.ViError) as e:
        g.set_state(0, cand=bad)
    assert e.value.status == -1
    after = [host(t) for t in g.get_state(0)]
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    g.reconstruct(0, vi.MEAN, want_out=False)  # still complete
    _, dsrc, _ = g.sets(0)
    nonsrc = cand.copy()
    nonsrc.ravel()[tgt[0]] = int(np.flatnonzero(host(dsrc).ravel() == 0)[0])
    g.set_state(0, cand=nonsrc)
    with pytest.raises(vi.ViError) as e:
        g.reconstruct(0, vi.MEAN, want_out=False)
    assert e.value.status == -4
    g.close()
