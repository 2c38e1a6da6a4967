"""Reconstructions that keep the pixels whose 125 contributing patches kept
their match, distance and voxel count since the previous reconstruction of
the same kind (Eq. 6 / Eq. 7 depend on nothing else: the source voxels never
change).  After every EM loop and after a search followed by a
reconstruction through the public entry points, a full recomputation (a
reconstruction with float output skips nothing) must leave the video as it is,
bit for bit, with a zero |change| sum."""
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


def recompute_changes_nothing(vi, g, level, mode):
    before = host(g.get_state(level)[0]).copy()
    _, absdiff = g.reconstruct(level, mode, want_out=True)
    assert int(host(absdiff)[0]) == 0
    assert np.array_equal(host(g.get_state(level)[0]), before)


@pytest.mark.parametrize("mode", [0, 1])
def test_skipping_reconstruction_equals_full_recomputation(vi, mode):
    print(f"[case] reconstruction skip recon_mode={mode}", flush=True)
    clip = synth.small(71, 96, 72, 14, levels=3, frac=0.06)
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=3, seed=5,
                recon_mode=mode, em_tol=-1.0, em_max_iters=5)
    g.onion_init()
    for lvl in (2, 1, 0):
        assert g.inpaint_level(lvl) == 5
        recompute_changes_nothing(vi, g, lvl, mode)
        # further EM iterations through the public search and reconstruction
        for k in range(5, 8):
            g.nnf_search(lvl, em_iter=k)
            g.reconstruct(lvl, mode, want_out=False)
        recompute_changes_nothing(vi, g, lvl, mode)
        if lvl > 0:
            g.transition(lvl - 1)
    g.close()
