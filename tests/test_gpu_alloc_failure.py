"""Failure handling of context creation, forced from the host: with the
library's failure injection (vi_debug_fail_allocs), vi_create is made to
meet an exhausted device at each of its allocations in turn.  Every such
call must return VI_E_NOMEM with no context, release every block it took,
and leave the library usable: a context created afterwards inpaints the clip
exactly as one created before the failures."""
import numpy as np
import pytest
import torch

from paper_1503_05528_amd import synth

pytestmark = pytest.mark.gpu

VI_E_NOMEM = -2


def test_create_fails_cleanly_at_every_allocation():
    from paper_1503_05528_amd import vi
    clip = synth.small(21, 61, 47, 11, levels=2, frac=0.05)
    video = torch.from_numpy(clip.occluded_input()).cuda()
    mask = torch.from_numpy(clip.mask).cuda()
    kw = dict(levels=2, seed=4, recon_mode=1, em_max_iters=3, em_tol=-1.0)
    g = vi.Clip(video, mask, **kw)
    ref = g.inpaint().cpu().numpy()
    g.close()
    live0 = vi.fail_allocs(-1)
    failures = 0
    try:
        for k in range(400):
            print(f"[case] creation with {k} allocations allowed", flush=True)
            vi.fail_allocs(k)
            try:
                c = vi.Clip(video, mask, **kw)
            except vi.ViError as e:
                assert e.status == VI_E_NOMEM, e
                failures += 1
                # nothing kept from the failed call
                assert vi.fail_allocs(-1) == live0
                continue
            vi.fail_allocs(-1)
            out = c.inpaint().cpu().numpy()
            c.close()
            break
        else:
            pytest.fail("creation never succeeded")
    finally:
        vi.fail_allocs(-1)
    assert failures == k and failures > 5
    assert np.array_equal(out, ref)
    assert vi.fail_allocs(-1) == live0
