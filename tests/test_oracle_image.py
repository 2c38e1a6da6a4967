"""Pins of the oracle on single images (T = 1, 5x5x1 patches): the method
applied to 2-D image inpainting (Sec. 3.1 and 3.5 discuss the image case).
The source and target sets against 2-D scipy morphology, distances by hand
(flat colours, border truncation to the in-frame 5x5 window), searches
against exact nearest neighbours by brute force, and a periodic image whose
hole content recurs exactly, inpainted bit for bit."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import vio
from paper_1503_05528_amd import synth

P2 = dict(patch=(5, 5, 1))


def test_image_sets_match_2d_morphology(oracle_lib):
    c = synth.image(91, 61, 47, frac=0.06, levels=1)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1, **P2)
    hole, dsrc, htil = o.sets(0)
    m = c.mask[0].astype(bool)
    want_t = ndimage.binary_dilation(m, np.ones((5, 5), bool))
    inner = np.zeros_like(m)
    inner[2:-2, 2:-2] = True
    want_d = inner & ~want_t
    assert np.array_equal(htil[0].astype(bool), want_t)
    assert np.array_equal(dsrc[0].astype(bool), want_d)


def test_image_distance_by_hand(oracle_lib):
    W, H = 26, 12
    v = np.zeros((1, H, W, 3), np.uint8)
    v[:, :, :13] = (10, 20, 30)
    v[:, :, 13:] = (13, 16, 30)
    m = np.zeros((1, H, W), np.uint8)
    m[0, 0, 25] = 1  # a hole voxel far away, so that the sets exist
    o = vio.Oracle(v, m, levels=1, lam=0, **P2)
    p = (0 * H + 6) * W + 5
    c = (0 * H + 6) * W + 20
    assert o.patch_ssd(0, p, c) == (25 * (3 * 3 + 4 * 4), 25)
    # a corner target compares its in-frame 3x3 window only
    assert o.patch_ssd(0, 0, c) == (9 * (3 * 3 + 4 * 4), 9)


def _brute(rgbt, dsrc, targets, lam):
    H, W = dsrc.shape[1:]
    src = np.flatnonzero(dsrc.ravel())
    w = np.array([1, 1, 1, lam, lam], np.int64)
    best = np.full(len(targets), np.iinfo(np.int64).max)
    for s_ in src:
        sx, sy = s_ % W, s_ // W
        d = np.zeros(len(targets), np.int64)
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                tx, ty = targets % W + dx, targets // W + dy
                ok = (tx >= 0) & (tx < W) & (ty >= 0) & (ty < H)
                a = rgbt[0, np.clip(ty, 0, H - 1), np.clip(tx, 0, W - 1)].astype(np.int64)
                b = rgbt[0, sy + dy, sx + dx].astype(np.int64)
                d += np.where(ok, ((a - b) ** 2 * w).sum(-1), 0)
        best = np.minimum(best, d)
    return best


def test_image_search_vs_brute_force(oracle_lib):
    c = synth.image(92, 40, 32, frac=0.05, levels=1)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1, seed=3, **P2)
    o.onion_init()
    o.nnf_search(0, 0)
    rgbt, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    tg = np.flatnonzero(htil.ravel())
    exact = _brute(rgbt, dsrc, tg, 50)
    got = dist.ravel()[tg].astype(np.int64)
    assert (got >= exact).all()
    assert (got == exact).mean() > 0.5
    assert (dsrc.ravel()[cand.ravel()[tg]] == 1).all()


@pytest.mark.parametrize("levels", [1, 2])
def test_periodic_image_is_inpainted_exactly(oracle_lib, levels):
    P, W, H = 7, 48, 40
    rng = np.random.default_rng(0)
    tile = rng.integers(0, 256, (P, P, 3)).astype(np.uint8)
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    v = tile[y % P, x % P][None]
    m = np.zeros((1, H, W), np.uint8)
    m[0, 15:24, 18:27] = 1
    o = vio.Oracle(np.where(m[..., None] == 1, 0, v).astype(np.uint8), m, levels=levels,
                   lam=0, seed=11, **P2)
    out = o.inpaint()
    assert np.array_equal(out, v)
    assert o.energy(0) == 0
