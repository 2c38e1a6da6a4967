"""Pins of the oracle's optional temporal subsampling of the pyramids
(Sec. 3.6: coarser levels may halve the frame count as well, for objects
that stay long behind the occlusion): 2x2x2 box means rounded half up and
OR-pooled occlusions against numpy reshapes (odd frame counts included),
texture features subsampled in time as in space, the level transition's
parent and doubled temporal shift with every inherited match a source, and
a periodic video whose hole content recurs exactly, inpainted bit for bit
through a temporally subsampled pyramid."""
import numpy as np
import pytest

from oracle import vio
from paper_1503_05528_amd import synth


def test_temporal_pyramid_box_mean_and_or_pool(oracle_lib):
    W, H, T = 11, 9, 11
    rng = np.random.default_rng(3)
    v = rng.integers(0, 256, (T, H, W, 3)).astype(np.uint8)
    m = np.zeros((T, H, W), np.uint8)
    m[2, 3, 4] = 1
    m[9, 8, 10] = 1
    m[10, 0, 0] = 1
    o = vio.Oracle(v, m, levels=2, patch=(3, 3, 3), temporal_subsample=1)
    assert o.dims(1) == (6, 5, 6)
    hole1 = o.sets(1)[0]
    rgbt1 = o.get_state(1)[0]
    mp = np.zeros((12, 10, 12), np.uint8)
    mp[:T, :H, :W] = m
    ref = mp.reshape(6, 2, 5, 2, 6, 2).max(axis=(1, 3, 5))
    assert np.array_equal(hole1, ref)
    # every block by hand, the ragged ones (last frame pair holds one frame,
    # last column and row one voxel) included
    for t in range(6):
        for y in range(5):
            for x in range(6):
                if ref[t, y, x]:
                    assert (rgbt1[t, y, x, :3] == 0).all()
                    continue
                blk = v[2 * t:2 * t + 2, 2 * y:2 * y + 2, 2 * x:2 * x + 2].reshape(-1, 3)
                c = blk.shape[0]
                exp = (blk.astype(int).sum(0) + c // 2) // c
                assert np.array_equal(rgbt1[t, y, x, :3], exp), (x, y, t)
    # the corner block (5, 4, 5) is a single voxel: copied exactly
    assert np.array_equal(rgbt1[5, 4, 5, :3], v[10, 8, 10])


def test_temporal_texture_is_subsampled_in_time(oracle_lib):
    c = synth.small(81, 48, 40, 20, levels=3, frac=0.03)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=3, temporal_subsample=1)
    r0 = o.get_state(0)[0]
    for lv in (1, 2):
        W, H, T = o.dims(lv)
        assert T == (20 + (1 << lv) - 1) >> lv
        rl = o.get_state(lv)[0]
        hole = o.sets(lv)[0].astype(bool)
        t, y, x = np.nonzero(~hole)
        assert np.array_equal(rl[t, y, x, 3:], r0[t << lv, y << lv, x << lv, 3:])
        assert (rl[hole][:, 3:] == 0).all()


def test_temporal_transition_doubles_the_time_shift(oracle_lib):
    c = synth.small(82, 52, 44, 18, levels=2, frac=0.05)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=2, seed=2, em_max_iters=2,
                   temporal_subsample=1)
    o.onion_init()
    o.inpaint_level(1)
    o.transition(0)
    _, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    tg = htil.ravel() == 1
    assert (dsrc.ravel()[cand.ravel()[tg]] == 1).all()
    _, cc, cd, cn = o.get_state(1)
    T, H, W = hole.shape
    Tc, Hc, Wc = cc.shape
    assert Tc == 9
    idx = np.flatnonzero(tg)
    x, y, t = idx % W, (idx // W) % H, idx // (W * H)
    par = ((t // 2) * Hc + y // 2) * Wc + x // 2
    assert np.array_equal(dist.ravel()[idx], cd.ravel()[par])
    assert np.array_equal(nvox.ravel()[idx], cn.ravel()[par])
    pc = cc.ravel()[par]
    px, py, pt = pc % Wc, (pc // Wc) % Hc, pc // (Wc * Hc)
    fc = cand.ravel()[idx]
    fx, fy, ft = fc % W, (fc // W) % H, fc // (W * H)
    assert np.array_equal(fx - x, 2 * (px - x // 2))
    assert np.array_equal(fy - y, 2 * (py - y // 2))
    assert np.array_equal(ft - t, 2 * (pt - t // 2))


def test_temporal_periodic_video_is_inpainted_exactly(oracle_lib):
    # spatial period 7, 1 px/frame: 2x2x2 block means keep the content a
    # function of (y, x - t), so exact matches exist at both levels
    P, W, H, T = 7, 40, 36, 12
    rng = np.random.default_rng(0)
    tile = rng.integers(0, 256, (P, P, 3)).astype(np.uint8)
    t, y, x = np.meshgrid(np.arange(T), np.arange(H), np.arange(W), indexing="ij")
    v = tile[y % P, (x - t) % P]
    m = np.zeros((T, H, W), np.uint8)
    m[4:8, 14:22, 16:24] = 1
    o = vio.Oracle(np.where(m[..., None] == 1, 0, v).astype(np.uint8), m, levels=2, lam=0,
                   seed=11, temporal_subsample=1)
    out = o.inpaint()
    assert np.array_equal(out, v)
    assert o.energy(0) == 0


def test_temporal_subsampling_needs_a_patch_deep_coarsest_level(oracle_lib):
    c = synth.small(83, 48, 40, 9, levels=2)
    with pytest.raises(vio.OracleError) as e:  # 9 frames -> 5 -> 3 < 5
        vio.Oracle(c.occluded_input(), c.mask, levels=3, temporal_subsample=1)
    assert e.value.status == -1
    vio.Oracle(c.occluded_input(), c.mask, levels=2, temporal_subsample=1)
