"""Pins of the oracle's reconstruction (Sec. 3.2, Eqs. (3.2)-(3.4)), level
loop (Alg. 4), transition (Sec. 3.6) and the complete algorithm against closed
forms: hand-built votes with known weights, the nearest-rank 75th percentile
of numpy, a float64 recomputation, and a periodic video whose hole content
recurs exactly elsewhere, which the method must reproduce bit for bit."""
import math

import numpy as np
import pytest

from oracle import vio
from paper_1503_05528_amd import synth

A = np.array([40, 90, 200])
B = np.array([220, 30, 10])


def _single_hole_setup(W=30, H=16, T=9):
    """Flat colour A on the left, flat colour B on the right, a one-voxel hole
    at p = (15, 8, 4).  Returns the oracle, p's coordinates, and a source
    centre inside each flat region."""
    v = np.zeros((T, H, W, 3), np.uint8)
    v[:, :, :11] = A
    v[:, :, 11:20] = 77
    v[:, :, 20:] = B
    m = np.zeros((T, H, W), np.uint8)
    m[4, 8, 15] = 1
    o = vio.Oracle(v, m, levels=1)
    a_src = (4 * H + 8) * W + 5
    b_src = (4 * H + 8) * W + 25
    return o, (15, 8, 4), a_src, b_src, (W, H, T)


def _offsets(h=2):
    return [(dx, dy, dt) for dt in range(-h, h + 1) for dy in range(-h, h + 1)
            for dx in range(-h, h + 1)]


def _set_votes(o, p, dims, assign):
    """assign(index, offset) -> (source centre, dist, nvox) for the
    contributor q = p - offset."""
    W, H, T = dims
    rgbt, cand, dist, nvox = o.get_state(0)
    cand[:] = -1
    dist[:] = -1
    nvox[:] = 0
    px, py, pt = p
    for i, (dx, dy, dt) in enumerate(_offsets()):
        q = ((pt - dt) * H + (py - dy)) * W + (px - dx)
        s, d, n = assign(i, (dx, dy, dt))
        cand.ravel()[q] = s
        dist.ravel()[q] = d
        nvox.ravel()[q] = n
    o.set_state(0, cand=cand, dist=dist, nvox=nvox)


def test_weighted_two_groups_closed_form(oracle_lib):
    o, p, a, b, dims = _single_hole_setup()
    d = 125 * 37
    # 93 exact votes for A, 32 votes for B at normalised distance 37:
    # the 94th smallest (nearest rank of 75 % of 125) is 37 = sigma^2, so the
    # B votes weigh exp(-1/2).
    _set_votes(o, p, dims, lambda i, off: (a, 0, 125) if i < 93 else (b, d, 125))
    out, _ = o.reconstruct(0, vio.WEIGHTED)
    wb = 32 * math.exp(-0.5)
    ref = (93 * A + wb * B) / (93 + wb)
    assert np.allclose(out[0, :3] * 255, ref, atol=2e-4)
    assert np.allclose(out[0, 3:], 0)
    rgbt = o.get_state(0)[0]
    assert np.array_equal(rgbt[p[2], p[1], p[0], :3], np.floor(ref + 0.5).astype(int))


def test_weighted_sigma_zero_keeps_exact_votes(oracle_lib):
    o, p, a, b, dims = _single_hole_setup()
    # 94 exact votes: the 94th smallest distance is 0, only exact votes count
    _set_votes(o, p, dims, lambda i, off: (a, 0, 125) if i < 94 else (b, 999, 125))
    out, _ = o.reconstruct(0, vio.WEIGHTED)
    assert np.array_equal(np.rint(out[0, :3] * 255), A)
    assert np.allclose(out[0, :3] * 255, A, atol=1e-4)


def test_mean_is_the_plain_average(oracle_lib):
    o, p, a, b, dims = _single_hole_setup()
    _set_votes(o, p, dims, lambda i, off: (a, 5 * i, 125) if i < 93 else (b, 7, 125))
    out, _ = o.reconstruct(0, vio.MEAN)
    ref = (93 * A + 32 * B) / 125
    assert np.allclose(out[0, :3] * 255, ref, atol=1e-4)


def test_best_takes_the_first_smallest(oracle_lib):
    o, p, a, b, dims = _single_hole_setup()
    # unique minimum at contributor 70 (votes B); a tie at 71 comes later.
    # Distances are compared as dist/n: 300/100 = 3 < 400/125 = 3.2.
    def f(i, off):
        if i == 70:
            return (b, 300, 100)
        if i == 71:
            return (a, 300, 100)
        return (a, 400, 125)
    _set_votes(o, p, dims, f)
    out, _ = o.reconstruct(0, vio.BEST)
    assert np.array_equal(np.rint(out[0, :3] * 255), B)


def test_vote_reads_the_shifted_voxel(oracle_lib):
    # each contributor q votes u(cand(q) + (p - q)): with a horizontal ramp
    # as the only source region, contributor with offset dx votes ramp(x0+dx)
    W, H, T = 40, 16, 9
    v = np.zeros((T, H, W, 3), np.uint8)
    for x in range(W):
        v[:, :, x] = 3 * x
    m = np.zeros((T, H, W), np.uint8)
    m[4, 8, 33] = 1
    o = vio.Oracle(v, m, levels=1, lam=0)
    src = (4 * H + 8) * W + 12
    # only the contributor with offset (dx=+2, 0, 0) has distance 0
    _set_votes(o, (33, 8, 4), (W, H, T),
               lambda i, off: (src, 0 if off == (2, 0, 0) else 50, 125))
    out, _ = o.reconstruct(0, vio.BEST)
    assert round(out[0, 0] * 255) == 3 * (12 + 2)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_weighted_matches_float64_with_numpy_percentile(oracle_lib, seed):
    o, p, a, b, dims = _single_hole_setup()
    rng = np.random.default_rng(seed)
    dist = rng.integers(0, 20000, 125)
    nv = rng.integers(60, 126, 125)
    src = [a if rng.uniform() < 0.6 else b for _ in range(125)]
    _set_votes(o, p, dims, lambda i, off: (src[i], int(dist[i]), int(nv[i])))
    out, _ = o.reconstruct(0, vio.WEIGHTED)
    delta = dist / nv
    sig2 = np.percentile(delta, 75, method="inverted_cdf")
    w = np.exp(-delta / (2 * sig2))
    votes = np.array([A if s == a else B for s in src], np.float64)
    ref = (w[:, None] * votes).sum(0) / w.sum()
    assert np.allclose(out[0, :3] * 255, ref, rtol=0, atol=1e-3)


def _periodic(P=7, W=40, H=36, T=10, seed=0):
    rng = np.random.default_rng(seed)
    tile = rng.integers(0, 256, (P, P, 3)).astype(np.uint8)
    t, y, x = np.meshgrid(np.arange(T), np.arange(H), np.arange(W), indexing="ij")
    v = tile[y % P, (x - t) % P]
    m = np.zeros((T, H, W), np.uint8)
    m[3:7, 14:22, 16:24] = 1
    return v, m


@pytest.mark.parametrize("levels", [1, 2])
def test_periodic_video_is_inpainted_exactly(oracle_lib, levels):
    # every hole patch recurs exactly outside the hole (spatial period 7,
    # 1 px/frame motion), so the exact-match shift map has energy 0 and both
    # the weighted mean and the best patch return the true colours.
    v, m = _periodic()
    o = vio.Oracle(np.where(m[..., None] == 1, 0, v).astype(np.uint8), m, levels=levels,
                   lam=0, seed=11)
    out = o.inpaint()
    assert np.array_equal(out, v)
    assert o.energy(0) == 0


def test_outside_hole_untouched_and_hole_values_never_read(oracle_lib):
    c = synth.small(7, 40, 32, 10, levels=2)
    o1 = vio.Oracle(c.occluded_input(0), c.mask, levels=2, seed=5)
    o2 = vio.Oracle(c.occluded_input(None), c.mask, levels=2, seed=5)
    rng = np.random.default_rng(1)
    junk = c.video.copy()
    junk[c.mask == 1] = rng.integers(0, 256, (int(c.mask.sum()), 3))
    o3 = vio.Oracle(junk, c.mask, levels=2, seed=5)
    a, b, d = o1.inpaint(), o2.inpaint(), o3.inpaint()
    assert np.array_equal(a, b) and np.array_equal(a, d)
    keep = c.mask == 0
    assert np.array_equal(a[keep], c.video[keep])


def test_stopping_rule(oracle_lib):
    c = synth.small(8, 36, 30, 9, levels=1)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1, em_tol=1e9, em_max_iters=20)
    o.onion_init()
    assert o.inpaint_level(0) == 1  # e <= tol after the first iteration
    o2 = vio.Oracle(c.occluded_input(), c.mask, levels=1, em_tol=-1.0, em_max_iters=7)
    o2.onion_init()
    assert o2.inpaint_level(0) == 7
    v, m = _periodic()
    o3 = vio.Oracle(v, m, levels=1, lam=0, seed=11)
    o3.onion_init()
    k = o3.inpaint_level(0)
    assert 1 <= k < 20  # the periodic case converges below 0.1


def test_transition_keeps_matches_valid(oracle_lib):
    c = synth.small(9, 52, 44, 10, levels=2, frac=0.05)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=2, seed=2, em_max_iters=2)
    o.onion_init()
    o.inpaint_level(1)
    o.transition(0)
    _, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    tg = htil.ravel() == 1
    assert (dsrc.ravel()[cand.ravel()[tg]] == 1).all()
    # inherited distances and counts are the parents'
    _, cc, cd, cn = o.get_state(1)
    T, H, W = hole.shape
    idx = np.flatnonzero(tg)
    x, y, t = idx % W, (idx // W) % H, idx // (W * H)
    Hc, Wc = cc.shape[1], cc.shape[2]
    par = (t * Hc + y // 2) * Wc + x // 2
    assert np.array_equal(dist.ravel()[idx], cd.ravel()[par])
    assert np.array_equal(nvox.ravel()[idx], cn.ravel()[par])
    # shift doubled in space, kept in time
    pc = cc.ravel()[par]
    px, py, pt = pc % Wc, (pc // Wc) % Hc, pc // (Wc * Hc)
    fc = cand.ravel()[idx]
    fx, fy, ft = fc % W, (fc // W) % H, fc // (W * H)
    assert np.array_equal(fx - x, 2 * (px - x // 2))
    assert np.array_equal(fy - y, 2 * (py - y // 2))
    assert np.array_equal(ft - t, pt - t)


def test_reconstruct_needs_a_complete_map(oracle_lib):
    c = synth.small(10, 36, 30, 9, levels=1)
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1)
    with pytest.raises(vio.OracleError) as e:
        o.reconstruct(0)
    assert e.value.status == -4
