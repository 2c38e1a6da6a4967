"""Pins of the oracle's realignment (Sec. 3.4, Alg. 2, and the inverse warp
of Alg. 4) against what is known independently of it:

* the motion of a scene filmed by a shaking camera is known exactly from
  the cameras (the generator renders every frame from the scene, without
  resampling): the estimated dominant motion of every frame pair matches it
  within 0.05 px at the frame corners, also with moving objects and an
  occlusion in view, and a pure translation is found exactly;
* the composition to the middle frame equals the product of 3x3 homogeneous
  matrices (numpy, with numpy's inverse after the reference);
* the warp of the identity returns the input, an integer translation a
  shifted copy with the uncovered border marked, a linear ramp its exact
  value at the source position (bilinear interpolation is exact on linear
  functions), and every stencil that touches the occlusion is marked;
* the unwarp keeps every known pixel and fills the occluded ones from the
  aligned video at their reference positions.
"""
import numpy as np
import pytest

from oracle import vio
from paper_1503_05528_amd import synth


def H3(m):
    return np.array([[m[0], m[1], m[2]], [m[3], m[4], m[5]], [0.0, 0.0, 1.0]])


def corner_error(a, b, W, H):
    c = np.array([[0, 0, 1], [W - 1, 0, 1], [0, H - 1, 1], [W - 1, H - 1, 1.0]]).T
    return np.abs((H3(a) @ c - H3(b) @ c)[:2]).max()


@pytest.mark.parametrize("seed,n_obj", [(4, 3), (5, 0), (6, 5)])
def test_estimate_recovers_the_camera_motion(oracle_lib, seed, n_obj):
    clip, cams = synth.jittered(seed=seed, W=240, H=180, T=10, n_obj=n_obj)
    T, H, W, _ = clip.video.shape
    th = vio.align_estimate(clip.occluded_input(), clip.mask)
    for n in range(T - 1):
        true = np.linalg.inv(H3(cams[n + 1])) @ H3(cams[n])
        err = corner_error(true[:2].ravel(), th[n], W, H)
        assert err < 0.05, (n, err)


def test_estimate_finds_a_translation(oracle_lib):
    rng = np.random.default_rng(0)
    W, H, T = 200, 150, 3
    # a smooth random field shifted by (3, -2) px per frame
    big = rng.normal(0, 1, (H + 40, W + 40))
    from scipy import ndimage
    big = ndimage.gaussian_filter(big, 3.0)
    big = 128 + 60 * big / big.std()
    v = np.zeros((T, H, W, 3), np.uint8)
    for t in range(T):
        fr = big[20 + 2 * t:20 + 2 * t + H, 20 - 3 * t:20 - 3 * t + W]
        v[t] = np.clip(np.floor(fr + 0.5), 0, 255).astype(np.uint8)[..., None]
    th = vio.align_estimate(v, np.zeros((T, H, W), np.uint8))
    for n in range(T - 1):
        assert corner_error(th[n], [1, 0, 3, 0, 1, -2], W, H) < 0.05, th[n]


def test_compose_is_the_product_to_the_middle_frame(oracle_lib):
    rng = np.random.default_rng(1)
    T = 7
    th = np.zeros((T - 1, 6))
    for n in range(T - 1):
        a = rng.uniform(-0.02, 0.02, 4)
        th[n] = (1 + a[0], a[1], rng.uniform(-3, 3), a[2], 1 + a[3], rng.uniform(-3, 3))
    M = vio.align_compose(th, T)
    ref = T // 2
    for n in range(T):
        P = np.eye(3)
        if n < ref:
            for k in range(n, ref):
                P = H3(th[k]) @ P
        elif n > ref:
            for k in range(ref, n):
                P = P @ np.linalg.inv(H3(th[k]))
        assert np.allclose(H3(M[n]), P, rtol=0, atol=1e-9), n
    # a frame's map followed by the reference's inverse chain is consistent:
    # M_n = M_{n+1} o theta_n for every n
    for n in range(T - 1):
        assert np.allclose(H3(M[n + 1]) @ H3(th[n]), H3(M[n]), atol=1e-9)


def _video(W=40, H=30, T=3, seed=2):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, (T, H, W, 3)).astype(np.uint8)


def test_warp_identity_and_integer_shift(oracle_lib):
    v = _video()
    T, H, W, _ = v.shape
    m = np.zeros((T, H, W), np.uint8)
    m[1, 10:14, 20:25] = 1
    M = np.tile([1.0, 0, 0, 0, 1.0, 0], (T, 1))
    out, om = vio.align_warp(v, m, M)
    assert np.array_equal(om, m)
    assert np.array_equal(out[m == 0], v[m == 0])
    # M maps the frame's pixel x to x + (3, -2): aligned y shows x = y - (3, -2)
    M[:] = [1.0, 0, 3.0, 0, 1.0, -2.0]
    out, om = vio.align_warp(v, np.zeros_like(m), M)
    assert np.array_equal(out[:, 0:H - 2, 3:], v[:, 2:, :W - 3])
    assert om[:, :, :3].all() and om[:, H - 2:, :].all()
    assert not om[:, 0:H - 2, 3:].any()


def test_warp_is_exact_on_a_linear_ramp(oracle_lib):
    W, H, T = 60, 50, 2
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")
    v = np.zeros((T, H, W, 3), np.uint8)
    v[..., 1] = (x + 2 * y + 5).astype(np.uint8)  # at most 162: no clipping
    M = np.array([[1.01, 0.02, 1.3, -0.015, 0.99, -0.7]] * T)
    out, om = vio.align_warp(v, np.zeros((T, H, W), np.uint8), M)
    inv = np.linalg.inv(H3(M[0]))
    xs = inv[0, 0] * x + inv[0, 1] * y + inv[0, 2]
    ys = inv[1, 0] * x + inv[1, 1] * y + inv[1, 2]
    ok = om[0] == 0
    assert ok.mean() > 0.8
    want = np.floor(xs + 2 * ys + 5 + 0.5)
    assert np.array_equal(out[0, ..., 1][ok], want[ok].astype(np.uint8))
    # the marked pixels are exactly those whose source leaves the frame
    inside = (xs >= 0) & (ys >= 0) & (np.ceil(xs) <= W - 1) & (np.ceil(ys) <= H - 1)
    assert np.array_equal(ok, inside)


def test_warp_marks_stencils_that_touch_the_occlusion(oracle_lib):
    v = _video(W=30, H=24, T=1)
    m = np.zeros((1, 24, 30), np.uint8)
    m[0, 10, 12] = 1
    M = np.array([[1.0, 0, 0.5, 0, 1.0, 0.25]])  # source = y - (0.5, 0.25)
    out, om = vio.align_warp(v, m, M)
    # x = y - 0.5 uses columns floor and floor + 1, rows likewise
    want = np.zeros((24, 30), bool)
    for yy in range(24):
        for xx in range(30):
            xs, ys = xx - 0.5, yy - 0.25
            x0, y0 = int(np.floor(xs)), int(np.floor(ys))
            cols = [x0, x0 + 1]
            rows = [y0, y0 + 1]
            if x0 < 0 or y0 < 0 or x0 + 1 > 29 or y0 + 1 > 23:
                want[yy, xx] = True
            elif any(m[0, r, c] for r in rows for c in cols):
                want[yy, xx] = True
    assert np.array_equal(om[0].astype(bool), want)


def test_unwarp_keeps_known_pixels_and_fills_the_hole(oracle_lib):
    W, H, T = 50, 40, 3
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")
    ramp = (2 * x + 3 * y + 5).astype(np.uint8)
    aligned = np.repeat(np.repeat(ramp[None, ..., None], T, 0), 3, -1)
    v = _video(W, H, T)
    m = np.zeros((T, H, W), np.uint8)
    m[:, 15:25, 20:30] = 1
    M = np.array([[1.0, 0.0, 1.5, 0.0, 1.0, -0.5]] * T)
    out = vio.align_unwarp(aligned, v, m, M)
    assert np.array_equal(out[m == 0], v[m == 0])
    xs, ys = x + 1.5, y - 0.5
    want = np.floor(2 * xs + 3 * ys + 5 + 0.5).astype(np.uint8)
    for t in range(T):
        hole = m[t] == 1
        assert np.array_equal(out[t, ..., 2][hole], want[hole])
