"""Seeded synthetic clips standing in for the paper's test videos.

The paper's own sequences (Sec. 4, execution-time table: Beach Umbrella
264x68x98 ... Museum 1120x754x200) are not available, so every workload
here is generated from a seed: panning sinusoidal-grating backgrounds with
Gaussian noise, rigid randomly textured objects on linear paths, an optional
periodic dynamic-texture region, and moving occlusion tubes.

This module holds none of the inpainting arithmetic.  It only produces
uint8 RGB videos ``[T][H][W][3]`` and uint8 occlusion masks ``[T][H][W]``
(1 = occluded).  Both the oracle and the HIP path consume the same arrays.
All float fields are rounded half-up and clipped to 0..255.
"""

from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import math
import os

import numpy as np


@dataclasses.dataclass
class Clip:
    name: str
    video: np.ndarray  # uint8 [T][H][W][3], ground truth everywhere
    mask: np.ndarray  # uint8 [T][H][W], 1 = occluded
    levels: int
    seed: int

    @property
    def shape(self):
        T, H, W, _ = self.video.shape
        return W, H, T

    def occluded_input(self, fill: int | None = 0) -> np.ndarray:
        """The video with the occluded voxels overwritten (the inpainter
        never reads them, so any fill is allowed)."""
        v = self.video.copy()
        if fill is not None:
            v[self.mask.astype(bool)] = fill
        return v


def _u8(a: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(a + 0.5), 0, 255).astype(np.uint8)


# ----------------------------------------------------------------------------
# tiny 32x32x8 clip (brute-force exact NNF is feasible on it)
# ----------------------------------------------------------------------------

def tiny(seed: int = 1) -> Clip:
    """32x32 px x 8 frames: sinusoidal background drifting 0.5 px/frame, two
    6x6 uniformly textured squares moving 1 px/frame in opposite directions,
    occlusion = the 8x8x4 box x,y in [12,20), t in [2,6)."""
    rng = np.random.default_rng(seed)
    W, H, T = 32, 32, 8
    t, y, x = np.meshgrid(np.arange(T), np.arange(H), np.arange(W), indexing="ij")
    bg = np.empty((T, H, W, 3))
    for c in range(3):
        bg[..., c] = (128 + 60 * np.sin(2 * np.pi * (x - 0.5 * t) / 16 + 2 * np.pi * c / 3)
                      + 40 * np.sin(2 * np.pi * y / 32 + c))
    vid = _u8(bg)
    texA = rng.integers(0, 256, (6, 6, 3)).astype(np.uint8)
    texB = rng.integers(0, 256, (6, 6, 3)).astype(np.uint8)
    for tt in range(T):
        ax, ay = 6 + tt, 8
        vid[tt, ay:ay + 6, ax:ax + 6] = texA
        bx, by = 20 - tt, 18
        vid[tt, by:by + 6, bx:bx + 6] = texB
    mask = np.zeros((T, H, W), np.uint8)
    mask[2:6, 12:20, 12:20] = 1
    return Clip("tiny", vid, mask, 1, seed)


# ----------------------------------------------------------------------------
# general procedural generator
# ----------------------------------------------------------------------------

def _background(rng, W, H, T, v_b, sigma, n_grat=6):
    f = rng.uniform(1 / 96, 1 / 12, n_grat)
    th = rng.uniform(0, np.pi, n_grat)
    ph = rng.uniform(0, 2 * np.pi, n_grat)
    A = rng.uniform(10, 25, n_grat)
    g = rng.uniform(0.5, 1.0, (n_grat, 3))
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")

    def gratings(t):
        acc = np.full((H, W, 3), 128.0)
        for i in range(n_grat):
            s = np.sin(2 * np.pi * f[i] * (np.cos(th[i]) * (x + v_b * t) + np.sin(th[i]) * y)
                       + ph[i])
            acc += A[i] * s[..., None] * g[i][None, None, :]
        return acc

    # the gratings of later frames are computed on worker threads (numpy
    # releases the GIL) while the noise is drawn here, frame by frame in
    # order, so the result does not depend on the thread count
    frames = np.empty((T, H, W, 3), np.uint8)
    workers = max(1, min(16, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        pending = collections.deque()
        nxt = 0
        for t in range(T):
            while nxt < T and len(pending) < 2 * workers:
                pending.append(ex.submit(gratings, nxt))
                nxt += 1
            acc = pending.popleft().result()
            if sigma > 0:
                acc += rng.normal(0.0, sigma, (H, W, 3))
            frames[t] = _u8(acc)
    return frames


def _objects(rng, vid, n_obj, ax_lo, ax_hi, sp_lo, sp_hi):
    T, H, W, _ = vid.shape
    for _ in range(n_obj):
        a = int(rng.integers(ax_lo, ax_hi + 1))
        b = int(rng.integers(ax_lo, ax_hi + 1))
        sp = rng.uniform(sp_lo, sp_hi)
        ang = rng.uniform(0, 2 * np.pi)
        vx, vy = sp * math.cos(ang), sp * math.sin(ang)
        cx0 = rng.uniform(0, W)
        cy0 = rng.uniform(0, H)
        tex = rng.integers(0, 256, (2 * b + 1, 2 * a + 1, 3)).astype(np.uint8)
        yy, xx = np.meshgrid(np.arange(-b, b + 1), np.arange(-a, a + 1), indexing="ij")
        inside = (xx / max(a, 1)) ** 2 + (yy / max(b, 1)) ** 2 <= 1.0
        for t in range(T):
            cx = int(math.floor(cx0 + vx * t + 0.5))
            cy = int(math.floor(cy0 + vy * t + 0.5))
            X = xx + cx
            Y = yy + cy
            ok = inside & (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
            vid[t, Y[ok], X[ok]] = tex[ok]


def _tube(rng, W, H, T, frac, kind, speed_lo=1.0, speed_hi=2.0):
    """Occlusion tube: a box or an ellipse of area ~frac*W*H per frame moving
    on a straight line that stays inside the frame."""
    area = frac * W * H
    aspect = rng.uniform(0.6, 1.6)
    if kind == "box":
        bw = max(2, int(round(math.sqrt(area * aspect))))
        bh = max(2, int(round(area / bw)))
        rx, ry = bw / 2, bh / 2
    else:
        ra = math.sqrt(area * aspect / math.pi)
        rb = area / (math.pi * ra)
        rx, ry = ra, rb
    sp = rng.uniform(speed_lo, speed_hi)
    ang = rng.uniform(0, 2 * np.pi)
    vx, vy = sp * math.cos(ang), sp * math.sin(ang)
    # keep the whole path inside the frame (with a 3 px margin) when possible
    m = 3
    lo_x = m + rx + max(0.0, -vx * (T - 1))
    hi_x = W - m - rx - max(0.0, vx * (T - 1))
    lo_y = m + ry + max(0.0, -vy * (T - 1))
    hi_y = H - m - ry - max(0.0, vy * (T - 1))
    cx0 = rng.uniform(lo_x, hi_x) if hi_x > lo_x else W / 2 - vx * (T - 1) / 2
    cy0 = rng.uniform(lo_y, hi_y) if hi_y > lo_y else H / 2 - vy * (T - 1) / 2
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")
    mask = np.zeros((T, H, W), np.uint8)
    for t in range(T):
        cx = cx0 + vx * t
        cy = cy0 + vy * t
        if kind == "box":
            m_t = (np.abs(x + 0.5 - cx) <= rx) & (np.abs(y + 0.5 - cy) <= ry)
        else:
            m_t = ((x + 0.5 - cx) / rx) ** 2 + ((y + 0.5 - cy) / ry) ** 2 <= 1.0
        mask[t] = m_t
    return mask


def sd(seed: int = 2, T: int = 100) -> Clip:
    """854x480 x 100 frames: 6-grating background panning 1.5 px/frame with
    N(0, 4^2) noise, 5 textured ellipses (semi-axes 20..60, 0.5..3 px/frame),
    occlusion = ellipse a=100, b=65 centred (327+2t, 240)."""
    rng = np.random.default_rng(seed)
    W, H = 854, 480
    vid = _background(rng, W, H, T, 1.5, 4.0)
    _objects(rng, vid, 5, 20, 60, 0.5, 3.0)
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")
    mask = np.zeros((T, H, W), np.uint8)
    for t in range(T):
        mask[t] = ((x - (327 + 2 * t)) / 100.0) ** 2 + ((y - 240) / 65.0) ** 2 <= 1.0
    return Clip("sd", vid, mask, 4, seed)


def hd(seed: int = 3, T: int = 60) -> Clip:
    """1920x1080 x 60 frames: same background, 12 ellipses (semi-axes
    30..120), a periodic dynamic-texture region x in [1380,1680),
    y in [620,900) cycling through 3 noise fields, occlusion = union of three
    144x96 rectangles moving 2 px/frame."""
    rng = np.random.default_rng(seed)
    W, H = 1920, 1080
    vid = _background(rng, W, H, T, 1.5, 4.0)
    _objects(rng, vid, 12, 30, 120, 0.5, 3.0)
    fields = rng.integers(0, 256, (3, 280, 300, 3)).astype(np.uint8)
    for t in range(T):
        vid[t, 620:900, 1380:1680] = fields[t % 3]
    mask = np.zeros((T, H, W), np.uint8)
    for t in range(T):
        for (x0, y0) in ((300 + 2 * t, 200), (900, 500 + 2 * t), (1500 - 2 * t, 700 + t)):
            mask[t, y0:y0 + 96, x0:x0 + 144] = 1
    return Clip("hd", vid, mask, 5, seed)


def batch_clip(seed: int) -> Clip:
    """One clip of the mixed-size batch: W in 160..640, H in 120..360,
    T in 16..96, 1..5 objects, an occlusion tube (box or ellipse, 1..8 % of
    the voxels) moving 1..2 px/frame, 2..4 pyramid levels."""
    rng = np.random.default_rng(seed)
    W = int(rng.integers(160, 641))
    H = int(rng.integers(120, 361))
    T = int(rng.integers(16, 97))
    n_obj = int(rng.integers(1, 6))
    frac = rng.uniform(0.01, 0.08)
    kind = "box" if rng.uniform() < 0.5 else "ellipse"
    L = int(rng.integers(2, 5))
    vid = _background(rng, W, H, T, rng.uniform(0.5, 2.0), 4.0)
    _objects(rng, vid, n_obj, 10, 40, 0.5, 3.0)
    mask = _tube(rng, W, H, T, frac, kind)
    return Clip(f"batch{seed}", vid, mask, L, seed)


def batch(n: int = 64, base_seed: int = 1000) -> list[Clip]:
    return [batch_clip(base_seed + i) for i in range(n)]


def small(seed: int, W: int, H: int, T: int, frac: float = 0.04, levels: int = 2,
          n_obj: int = 2, kind: str = "ellipse", noise: float = 4.0) -> Clip:
    """A small clip of chosen size from the same generator (test cases)."""
    rng = np.random.default_rng(seed)
    vid = _background(rng, W, H, T, 1.0, noise)
    _objects(rng, vid, n_obj, max(2, min(W, H) // 12), max(3, min(W, H) // 6), 0.5, 2.0)
    mask = _tube(rng, W, H, T, frac, kind)
    return Clip(f"small{seed}", vid, mask, levels, seed)


def jittered(seed: int = 4, W: int = 320, H: int = 240, T: int = 24, n_obj: int = 3,
             max_rot_deg: float = 0.6, max_scale: float = 0.012, max_shift: float = 3.0,
             sigma: float = 2.0, hole_frac: float = 0.04):
    """A scene filmed by a shaking camera: a static grating background and
    textured ellipses moving in world coordinates, seen through a random
    affine camera per frame (rotation, scale and translation about the frame
    centre).  Returns (clip, cams): cams [T][6] maps a frame's pixel (x, y)
    to world coordinates, w = (c0 x + c1 y + c2, c3 x + c4 y + c5).  The
    occlusion is a world-fixed ellipse seen through the same cameras.  Every
    pixel is rendered from the scene at its world position (no resampling
    of other frames)."""
    rng = np.random.default_rng(seed)
    n_grat = 6
    f = rng.uniform(1 / 64, 1 / 10, n_grat)
    th = rng.uniform(0, np.pi, n_grat)
    ph = rng.uniform(0, 2 * np.pi, n_grat)
    A = rng.uniform(10, 25, n_grat)
    g = rng.uniform(0.5, 1.0, (n_grat, 3))
    cx, cy = (W - 1) / 2.0, (H - 1) / 2.0
    cams = np.zeros((T, 6))
    for t in range(T):
        a = np.deg2rad(rng.uniform(-max_rot_deg, max_rot_deg))
        sc = 1.0 + rng.uniform(-max_scale, max_scale)
        tx, ty = rng.uniform(-max_shift, max_shift, 2)
        c, sn = sc * np.cos(a), sc * np.sin(a)
        # w = R (x - centre) + centre + shift
        cams[t] = (c, -sn, cx - c * cx + sn * cy + tx, sn, c, cy - sn * cx - c * cy + ty)
    objs = []
    for _ in range(n_obj):
        a_ = int(rng.integers(8, 24))
        b_ = int(rng.integers(8, 24))
        sp = rng.uniform(0.5, 2.0)
        ang = rng.uniform(0, 2 * np.pi)
        objs.append((a_, b_, sp * np.cos(ang), sp * np.sin(ang), rng.uniform(0, W),
                     rng.uniform(0, H), rng.integers(0, 256, (2 * b_ + 1, 2 * a_ + 1, 3))))
    ha = np.sqrt(hole_frac * W * H * 1.3 / np.pi)
    hb = hole_frac * W * H / (np.pi * ha)
    hx, hy = rng.uniform(0.35 * W, 0.65 * W), rng.uniform(0.35 * H, 0.65 * H)
    y, x = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                       indexing="ij")
    vid = np.empty((T, H, W, 3), np.uint8)
    mask = np.zeros((T, H, W), np.uint8)
    for t in range(T):
        c0, c1, c2, c3, c4, c5 = cams[t]
        wx = c0 * x + c1 * y + c2
        wy = c3 * x + c4 * y + c5
        acc = np.full((H, W, 3), 128.0)
        for i in range(n_grat):
            sgr = np.sin(2 * np.pi * f[i] * (np.cos(th[i]) * wx + np.sin(th[i]) * wy) + ph[i])
            acc += A[i] * sgr[..., None] * g[i][None, None, :]
        for (a_, b_, vx, vy, ox, oy, tex) in objs:
            dx = wx - (ox + vx * t)
            dy = wy - (oy + vy * t)
            inside = (dx / a_) ** 2 + (dy / b_) ** 2 <= 1.0
            ix = np.clip(np.floor(dx + 0.5).astype(np.int64) + a_, 0, 2 * a_)
            iy = np.clip(np.floor(dy + 0.5).astype(np.int64) + b_, 0, 2 * b_)
            acc[inside] = tex[iy[inside], ix[inside]]
        if sigma > 0:
            acc += rng.normal(0.0, sigma, (H, W, 3))
        vid[t] = _u8(acc)
        mask[t] = ((wx - hx) / ha) ** 2 + ((wy - hy) / hb) ** 2 <= 1.0
    return Clip(f"jitter{seed}", vid, mask, 2, seed), cams


def image(seed: int, W: int, H: int, frac: float = 0.04, levels: int = 2, n_obj: int = 3,
          kind: str = "ellipse", noise: float = 4.0) -> Clip:
    """One still image (T = 1) from the same generator: grating background,
    textured ellipses and a box or ellipse hole of about frac of the
    pixels (2-D image inpainting with 5x5x1 patches)."""
    return small(seed, W, H, 1, frac=frac, levels=levels, n_obj=n_obj, kind=kind, noise=noise)


def noise(seed: int, shape, sigma2: float = 25.0, mean: int = 128) -> np.ndarray:
    """Grey white noise for the textured-patch experiment of App. B: i.i.d.
    centred normal values of variance sigma2 (25 grey levels squared in the
    paper's table) around ``mean``, rounded half up to integers and clipped
    to 0..255 (at sigma = 5 the clip is never reached).  ``shape`` is
    [T][H][W] for a volume or [n][pt][ph][pw] for a list of patches."""
    rng = np.random.default_rng(seed)
    return _u8(mean + math.sqrt(sigma2) * rng.standard_normal(tuple(shape)))


def served_trace(duration_s: float = 120.0, rate: float = 4.0, seed: int = 2000,
                 sd_frac: float = 0.10):
    """Poisson arrivals: list of (arrival_time_s, kind, seed) where kind is
    'batch' (a batch_clip draw) or 'sd' (an 854x480x100 clip)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    j = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration_s:
            break
        kind = "sd" if rng.uniform() < sd_frac else "batch"
        out.append((t, kind, seed + j))
        j += 1
    return out


CONFIGS = {
    "tiny": dict(W=32, H=32, T=8, levels=1),
    "sd": dict(W=854, H=480, T=100, levels=4),
    "hd": dict(W=1920, H=1080, T=60, levels=5),
}
