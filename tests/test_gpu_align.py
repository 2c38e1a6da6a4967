"""Realignment on the GPU (vi_align_*) against the CPU oracle (Sec. 3.4,
Alg. 2, and the inverse warp of Alg. 4).

* The estimated motions agree with the oracle's within 1e-3 px at the frame
  corners (both sum the same normal equations in double precision, in
  different orders) and with the shaking camera's true motion within
  0.1 px.
* Given the same maps, the warp (video and occlusion) and the unwarp are bit
  for bit the oracle's: both evaluate every product and sum in double
  precision, rounded one by one, in the same order.
* Inpainting in the aligned domain with the same maps gives, in MEAN mode,
  the oracle's output bit for bit, and every known pixel is the input's.
"""
import numpy as np
import pytest
import torch

from oracle import vio
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


def H3(m):
    return np.array([[m[0], m[1], m[2]], [m[3], m[4], m[5]], [0.0, 0.0, 1.0]])


def corner_error(a, b, W, H):
    c = np.array([[0, 0, 1], [W - 1, 0, 1], [0, H - 1, 1], [W - 1, H - 1, 1.0]]).T
    return np.abs((H3(a) @ c - H3(b) @ c)[:2]).max()


@pytest.mark.parametrize("seed,W,H,T", [(4, 240, 180, 10), (7, 197, 133, 9)])
def test_estimate_matches_oracle_and_truth(vi, seed, W, H, T):
    print(f"[case] align estimate seed={seed} {W}x{H}x{T}", flush=True)
    clip, cams = synth.jittered(seed=seed, W=W, H=H, T=T)
    v, m = clip.occluded_input(), clip.mask
    ot = vio.align_estimate(v, m)
    gt = vi.align_estimate(dev(v), dev(m))
    for n in range(T - 1):
        assert corner_error(ot[n], gt[n], W, H) < 1e-3, n
        true = (np.linalg.inv(H3(cams[n + 1])) @ H3(cams[n]))[:2].ravel()
        assert corner_error(true, gt[n], W, H) < 0.1, n
    assert np.allclose(vi.align_compose(gt, T), vio.align_compose(gt, T), rtol=0, atol=0)


@pytest.mark.parametrize("seed", [4, 8])
def test_warp_and_unwarp_bitexact(vi, seed):
    print(f"[case] align warp/unwarp seed={seed}", flush=True)
    clip, cams = synth.jittered(seed=seed, W=203, H=151, T=9)
    v, m = clip.occluded_input(), clip.mask
    M = vio.align_compose(vio.align_estimate(v, m), 9)
    # larger maps too: a shift that pushes pixels out of the frame
    M2 = M.copy()
    M2[:, 2] += np.linspace(-30.5, 30.25, 9)
    for MM in (M, M2):
        ov, om = vio.align_warp(v, m, MM)
        gv, gm = vi.align_warp(dev(v), dev(m), MM)
        assert np.array_equal(om, host(gm))
        assert np.array_equal(ov, host(gv))
        # unwarp an "inpainted" aligned video: the true video warped
        full, _ = vio.align_warp(clip.video, np.zeros_like(m), MM)
        ou = vio.align_unwarp(full, v, m, MM)
        gu = vi.align_unwarp(dev(full), dev(v), dev(m), MM)
        assert np.array_equal(ou, host(gu))


def test_inpaint_in_the_aligned_domain_matches_oracle(vi):
    print("[case] realigned MEAN inpainting vs oracle", flush=True)
    clip, cams = synth.jittered(seed=9, W=96, H=80, T=10, hole_frac=0.03)
    v, m = clip.occluded_input(), clip.mask
    T = v.shape[0]
    M = vio.align_compose(vio.align_estimate(v, m), T)
    kw = dict(levels=2, seed=3, recon_mode=1)
    av, am = vio.align_warp(v, m, M)
    ref = vio.align_unwarp(vio.Oracle(av, am, **kw).inpaint(), v, m, M)
    gav, gam = vi.align_warp(dev(v), dev(m), M)
    g = vi.Clip(gav, gam, **kw)
    out = host(vi.align_unwarp(g.inpaint(), dev(v), dev(m), M))
    g.close()
    assert np.array_equal(out, ref)
    assert np.array_equal(out[m == 0], v[m == 0])


def test_inpaint_realigned_pipeline(vi):
    print("[case] realigned pipeline", flush=True)
    clip, _ = synth.jittered(seed=10, W=128, H=96, T=10, hole_frac=0.03)
    v, m = clip.occluded_input(), clip.mask
    out, theta, M = vi.inpaint_realigned(dev(v), dev(m), levels=2, seed=1)
    out = host(out)
    assert theta.shape == (9, 6) and M.shape == (10, 6)
    assert np.array_equal(out[m == 0], v[m == 0])
    # the hole is filled with plausible content (close to the true scene)
    err = np.abs(out[m == 1].astype(float) - clip.video[m == 1].astype(float)).mean()
    print(f"mean |error| in the hole: {err:.1f} grey levels", flush=True)
    assert err < 40


def test_align_errors(vi):
    clip, _ = synth.jittered(seed=4, W=64, H=48, T=4)
    v, m = dev(clip.occluded_input()), dev(clip.mask)
    with pytest.raises(vi.ViError) as e:
        vi.align_estimate(v[:1], m[:1])
    assert e.value.status == -1
    with pytest.raises(vi.ViError):
        vi.align_estimate(v, m, levels=5)  # 64 x 48 -> coarsest below 8 x 8
    with pytest.raises(vi.ViError):
        vi.align_warp(v, m, np.zeros((4, 6)))  # singular maps
