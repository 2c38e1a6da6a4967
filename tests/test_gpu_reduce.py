"""The dimensionality-reduced patch space (Sec. 5) on the GPU against the
CPU oracle.

* The exact integer moments of the sampled source patches equal the
  oracle's (video and image patches, all sources and every k-th).
* Given the same basis, the features of every voxel equal the oracle's bit
  for bit (integer arithmetic on both sides), for a PCA basis and for a
  wide random one, and so does the shift map of a search with the reduced
  distance followed by the exact re-evaluation (candidates, distances,
  counts), and a whole MEAN-mode inpainting with a basis on every level.
* The GPU's own basis (orthogonal iteration) captures the variance of the
  oracle's (numpy's symmetric eigensolver) to 1e-3 relative; its rows are
  orthogonal after undoing the weights and the scale.
* A clip created with reduce_dims inpaints end to end; argument errors.
"""
import numpy as np
import pytest
import torch

from oracle import pca, vio
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


def pair(vi, clip, **kw):
    v, m = clip.occluded_input(), clip.mask
    return vi.Clip(dev(v), dev(m), **kw), vio.Oracle(v, m, **kw)


CLIP = dict(seed=61, W=52, H=44, T=12, frac=0.05, levels=2)


@pytest.mark.parametrize("n_max", [65536, 97])
def test_moments_bitexact(vi, n_max):
    print(f"[case] pca moments n_max={n_max}", flush=True)
    g, o = pair(vi, synth.small(**CLIP), levels=2)
    for level in range(2):
        a = g.pca_moments(level, n_max)
        b = o.pca_moments(level, n_max)
        assert a[2] == b[2]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    g.close()
    img = synth.image(62, 70, 50, levels=2)
    g, o = pair(vi, img, levels=2, patch=(5, 5, 1))
    a, b = g.pca_moments(0, n_max), o.pca_moments(0, n_max)
    assert a[1].shape == (125, 125) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    g.close()


def test_features_and_search_bitexact(vi):
    print("[case] reduced features and search", flush=True)
    g, o = pair(vi, synth.small(**CLIP), levels=2, seed=5)
    rng = np.random.default_rng(3)
    wide = rng.integers(-3000, 3000, (8, 625)).astype(np.int16)
    for level, Q in ((1, o.pca_basis(1, 16)), (0, o.pca_basis(0, 12)), (1, wide)):
        d = Q.shape[0]
        g.set_reduction(level, Q)
        o.set_reduction(level, Q)
        assert np.array_equal(host(g.features(level, d)), o.features(level, d)), level
        for it in range(2):
            g.nnf_search(level, it)
            o.nnf_search(level, it)
            gs, os_ = [host(t) for t in g.get_state(level)], o.get_state(level)
            for a, b in zip(gs[1:], os_[1:]):
                assert np.array_equal(a, b), (level, it)
            g.reconstruct(level, vi.MEAN)
            o.reconstruct(level, vio.MEAN)
    g.close()


@pytest.mark.parametrize("patch", [(5, 5, 5), (5, 5, 1)])
def test_inpaint_mean_with_forced_bases_bitexact(vi, patch):
    print(f"[case] reduced MEAN inpainting patch={patch}", flush=True)
    if patch[2] == 1:
        clip = synth.image(63, 96, 72, levels=2)
    else:
        clip = synth.small(64, 60, 48, 10, frac=0.04, levels=2)
    kw = dict(levels=2, seed=9, recon_mode=1, patch=patch)
    g, o = pair(vi, clip, **kw)
    for level in range(2):
        Q = o.pca_basis(level, 8)
        g.set_reduction(level, Q)
        o.set_reduction(level, Q)
    out = host(g.inpaint())
    ref = o.inpaint()
    g.close()
    assert np.array_equal(out, ref)
    assert np.array_equal(out[clip.mask == 0], clip.video[clip.mask == 0])


def test_gpu_basis_captures_the_variance(vi):
    print("[case] GPU PCA basis", flush=True)
    g, o = pair(vi, synth.small(**CLIP), levels=2)
    for level, d in ((0, 16), (1, 8), (0, 32)):
        Q, var = g.pca_basis(level, d)
        S1, S2, n = o.pca_moments(level)
        C = pca.covariance(S1, S2, n, 50)
        vals, _ = pca.basis(C, d)
        print(f"    level {level} d {d}: captured {var.sum():.6g} of {vals.sum():.6g}")
        assert var.sum() >= (1 - 1e-3) * vals.sum()
        assert var.sum() <= (1 + 1e-9) * vals.sum()
        # the basis itself: rows orthonormal once the weights and scale are undone
        B = Q.astype(np.float64) / 256.0 / pca.weights(625, 50)[None, :]
        G = B @ B.T
        assert np.abs(G - np.eye(d)).max() < 0.02
        # and they capture what the Rayleigh quotients say (to quantisation)
        cap = np.einsum("ki,ij,kj->k", B, C, B)
        assert np.allclose(cap.sum(), var.sum(), rtol=0.02)
    g.close()


def test_reduce_dims_end_to_end(vi):
    print("[case] reduce_dims end to end", flush=True)
    clip = synth.small(65, 96, 80, 16, frac=0.04, levels=2)
    v, m = dev(clip.occluded_input()), dev(clip.mask)
    outs = {}
    for rd in (0, 16):
        g = vi.Clip(v, m, levels=2, seed=3, reduce_dims=rd)
        outs[rd] = host(g.inpaint())
        g.close()
    hole = clip.mask == 1
    err = {k: np.abs(o[hole].astype(float) - clip.video[hole].astype(float)).mean()
           for k, o in outs.items()}
    print(f"    mean |error| in the hole: exact {err[0]:.2f}, reduced {err[16]:.2f}")
    assert np.array_equal(outs[16][~hole], clip.video[~hole])
    assert err[16] < 1.5 * err[0] + 2.0


def test_reduction_errors(vi):
    clip = synth.small(**CLIP)
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=2)
    with pytest.raises(vi.ViError) as e:
        g.features(0, 4)
    assert e.value.status == -4
    with pytest.raises(vi.ViError):
        g.set_reduction(0, np.zeros((33, 625), np.int16))
    with pytest.raises(vi.ViError):
        g.set_reduction(0, np.full((2, 625), 32767, np.int16))  # sums overflow 32 bits
    with pytest.raises(vi.ViError):
        g.pca_basis(0, 0)
    g.set_reduction(0, np.zeros((4, 625), np.int16))
    g.set_reduction(0, None)
    with pytest.raises(vi.ViError):
        g.features(0, 4)
    g.set_reduction(1, np.eye(4, 625, dtype=np.int16))
    with pytest.raises(vi.ViError):
        g.features(1, 3)  # not the level's feature count
    b = vi.Batch()
    with pytest.raises(vi.ViError):
        b.add(g)
    b.close()
    g.close()
