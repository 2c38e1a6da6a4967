"""Pins of the oracle's dimensionality-reduced patch distance (the
acceleration Sec. 5 proposes; PCA of the level's source patches is this
implementation's reading) against what is known independently of it:

* the exact integer moments of the sampled source patches equal a numpy
  computation over patch vectors extracted by fancy indexing;
* the covariance formed from them equals numpy's covariance of the
  weighted vectors, and the basis's eigenvalues equal the squared singular
  values of the centred data matrix (numpy's SVD) over n;
* the features equal a direct pure-Python evaluation of their definition
  (clamped patch vectors, floor of (Q x + 128) / 256);
* with the identity as basis (every coordinate, lambda = 4 so that the
  texture weight 2 is an integer) the features are the weighted patch
  vectors, the reduced distance is the patch distance, and the reduced
  search reproduces the exact search's shift map bit for bit;
* with a 16-dimensional PCA basis the matches the reduced search finds are
  good ones: their exact energy stays within 25 % of the exact search's;
* the exact distance is restored after every reduced search.
"""
import math

import numpy as np
import pytest

from oracle import pca, vio
from paper_1503_05528_amd import synth


def interior_clip(seed=5, W=28, H=24, T=11):
    c = synth.small(seed, W, H, T, levels=1)
    m = np.zeros((T, H, W), np.uint8)
    m[4:T - 4, 8:14, 9:17] = 1  # H~ (the hole grown by 2) stays 2 from every border
    return c.video, m


def patch_vectors(rgbt, centres, h=(2, 2, 2)):
    T, H, W, _ = rgbt.shape
    t, y, x = np.unravel_index(centres, (T, H, W))
    out = []
    for dt in range(-h[2], h[2] + 1):
        for dy in range(-h[1], h[1] + 1):
            for dx in range(-h[0], h[0] + 1):
                out.append(rgbt[t + dt, y + dy, x + dx, :])
    return np.stack(out, 1).reshape(len(centres), -1).astype(np.int64)


def test_moments_match_numpy(oracle_lib):
    v, m = interior_clip()
    o = vio.Oracle(v, m, levels=1)
    rgbt, *_ = o.get_state(0)
    _, dsrc, _ = o.sets(0)
    src = np.flatnonzero(dsrc.ravel())
    for n_max in (10 ** 6, 97):
        S1, S2, n = o.pca_moments(0, n_max)
        k = -(-len(src) // n_max)
        X = patch_vectors(rgbt, src[::k])
        assert n == len(X)
        assert np.array_equal(S1, X.sum(0).astype(np.uint64))
        assert np.array_equal(S2, (X.T @ X).astype(np.uint64))


def test_covariance_and_basis(oracle_lib):
    v, m = interior_clip(seed=6)
    o = vio.Oracle(v, m, levels=1)
    rgbt, *_ = o.get_state(0)
    _, dsrc, _ = o.sets(0)
    S1, S2, n = o.pca_moments(0)
    X = patch_vectors(rgbt, np.flatnonzero(dsrc.ravel())).astype(np.float64)
    Y = X * pca.weights(X.shape[1], 50)
    C = pca.covariance(S1, S2, n, 50)
    ref = np.cov(Y.T, bias=True)
    assert np.allclose(C, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())
    vals, B = pca.basis(C, 16)
    sv = np.linalg.svd(Y - Y.mean(0), compute_uv=False)
    assert np.allclose(vals, sv[:16] ** 2 / n, rtol=1e-8)
    assert np.allclose(B.T @ B, np.eye(16), atol=1e-10)
    Q = pca.quantize(B, 50)
    assert Q.shape == (16, 625) and Q.dtype == np.int16


def test_features_match_definition(oracle_lib):
    v, m = interior_clip(seed=7, W=12, H=10, T=7)
    o = vio.Oracle(v, m, levels=1)
    rgbt, *_ = o.get_state(0)
    rng = np.random.default_rng(1)
    Q = rng.integers(-2000, 2000, (3, 625)).astype(np.int16)
    o.set_reduction(0, Q)
    f = o.features(0, 3)
    T, H, W, _ = rgbt.shape
    for (t, y, x) in [(0, 0, 0), (3, 4, 5), (6, 9, 11), (2, 0, 7), (5, 8, 1)]:
        xs = []
        for dt in range(-2, 3):
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    tt, yy, xx = (min(max(t + dt, 0), T - 1), min(max(y + dy, 0), H - 1),
                                  min(max(x + dx, 0), W - 1))
                    xs += [int(c) for c in rgbt[tt, yy, xx]]
        for k in range(3):
            acc = sum(int(q) * xv for q, xv in zip(Q[k], xs))
            assert f[t, y, x, k] == (acc + 128) // 256, (t, y, x, k)


def test_identity_basis_reproduces_the_exact_search(oracle_lib):
    v, m = interior_clip(seed=8)
    kw = dict(levels=1, seed=4, lam=4)
    a = vio.Oracle(v, m, **kw)
    b = vio.Oracle(v, m, **kw)
    w = pca.weights(625, 4)
    Q = np.diag(256 * w).astype(np.int16)  # weights 1 and 2: exact
    b.set_reduction(0, Q)
    rgbt, *_ = b.get_state(0)
    f = b.features(0, 625)
    hole, _, htil = b.sets(0)
    p = np.flatnonzero(htil.ravel())
    # the features of interior voxels are the weighted patch vectors
    assert np.array_equal(f.reshape(-1, 625)[p], patch_vectors(rgbt, p) * w.astype(np.int64))
    for it in range(2):
        a.nnf_search(0, it)
        b.nnf_search(0, it)
        _, ca, da, na = a.get_state(0)
        _, cb, db, nb = b.get_state(0)
        assert np.array_equal(ca, cb) and np.array_equal(da, db) and np.array_equal(na, nb)
        a.reconstruct(0, vio.MEAN)
        b.reconstruct(0, vio.MEAN)


def test_pca_search_quality_and_exact_distances(oracle_lib):
    c = synth.small(9, 48, 40, 12, levels=1, frac=0.05)
    v, m = c.occluded_input(), c.mask
    a = vio.Oracle(v, m, levels=1, seed=2)
    b = vio.Oracle(v, m, levels=1, seed=2, reduce_dims=16)
    for o in (a, b):
        o.nnf_search(0, 0)
    _, _, htil = b.sets(0)
    _, cb, db, nb = b.get_state(0)
    sel = htil.astype(bool)
    # distances are exact after the search
    for p in np.flatnonzero(sel.ravel())[::37]:
        assert db.ravel()[p] == b.patch_ssd(0, p, cb.ravel()[p])[0]
    ea, eb = a.energy(0), b.energy(0)
    print("exact-search energy", ea, "reduced-search energy", eb, eb / ea)
    assert eb <= 1.25 * ea
