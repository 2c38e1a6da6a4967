"""Pins of the oracle's ANN search (Sec. 3.1, Alg. 1, Eq. (3.1)) against the
exact nearest neighbours found by brute force, and the invariants an ANN
search must keep: every match is a source of D~ (Sec. 2), the stored distance
is the distance of the stored match, no target gets worse, and a set with a
single source forces that source.  Results are independent of the thread
count because every pass reads the state from before the pass."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import vio
from paper_1503_05528_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def brute_force_nn(rgbt, dsrc, targets, lam, h=2):
    """Exact minimum over all sources of the integer SSD (voxels of the
    target patch outside the volume are not compared), by dense linear
    algebra in float64 (exact: every term is an integer below 2^53)."""
    T, H, W, _ = rgbt.shape
    w = np.array([1, 1, 1, lam, lam], np.float64)
    P = 2 * h + 1
    pad = np.zeros((T + 2 * h, H + 2 * h, W + 2 * h, 5), np.float64)
    pad[h:-h, h:-h, h:-h] = rgbt
    val = np.zeros((T + 2 * h, H + 2 * h, W + 2 * h), np.float64)
    val[h:-h, h:-h, h:-h] = 1

    def patches(arr, idx):
        x, y, t = idx % W, (idx // W) % H, idx // (W * H)
        out = []
        for i in range(len(idx)):
            out.append(arr[t[i]:t[i] + P, y[i]:y[i] + P, x[i]:x[i] + P].reshape(P ** 3, -1))
        return np.stack(out)

    src = np.flatnonzero(dsrc.ravel())
    A = patches(pad, targets)  # [nt, 125, 5]
    M = patches(val[..., None], targets)[..., 0]  # [nt, 125]
    B = patches(pad, src).reshape(len(src), -1)  # [ns, 625]
    Mw = (M[:, :, None] * w).reshape(len(targets), -1)
    Aw = (A * M[:, :, None] * w).reshape(len(targets), -1)
    D = (Aw * A.reshape(len(targets), -1)).sum(1)[:, None] + Mw @ (B ** 2).T - 2 * Aw @ B.T
    j = np.argmin(D, axis=1)
    return np.rint(D.min(1)).astype(np.int64), src[j]


@pytest.fixture(scope="module")
def tiny_state(oracle_lib):
    c = synth.tiny()
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1, seed=1)
    o.onion_init()
    return c, o


def test_search_vs_brute_force_tiny(tiny_state):
    c, o = tiny_state
    o.nnf_search(0, 0)
    rgbt, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    tg = np.flatnonzero(htil.ravel())
    ex, _ = brute_force_nn(rgbt.astype(np.float64), dsrc, tg, 50)
    pm = dist.ravel()[tg].astype(np.int64)
    # an ANN is never better than the exact NN
    assert (pm >= ex).all()
    # and PatchMatch reaches the exact NN distance for most targets
    assert (pm == ex).mean() > 0.5
    assert pm.sum() <= 1.15 * ex.sum()
    # E(u, exact NN) <= E(u, phi)
    assert ex.sum() <= o.energy(0)


def test_search_invariants_tiny(tiny_state):
    c, o = tiny_state
    o.nnf_search(0, 3)
    rgbt, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    T, H, W = hole.shape
    tg = np.flatnonzero(htil.ravel())
    cf = cand.ravel()
    # matches are sources; non-targets are unset
    assert (dsrc.ravel()[cf[tg]] == 1).all()
    assert (cf[htil.ravel() == 0] == -1).all()
    assert (dist.ravel()[htil.ravel() == 0] == -1).all()
    # stored distance and count are those of the stored match
    rng = np.random.default_rng(0)
    for p in rng.choice(tg, 60, replace=False):
        d, n = o.patch_ssd(0, p, cf[p])
        assert d == dist.ravel()[p] and n == nvox.ravel()[p]
    # count = in-volume part of the 5x5x5 patch
    for p in rng.choice(tg, 60, replace=False):
        x, y, t = p % W, (p // W) % H, p // (W * H)
        nx = min(x + 2, W - 1) - max(x - 2, 0) + 1
        ny = min(y + 2, H - 1) - max(y - 2, 0) + 1
        nt = min(t + 2, T - 1) - max(t - 2, 0) + 1
        assert nvox.ravel()[p] == nx * ny * nt


def test_search_never_worsens_a_target(tiny_state):
    c, o = tiny_state
    o.nnf_search(0, 4)
    d0 = o.get_state(0)[2].copy()
    for it in (5, 6):
        o.nnf_search(0, it)  # same u: re-evaluation gives the same distances
        d1 = o.get_state(0)[2]
        assert (d1 <= d0).all()
        d0 = d1.copy()


def test_single_source_forces_the_match(oracle_lib):
    # a 5-frame clip whose only hole-free 5x5x5 window is centred at (2,2,2)
    W, H, T = 12, 5, 5
    rng = np.random.default_rng(3)
    v = rng.integers(0, 256, (T, H, W, 3)).astype(np.uint8)
    m = np.zeros((T, H, W), np.uint8)
    m[:, :, 5:] = 1
    o = vio.Oracle(v, m, levels=1)
    (_, _, _), (nH, nHt, nD) = o.info(0)
    assert nD == 1
    o.nnf_search(0, 0)
    _, cand, _, _ = o.get_state(0)
    htil = o.sets(0)[2]
    src = (2 * H + 2) * W + 2
    assert (cand[htil == 1] == src).all()


def test_unset_and_invalid_matches_are_reinitialised(tiny_state):
    c, o = tiny_state
    rgbt, cand, dist, nvox = o.get_state(0)
    hole, dsrc, htil = o.sets(0)
    bad = cand.copy()
    tg = np.flatnonzero(htil.ravel())
    bad.ravel()[tg[::3]] = -1
    nonsrc = np.flatnonzero((dsrc.ravel() == 0))
    bad.ravel()[tg[1::3]] = nonsrc[0]
    o.set_state(0, cand=bad)
    o.nnf_search(0, 7)
    cand2 = o.get_state(0)[1]
    assert (dsrc.ravel()[cand2.ravel()[tg]] == 1).all()


def test_random_search_radius_limits(oracle_lib):
    # with pm_iters = 0 only the initialisation runs; with no propagation
    # steps and rho = 0.5 the window radius at iteration k is r_max >> k.
    c = synth.tiny()
    o = vio.Oracle(c.occluded_input(), c.mask, levels=1, pm_iters=0, seed=9)
    o.nnf_search(0, 0)
    cand0 = o.get_state(0)[1]
    o2 = vio.Oracle(c.occluded_input(), c.mask, levels=1, pm_iters=6, jf_steps=[], seed=9)
    o2.set_state(0, cand=cand0)
    o2.nnf_search(0, 0)
    cand1 = o2.get_state(0)[1]
    htil = o.sets(0)[2]
    W, H, T = 32, 32, 8
    tg = np.flatnonzero(htil.ravel())
    a, b = cand0.ravel()[tg], cand1.ravel()[tg]
    dx = np.abs(a % W - b % W)
    dy = np.abs((a // W) % H - (b // W) % H)
    dt = np.abs(a // (W * H) - b // (W * H))
    # a chain of accepted moves: sum of radii 16 + 8 + 4 + 2 + 1 (+0) = 31
    assert dx.max() <= 31 and dy.max() <= 31 and dt.max() <= 31
    assert (a != b).any()


def _run_threads(n):
    code = (
        "import sys, hashlib; sys.path.insert(0, %r)\n"
        "from oracle import vio\n"
        "from paper_1503_05528_amd import synth\n"
        "c = synth.small(4, 48, 40, 12, levels=2)\n"
        "o = vio.Oracle(c.occluded_input(), c.mask, levels=2, seed=3)\n"
        "out = o.inpaint()\n"
        "print(vio.num_threads(), hashlib.sha256(out.tobytes()).hexdigest())\n" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS=str(n))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600, check=True)
    return r.stdout.split()


def test_thread_count_does_not_change_results(oracle_lib):
    a = _run_threads(1)
    b = _run_threads(4)
    assert a[0] == "1" and b[0] == "4"
    assert a[1] == b[1]
