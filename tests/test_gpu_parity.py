"""GPU (libvi, HIP on gfx950) against the CPU oracle, element by element.

Integer work (pyramids, texture features, sets, shift maps, distances,
counts, MEAN and BEST reconstructions) must match bit for bit.  The weighted
reconstruction is float32 on both sides; the two differ only in the
exponential and the order of the float sums, so out_f must agree within 1e-4
on [0, 1] and the uint8 requantisation may differ by one only where the
oracle's value lies within that tolerance of a rounding boundary.

Searches and reconstructions are teacher-forced: both sides start from the
same state, set through vi_set_state / vio_set_state.
"""
import numpy as np
import pytest
import torch

from oracle import vio
from paper_1503_05528_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-4


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


def make_pair(vi, clip, wide=-1, **kw):
    """wide: the library's wide_pass_max (which form its passes take; the
    results do not depend on it): -1 its own choice, which takes the wide
    form on these small levels, 0 the one-lane form everywhere."""
    print(f"[case] {clip.name} {clip.shape} levels={kw.get('levels')} wide={wide}", flush=True)
    o = vio.Oracle(clip.occluded_input(), clip.mask, **kw)
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), wide_pass_max=wide, **kw)
    return o, g


# both forms of the search pass (one lane with early exit, or eight lanes per
# candidate)
WIDE = [pytest.param(0, id="onelane"), pytest.param(-1, id="wide")]


CLIPS = {
    "tiny": lambda: (synth.tiny(), 1),
    "small2": lambda: (synth.small(21, 61, 47, 11, levels=2, frac=0.05), 2),
    "small3": lambda: (synth.small(22, 83, 66, 9, levels=3, frac=0.04, kind="box"), 3),
    "edge": lambda: (_edge_clip(), 2),
}


def _edge_clip():
    # hole touching the volume border in x, y and t
    c = synth.small(23, 40, 34, 8, levels=2, frac=0.03)
    c.mask[:] = 0
    c.mask[0:3, 0:6, 0:7] = 1
    c.mask[5:8, 28:34, 30:40] = 1
    return c


def assert_recon_close(o_out, g_out, o_rgbt, g_rgbt, hole_idx):
    assert o_out.shape == g_out.shape
    err = np.abs(o_out.astype(np.float64) - g_out.astype(np.float64)).max() if len(o_out) else 0
    assert err <= TOL, f"max |out_f difference| = {err}"
    a = o_rgbt.reshape(-1, 5)[hole_idx].astype(int)
    b = g_rgbt.reshape(-1, 5)[hole_idx].astype(int)
    diff = np.abs(a - b)
    assert diff.max(initial=0) <= 1
    if diff.any():
        # only where the oracle's value is within the tolerance of a .5 boundary
        v = o_out * 255.0
        frac = np.abs(v - np.floor(v) - 0.5)
        assert (frac[diff > 0] <= TOL * 255.0 + 1e-3).all()


@pytest.mark.parametrize("name", list(CLIPS))
def test_create_matches_oracle(vi, name):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, levels=L)
    for lv in range(L):
        assert o.info(lv) == g.info(lv)
        for a, b in zip(o.sets(lv), g.sets(lv)):
            assert np.array_equal(a, host(b))
        og = o.get_state(lv)
        gg = g.get_state(lv)
        for a, b in zip(og, gg):
            assert np.array_equal(a, host(b)), lv


def _forced_state(o, lv, seed):
    """A state to teacher-force from: the oracle's video with random (valid
    or unset) matches on the targets."""
    rgbt, cand, dist, nvox = o.get_state(lv)
    hole, dsrc, htil = o.sets(lv)
    rng = np.random.default_rng(seed)
    src = np.flatnonzero(dsrc.ravel())
    tg = np.flatnonzero(htil.ravel())
    cand = np.full(cand.shape, -1, np.int32)
    pick = rng.integers(0, len(src), len(tg))
    cand.ravel()[tg] = src[pick]
    cand.ravel()[tg[::7]] = -1  # some unset
    # a random fill of the hole so that reconstructions are not trivial
    rgbt = rgbt.copy()
    hv = hole.ravel() == 1
    rgbt.reshape(-1, 5)[hv] = rng.integers(0, 256, (int(hv.sum()), 5))
    return rgbt, cand


@pytest.mark.parametrize("name", list(CLIPS))
@pytest.mark.parametrize("em_iter", [0, 3])
@pytest.mark.parametrize("wide", WIDE)
def test_search_bitexact(vi, name, em_iter, wide):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, wide=wide, levels=L, seed=7)
    for lv in range(L):
        rgbt, cand = _forced_state(o, lv, 100 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        g.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, em_iter)
        g.nnf_search(lv, em_iter)
        _, oc, od, on = o.get_state(lv)
        _, gc, gd, gn = g.get_state(lv)
        assert np.array_equal(oc, host(gc)), f"cand level {lv}"
        assert np.array_equal(od, host(gd)), f"dist level {lv}"
        assert np.array_equal(on, host(gn)), f"nvox level {lv}"


@pytest.mark.parametrize("wide", WIDE)
def test_search_variants_bitexact(vi, wide):
    # other iteration counts, steps and lambda (odd pass count: state copied back)
    clip, L = CLIPS["small2"]()
    for kw in (dict(pm_iters=3, jf_steps=[1]), dict(pm_iters=4, jf_steps=[]),
               dict(pm_iters=2, jf_steps=[3, 1], lam=0), dict(pm_iters=5, rho=0.7, lam=130)):
        o, g = make_pair(vi, clip, wide=wide, levels=L, seed=3, **kw)
        rgbt, cand = _forced_state(o, 0, 5)
        o.set_state(0, rgbt=rgbt, cand=cand)
        g.set_state(0, rgbt=rgbt, cand=cand)
        o.nnf_search(0, 1)
        g.nnf_search(0, 1)
        _, oc, od, _ = o.get_state(0)
        _, gc, gd, _ = g.get_state(0)
        assert np.array_equal(oc, host(gc)), kw
        assert np.array_equal(od, host(gd)), kw


@pytest.mark.parametrize("name", list(CLIPS))
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_reconstruct_parity(vi, name, mode):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, levels=L, seed=9)
    for lv in range(L):
        rgbt, cand = _forced_state(o, lv, 200 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, 0)
        r, c, d, n = o.get_state(lv)
        g.set_state(lv, rgbt=r, cand=c, dist=d, nvox=n)
        oo, os_ = o.reconstruct(lv, mode)
        go, gs = g.reconstruct(lv, mode)
        o_r = o.get_state(lv)[0]
        g_r = host(g.get_state(lv)[0])
        hole_idx = np.flatnonzero(o.sets(lv)[0].ravel())
        if mode == 0:
            assert_recon_close(oo, host(go), o_r, g_r, hole_idx)
        else:
            assert np.array_equal(o_r, g_r)
            assert np.abs(oo - host(go)).max(initial=0) <= 1e-6
            assert os_ == int(host(gs)[0])


# "edge": masked distances whose rows start before the first voxel or end
# after the last one of the volume
@pytest.mark.parametrize("name", ["tiny", "small2", "small3", "edge"])
@pytest.mark.parametrize("wide", WIDE)
def test_onion_mean_bitexact(vi, name, wide):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, wide=wide, levels=L, seed=4, recon_mode=1)
    assert o.onion_init() == g.onion_init()
    for a, b in zip(o.get_state(L - 1), g.get_state(L - 1)):
        assert np.array_equal(a, host(b))


@pytest.mark.parametrize("name", ["tiny", "small2", "small3"])
def test_onion_weighted_close(vi, name):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, levels=L, seed=4)
    assert o.onion_init() == g.onion_init()
    a = o.get_state(L - 1)[0]
    b = host(g.get_state(L - 1)[0])
    hole = o.sets(L - 1)[0].astype(bool)
    d = np.abs(a[hole].astype(int) - b[hole].astype(int))
    # rounding flips can propagate through later layers; nearly all agree
    assert (d == 0).mean() > 0.97


def test_transition_bitexact(vi):
    clip, L = CLIPS["small3"]()
    o, g = make_pair(vi, clip, levels=L, seed=5, recon_mode=1)
    rgbt, cand = _forced_state(o, 2, 1)
    o.set_state(2, rgbt=rgbt, cand=cand)
    o.nnf_search(2, 0)
    for lv in (2,):
        r, c, d, n = o.get_state(lv)
        g.set_state(lv, rgbt=r, cand=c, dist=d, nvox=n)
    o.transition(1)
    g.transition(1)
    for a, b in zip(o.get_state(1), g.get_state(1)):
        assert np.array_equal(a, host(b))


@pytest.mark.parametrize("name", ["tiny", "small2", "small3", "edge"])
@pytest.mark.parametrize("wide", WIDE)
def test_inpaint_mean_end_to_end_bitexact(vi, name, wide):
    # MEAN reconstructions are exact in float32 (integer sums, one division),
    # so the whole algorithm is deterministic across implementations
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, wide=wide, levels=L, seed=12, recon_mode=1)
    a = o.inpaint()
    b = host(g.inpaint())
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["tiny", "small2", "small3", "edge"])
def test_inpaint_weighted_end_to_end(vi, name):
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, levels=L, seed=12)
    a = o.inpaint()
    b = host(g.inpaint())
    keep = clip.mask == 0
    assert np.array_equal(b[keep], clip.video[keep])
    hole = ~keep
    same = (a[hole] == b[hole]).all(axis=-1).mean()
    print(f"[{name}] un-forced weighted end-to-end: {100 * same:.2f} % hole voxels identical")
    assert same > 0.9


def test_inpaint_level_iterations_match(vi):
    clip, L = CLIPS["small2"]()
    o, g = make_pair(vi, clip, levels=1, seed=2, recon_mode=1)
    o.onion_init()
    g.onion_init()
    assert o.inpaint_level(0) == g.inpaint_level(0)
    for a, b in zip(o.get_state(0), g.get_state(0)):
        assert np.array_equal(a, host(b))


def test_errors(vi):
    clip, L = CLIPS["tiny"]()
    g = vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=1)
    with pytest.raises(vi.ViError) as e:
        g.reconstruct(0)
    assert e.value.status == -4
    with pytest.raises(vi.ViError):
        g.nnf_search(3)
    bad = torch.full((8, 32, 32), 10 ** 6, dtype=torch.int32, device="cuda")
    with pytest.raises(vi.ViError) as e:
        g.set_state(0, cand=bad)
    assert e.value.status == -1
    with pytest.raises(vi.ViError) as e:
        vi.Clip(dev(clip.occluded_input()), dev(clip.mask), levels=1, jf_steps=[5])
    assert e.value.status == -1
    m = np.zeros_like(clip.mask)
    m[2:5] = 1
    with pytest.raises(vi.ViError) as e:
        vi.Clip(dev(clip.occluded_input()), dev(m), levels=1)
    assert e.value.status == -5


@pytest.mark.parametrize("name", ["tiny", "small2", "small3", "edge"])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("wide", WIDE)
def test_onion_layers_teacher_forced(vi, name, mode, wide):
    # the peel one layer at a time, each layer started from the oracle's
    # state: the layer (erosion), the masked search of its targets and the
    # reconstruction from contributors outside H' (Eqs. (3.10)-(3.11))
    clip, L = CLIPS[name]()
    o, g = make_pair(vi, clip, wide=wide, levels=L, seed=4, recon_mode=mode)
    lv = L - 1
    Hp = o.sets(lv)[0].copy()
    gHp = dev(Hp)
    layer = 0
    while Hp.any():
        if layer > 0:
            r, c, d, n = o.get_state(lv)
            g.set_state(lv, rgbt=r, cand=c, dist=d, nvox=n)
        E, bd, _, oo = o.onion_layer(Hp, layer)
        go = host(g.onion_layer(gHp, layer))
        assert np.array_equal(E, host(gHp)), layer
        ro, co, do, no = o.get_state(lv)
        rg, cg, dg, ng = (host(t) for t in g.get_state(lv))
        assert np.array_equal(co, cg), f"cand layer {layer}"
        assert np.array_equal(do, dg), f"dist layer {layer}"
        assert np.array_equal(no, ng), f"nvox layer {layer}"
        px = np.flatnonzero(bd.ravel())
        assert len(go) == len(px) == len(oo)
        if mode == 0:
            assert_recon_close(oo, go, ro, rg, px)
        else:
            assert np.array_equal(ro, rg), layer
            assert np.abs(oo - go).max(initial=0) <= 1e-6
        Hp = E
        layer += 1
    assert layer >= 2


# ---------------------------------------------------------------------------
# temporally subsampled pyramids (Sec. 3.6): 20 -> 10 -> 5 frames
# ---------------------------------------------------------------------------

def _temporal_clip():
    return synth.small(24, 61, 47, 20, levels=3, frac=0.05)


def test_temporal_create_matches_oracle(vi):
    clip = _temporal_clip()
    o, g = make_pair(vi, clip, levels=3, temporal_subsample=1)
    for lv in range(3):
        assert o.info(lv) == g.info(lv)
        assert o.dims(lv)[2] == (20, 10, 5)[lv]
        for a, b in zip(o.sets(lv), g.sets(lv)):
            assert np.array_equal(a, host(b)), lv
        for a, b in zip(o.get_state(lv), g.get_state(lv)):
            assert np.array_equal(a, host(b)), lv


@pytest.mark.parametrize("em_iter", [0, 2])
@pytest.mark.parametrize("wide", WIDE)
def test_temporal_search_bitexact(vi, em_iter, wide):
    clip = _temporal_clip()
    o, g = make_pair(vi, clip, wide=wide, levels=3, seed=7, temporal_subsample=1)
    for lv in range(3):
        rgbt, cand = _forced_state(o, lv, 300 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        g.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, em_iter)
        g.nnf_search(lv, em_iter)
        for a, b in zip(o.get_state(lv)[1:], g.get_state(lv)[1:]):
            assert np.array_equal(a, host(b)), lv


def test_temporal_transition_bitexact(vi):
    clip = _temporal_clip()
    o, g = make_pair(vi, clip, levels=3, seed=5, recon_mode=1, temporal_subsample=1)
    for lv in (2, 1):
        rgbt, cand = _forced_state(o, lv, 10 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, 0)
        g.set_state(lv, *o.get_state(lv))
        o.transition(lv - 1)
        g.transition(lv - 1)
        for a, b in zip(o.get_state(lv - 1), g.get_state(lv - 1)):
            assert np.array_equal(a, host(b)), lv


def test_temporal_inpaint_mean_end_to_end_bitexact(vi):
    clip = _temporal_clip()
    o, g = make_pair(vi, clip, levels=3, seed=12, recon_mode=1, temporal_subsample=1)
    assert np.array_equal(o.inpaint(), host(g.inpaint()))


def test_temporal_weighted_reconstruction_close(vi):
    clip = _temporal_clip()
    o, g = make_pair(vi, clip, levels=3, seed=9, temporal_subsample=1)
    for lv in range(3):
        rgbt, cand = _forced_state(o, lv, 400 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, 0)
        g.set_state(lv, *o.get_state(lv))
        oo, _ = o.reconstruct(lv, 0)
        go, _ = g.reconstruct(lv, 0)
        hole_idx = np.flatnonzero(o.sets(lv)[0].ravel())
        assert_recon_close(oo, host(go), o.get_state(lv)[0], host(g.get_state(lv)[0]), hole_idx)


# ---------------------------------------------------------------------------
# single images (T = 1, 5x5x1 patches): 2-D image inpainting
# ---------------------------------------------------------------------------

def _edge_image():
    c = synth.image(95, 64, 52, levels=2)
    c.mask[:] = 0
    c.mask[0, 0:7, 0:9] = 1
    c.mask[0, 44:52, 50:64] = 1
    return c


IMAGES = {
    "img2": lambda: (synth.image(93, 77, 61, frac=0.05, levels=2), 2),
    "img3": lambda: (synth.image(94, 160, 120, frac=0.04, levels=3, kind="box"), 3),
    "imgedge": lambda: (_edge_image(), 2),
}
P2 = dict(patch=(5, 5, 1))


@pytest.mark.parametrize("name", list(IMAGES))
@pytest.mark.parametrize("wide", WIDE)
def test_image_create_and_search_bitexact(vi, name, wide):
    clip, L = IMAGES[name]()
    o, g = make_pair(vi, clip, wide=wide, levels=L, seed=7, **P2)
    for lv in range(L):
        assert o.info(lv) == g.info(lv)
        for a, b in zip(o.sets(lv), g.sets(lv)):
            assert np.array_equal(a, host(b)), lv
        for a, b in zip(o.get_state(lv), g.get_state(lv)):
            assert np.array_equal(a, host(b)), lv
        rgbt, cand = _forced_state(o, lv, 500 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        g.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, 1)
        g.nnf_search(lv, 1)
        for a, b in zip(o.get_state(lv)[1:], g.get_state(lv)[1:]):
            assert np.array_equal(a, host(b)), lv


@pytest.mark.parametrize("name", list(IMAGES))
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_image_reconstruct_parity(vi, name, mode):
    clip, L = IMAGES[name]()
    o, g = make_pair(vi, clip, levels=L, seed=9, **P2)
    for lv in range(L):
        rgbt, cand = _forced_state(o, lv, 600 + lv)
        o.set_state(lv, rgbt=rgbt, cand=cand)
        o.nnf_search(lv, 0)
        g.set_state(lv, *o.get_state(lv))
        oo, os_ = o.reconstruct(lv, mode)
        go, gs = g.reconstruct(lv, mode)
        o_r = o.get_state(lv)[0]
        g_r = host(g.get_state(lv)[0])
        hole_idx = np.flatnonzero(o.sets(lv)[0].ravel())
        if mode == 0:
            assert_recon_close(oo, host(go), o_r, g_r, hole_idx)
        else:
            assert np.array_equal(o_r, g_r)
            assert os_ == int(host(gs)[0])


@pytest.mark.parametrize("name", list(IMAGES))
def test_image_inpaint_mean_end_to_end_bitexact(vi, name):
    clip, L = IMAGES[name]()
    o, g = make_pair(vi, clip, levels=L, seed=12, recon_mode=1, **P2)
    assert np.array_equal(o.inpaint(), host(g.inpaint()))


def test_image_weighted_end_to_end(vi):
    clip, L = IMAGES["img3"]()
    o, g = make_pair(vi, clip, levels=L, seed=12, **P2)
    a = o.inpaint()
    b = host(g.inpaint())
    keep = clip.mask == 0
    assert np.array_equal(b[keep], clip.video[keep])
    same = (a[~keep] == b[~keep]).all(axis=-1).mean()
    print(f"[img3] un-forced weighted end-to-end: {100 * same:.2f} % hole pixels identical")
    assert same > 0.9


def test_image_parameter_errors(vi):
    clip, _ = IMAGES["img2"]()
    v = dev(clip.occluded_input())
    m = dev(clip.mask)
    with pytest.raises(vi.ViError):  # 5x5x1 patches on a video
        vi.Clip(dev(np.repeat(clip.occluded_input(), 3, 0)), dev(np.repeat(clip.mask, 3, 0)),
                levels=1, **P2)
    with pytest.raises(vi.ViError):  # no temporal subsampling of one image
        vi.Clip(v, m, levels=2, temporal_subsample=1, **P2)
    with pytest.raises(vi.ViError):  # 5x5x5 patches on one image
        vi.Clip(v, m, levels=2)
