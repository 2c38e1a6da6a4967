"""Whole inpaintings in MEAN mode (bit-exact by construction) against the
oracle over seeded random configurations: clip sizes that are not multiples
of anything, 1-3 pyramid levels, lambda, PatchMatch iterations, jump-flood
strides, rho, EM iteration counts, seeds, hole shapes and sizes, temporal
subsampling, and 5x5x1 images.  Each case is independent; the parameters
are printed before it runs."""
import numpy as np
import pytest
import torch

from oracle import vio
from paper_1503_05528_amd import synth

pytestmark = pytest.mark.gpu


def _cases(n=40, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        image = i % 4 == 3
        W = int(rng.integers(30, 90))
        H = int(rng.integers(24, 70))
        T = 1 if image else int(rng.integers(6, 14))
        levels = int(rng.integers(1, 4))
        temporal = (not image) and levels > 1 and T >= 10 and bool(rng.integers(0, 2))
        # every level must keep a patch's worth of pixels and frames
        while levels > 1 and (min(W, H) >> (levels - 1) < 6 or
                              (temporal and (T + (1 << (levels - 1)) - 1) >> (levels - 1) < 5)):
            levels -= 1
        if levels == 1:
            temporal = False
        n_jf = int(rng.integers(1, 4))
        prm = dict(levels=levels, lam=int(rng.choice([0, 7, 50, 130])),
                   pm_iters=int(rng.integers(1, 8)), n_jf=n_jf,
                   jf_steps=tuple(int(s) for s in rng.integers(1, 5, n_jf)),
                   rho=float(rng.choice([0.5, 0.6, 0.75])),
                   em_max_iters=int(rng.integers(1, 6)), em_tol=-1.0, recon_mode=1,
                   seed=int(rng.integers(0, 2**31)),
                   temporal_subsample=1 if temporal else 0)
        if image:
            prm["patch"] = (5, 5, 1)
        clip = dict(seed=int(rng.integers(0, 10000)), W=W, H=H, T=T,
                    frac=float(rng.uniform(0.01, 0.08)),
                    kind=str(rng.choice(["box", "ellipse"])))
        out.append((clip, prm))
    return out


CASES = _cases()


@pytest.mark.parametrize("i", range(len(CASES)))
def test_random_configuration_mean_inpainting_bitexact(i):
    from paper_1503_05528_amd import vi
    c, prm = CASES[i]
    print(f"[case] {i}: clip {c} params {prm}", flush=True)
    clip = synth.small(c["seed"], c["W"], c["H"], c["T"], frac=c["frac"],
                       levels=prm["levels"], kind=c["kind"])
    v, m = clip.occluded_input(), clip.mask
    kw = {k: v for k, v in prm.items() if k != "n_jf"}  # jf_steps sets n_jf
    op = vio.default_params(**kw)
    gp = vi.default_params(**kw)
    # which form the search passes take (results do not depend on it): the
    # library's choice, one lane everywhere, or the wide form up to a list
    # size that splits these clips' levels between the two
    gp.wide_pass_max = (-1, 0, 600, 4000)[(i // 2) % 4]
    print(f"    wide_pass_max {gp.wide_pass_max}", flush=True)
    try:
        ref = vio.Oracle(v, m, params=op).inpaint()
    except vio.OracleError as e:
        # a level without any hole-free patch: the library refuses it too
        with pytest.raises(vi.ViError):
            vi.Clip(torch.from_numpy(v).cuda(), torch.from_numpy(m).cuda(), params=gp)
        print(f"    refused by both: {e}", flush=True)
        return
    g = vi.Clip(torch.from_numpy(v).cuda(), torch.from_numpy(m).cuda(), params=gp)
    out = g.inpaint().cpu().numpy()
    g.close()
    assert np.array_equal(out, ref)
