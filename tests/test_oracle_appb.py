"""Pins of the oracle's textured-patch experiment (App. B) against what is
known independently of it:

* the exact probability P(N) = E[Q(sqrt(chi2_N) / 2)] reduces, for N = 1
  and N = 2, to closed forms derived by hand (1/2 - arctan(1/2)/pi and
  1/2 - 1/(2 sqrt 5));
* it equals the same probability integrated in the other order,
  Prob(2 Z > R) with Z standard normal and R ~ chi_N independent, i.e. the
  integral of phi(z) F_chi2_N(4 z^2) over z > 0;
* a plain Monte-Carlo simulation of continuous normal patches lands
  within five standard errors of it;
* it agrees with the seven values the paper prints (App. B table): within
  30 % for the four rows the paper's ten runs could resolve (P >= 4e-4),
  within a factor 3 for the three rarest;
* the brute-force count of closer patches matches a pure-Python
  enumeration on tiny volumes, is 0 for a constant reference of value mu
  and for a volume smaller than the patch, counts a candidate equal to the
  reference, and on a noise volume its rate is the exact probability
  within the simulation's error (rounding to integers moves it by about
  1 %).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

from oracle import appb, vio
from paper_1503_05528_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "appb_table.json")


def test_closed_forms_for_one_and_two_components():
    assert abs(appb.closer_probability(1) - (0.5 - math.atan(0.5) / math.pi)) < 1e-12
    assert abs(appb.closer_probability(2) - (0.5 - 1.0 / (2.0 * math.sqrt(5.0)))) < 1e-12


@pytest.mark.parametrize("N", [1, 3, 9, 25, 27, 49, 81, 121, 125])
def test_other_order_of_integration(N):
    other, _ = integrate.quad(lambda z: stats.norm.pdf(z) * stats.chi2.cdf(4 * z * z, N),
                              0.0, 40.0, points=[math.sqrt(N) / 2], limit=500, epsabs=0.0,
                              epsrel=1e-12)
    assert abs(appb.closer_probability(N) / other - 1.0) < 1e-9


@pytest.mark.parametrize("N", [9, 25])
def test_monte_carlo_of_continuous_patches(N):
    rng = np.random.default_rng(11)
    hits, n = 0, 0
    for _ in range(8):
        W = rng.normal(0.0, 5.0, (250_000, N))
        V = rng.normal(0.0, 5.0, (250_000, N))
        hits += int((((W - V) ** 2).sum(1) < (W ** 2).sum(1)).sum())
        n += W.shape[0]
    P = appb.closer_probability(N)
    se = math.sqrt(P * (1 - P) / n)
    assert abs(hits / n - P) < 5 * se, (hits / n, P, se)


def test_paper_table():
    gold = json.load(open(GOLD))
    for row in gold["rows"]:
        N = int(np.prod(row["patch"]))
        P, printed = appb.closer_probability(N), row["probability"]
        if printed >= 4e-4:
            assert abs(P / printed - 1.0) < 0.30, (row, P)
        else:
            assert 1 / 3 < P / printed < 3, (row, P)
    # the paper's closing example: one closer 5x5x5 patch in about 170^3
    # candidates
    assert 0.3 < appb.closer_probability(125) * 170 ** 3 < 3


def _brute(ref, vol, patch, mu):
    pw, ph, pt = patch
    T, H, W = vol.shape
    out = []
    for w in ref.reshape(len(ref), -1).astype(int):
        dz = sum((int(a) - mu) ** 2 for a in w)
        c = 0
        for t in range(T - pt + 1):
            for y in range(H - ph + 1):
                for x in range(W - pw + 1):
                    v = vol[t:t + pt, y:y + ph, x:x + pw].astype(int).ravel()
                    c += sum((a - b) ** 2 for a, b in zip(w, v)) < dz
        out.append(c)
    return np.array(out, np.uint64)


@pytest.mark.parametrize("patch,mu", [((3, 3, 3), 128), ((2, 3, 1), 128), ((3, 1, 2), 100),
                                      ((1, 1, 1), 140)])
def test_count_matches_enumeration(oracle_lib, patch, mu):
    vol = synth.noise(3, (5, 7, 9))
    ref = synth.noise(4, (6, patch[2], patch[1], patch[0]))
    assert np.array_equal(vio.closer_than_constant(ref, vol, patch, mu),
                          _brute(ref, vol, patch, mu))


def test_count_special_cases(oracle_lib):
    vol = synth.noise(5, (6, 8, 10))
    p = (3, 3, 3)
    const = np.full((1, 3, 3, 3), 131, np.uint8)
    assert vio.closer_than_constant(const, vol, p, 131)[0] == 0  # SSD(W, Z) = 0
    inside = vol[1:4, 2:5, 4:7][None].copy()
    assert vio.closer_than_constant(inside, vol, p, 128)[0] >= 1  # itself, at distance 0
    assert not vio.closer_than_constant(inside, vol[:2], p, 128).any()  # T < 3: no candidate
    assert vio.closer_than_constant(inside[:0], vol, p, 128).shape == (0,)


def test_count_rate_is_the_probability(oracle_lib):
    # 3x3 patches over a 200 x 200 x 4 noise stack: about 1e7 pairs
    vol = synth.noise(6, (4, 200, 200))
    ref = synth.noise(7, (64, 1, 3, 3))
    c = vio.closer_than_constant(ref, vol, (3, 3, 1), 128).astype(np.float64)
    n_cand = 4 * 198 * 198
    rate = c / n_cand
    # standard error from the spread over reference patches (the candidates
    # of one reference share it, so the pairs are not independent)
    se = rate.std(ddof=1) / math.sqrt(len(rate))
    P = appb.closer_probability(9)
    assert abs(rate.mean() - P) < 5 * se + 0.02 * P, (rate.mean(), P, se)


def test_noise_generator_law():
    v = synth.noise(8, (8, 128, 128)).astype(np.float64)
    assert abs(v.mean() - 128) < 0.05
    # rounding adds 1/12 to the variance of the continuous law
    assert abs(v.var() - (25 + 1 / 12)) < 0.2
