"""Exact probability behind the textured-patch table of App. B (test
infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the HIP library never does).

App. B compares, for a white-noise reference patch W of N i.i.d. normal
components (variance sigma^2), a random patch V of the same law with the
constant patch Z of the law's mean mu.  It observes that the squared
distance from W to V is chi-square distributed with twice the scale of the
distance from W to Z, and estimates P = Prob(||W - V||^2 < ||W - Z||^2) by
simulation for seven patch sizes.

The probability has an exact one-dimensional form.  Centre at mu; the
event is ||V||^2 < 2 <W, V>.  Given V, <W, V> is normal with variance
sigma^2 ||V||^2, so the event has conditional probability
Q(||V|| / (2 sigma)), Q the standard normal upper tail; ||V||^2 / sigma^2
is chi-square with N degrees of freedom.  Hence

    P(N) = E[ Q( sqrt(X) / 2 ) ],   X ~ chi2(N),

independent of sigma.  It is evaluated here by adaptive quadrature of the
chi-square density times Q over the interval that holds all but 1e-17 of
the chi-square mass, in double precision.
"""
from __future__ import annotations

import math

from scipy import integrate, stats


def closer_probability(N: int) -> float:
    """P(N) of App. B: the probability that a random patch of N i.i.d.
    normal components is closer (squared l2) to a random reference patch
    of the same law than the constant patch of the law's mean."""
    if N < 1:
        raise ValueError("N >= 1")
    hi = stats.chi2.isf(1e-17, N)

    def f(x):
        return stats.chi2.pdf(x, N) * stats.norm.sf(math.sqrt(x) / 2.0)

    v, _ = integrate.quad(f, 0.0, hi, points=[max(N - 2.0, 0.5)], limit=500, epsabs=0.0,
                          epsrel=1e-12)
    return float(v)
