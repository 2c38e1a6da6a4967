"""Basis of the dimensionality-reduced patch space (test infrastructure
only: the tests, the smoke check and the benchmark's CPU-baseline leg use
it; the HIP library never does).

Sec. 5 proposes dimensionality-reducing transformations of the patch space
as an acceleration without giving one; the reading here is principal
component analysis of a level's source patches:

* the patch vector x lists, offset by offset (dt, dy, dx), the channels
  R, G, B, Tx, Ty; weighting the texture channels by sqrt(lambda) makes the
  squared Euclidean distance of weighted vectors the patch distance;
* the covariance of the weighted vectors of a sample of sources (every
  k-th source in ascending order) is formed from exact integer moments:
  C_ij = (w_i w_j) (S_ij / n - (S_i / n)(S_j / n)) in double precision;
* the basis is its d leading eigenvectors (numpy's symmetric eigensolver),
  quantised as Q[k][i] = rint(256 w_i b_ik) to 16-bit integers, so that
  features f = (Q x + 128) >> 8 approximate the projections b_k . (w x).
"""
from __future__ import annotations

import math

import numpy as np


def weights(dim: int, lam: int) -> np.ndarray:
    w = np.ones(dim, np.float64)
    w[3::5] = math.sqrt(lam)
    w[4::5] = math.sqrt(lam)
    return w


def covariance(S1, S2, n: int, lam: int) -> np.ndarray:
    """Covariance of the weighted patch vectors from the exact moments."""
    dim = len(S1)
    w = weights(dim, lam)
    m = np.asarray(S1, np.float64) / n
    e2 = np.asarray(S2, np.float64).reshape(dim, dim) / n
    return np.outer(w, w) * (e2 - np.outer(m, m))


def basis(C: np.ndarray, d: int):
    """(eigenvalues [d] descending, eigenvectors [dim][d]) of the d
    leading principal directions."""
    vals, vecs = np.linalg.eigh(C)
    order = np.argsort(vals)[::-1][:d]
    return vals[order], vecs[:, order]


def quantize(B: np.ndarray, lam: int) -> np.ndarray:
    """Q [d][dim] int16 = rint(256 w_i b_ik)."""
    dim = B.shape[0]
    q = np.rint(256.0 * weights(dim, lam)[:, None] * B).T
    if np.abs(q).max() > 32767:
        raise ValueError("basis entries out of range")
    return np.ascontiguousarray(q.astype(np.int16))
