"""Comparison metrics (oracle side; TEST INFRASTRUCTURE ONLY).

relative_error   ||X - Xhat||_F / ||X||_F, the accuracy measure of Section 4,
                 computed in float64 slab by slab from (lambda, factors).
congruence       factor match score of two Kruskal tensors: for components
                 r, s the product over modes of |cos(a_{n,r}, b_{n,s})|,
                 matched one-to-one by the Hungarian method.  CP factors are
                 unique only up to permutation, scaling and sign, so this is
                 what two correct decompositions can be compared on.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
from scipy.optimize import linear_sum_assignment

from .rcp import khatri_rao


def relative_error(X: np.ndarray, lam: np.ndarray, factors: Sequence[np.ndarray],
                   slab_elems: int = 1 << 24) -> float:
    X = np.asarray(X)
    shape = X.shape
    tail = khatri_rao([np.asarray(A, dtype=np.float64) for A in factors[1:]])
    head = np.asarray(factors[0], dtype=np.float64) * np.asarray(lam, dtype=np.float64)[None, :]
    rest = int(np.prod(shape[1:]))
    slab = max(1, slab_elems // max(1, rest))
    num = 0.0
    den = 0.0
    Xm = X.reshape(shape[0], rest)
    for i0 in range(0, shape[0], slab):
        i1 = min(shape[0], i0 + slab)
        blk = Xm[i0:i1].astype(np.float64)
        diff = blk - head[i0:i1] @ tail.T
        num += float(np.sum(diff * diff))
        den += float(np.sum(blk * blk))
    return float(np.sqrt(num / den)) if den > 0 else 0.0


def congruence(fa: Sequence[np.ndarray], fb: Sequence[np.ndarray]):
    """Returns (mean, min, permutation) of the matched congruences.

    permutation[r] is the component of ``fb`` matched to component r of ``fa``.
    """
    Ra = fa[0].shape[1]
    Rb = fb[0].shape[1]
    C = np.ones((Ra, Rb))
    for A, B in zip(fa, fb):
        A = np.asarray(A, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        na = np.linalg.norm(A, axis=0)
        nb = np.linalg.norm(B, axis=0)
        na[na == 0] = 1.0
        nb[nb == 0] = 1.0
        C = C * np.abs((A / na).T @ (B / nb))
    rows, cols = linear_sum_assignment(-C)
    vals = C[rows, cols]
    perm = np.full(Ra, -1)
    perm[rows] = cols
    return float(np.mean(vals)), float(np.min(vals)), perm


def compression_ratios(I: int, J: int, K: int, R: int):
    """Storage ratios of Section 4.2.1's compression note: a rank-R SVD of a
    reshaped I*J x K matrix vs a rank-R CP model of the I x J x K tensor."""
    c_svd = (I * J * K) / (R * (I * J + K + 1))
    c_cp = (I * J * K) / (R * (I + J + K + 1))
    return c_svd, c_cp
