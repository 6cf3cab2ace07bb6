"""Seeded synthetic workloads shaped like the paper's experiments.

The paper evaluates randomized CP on random low-rank tensors with additive
white noise (Section 4.1: 100x100x100, 400x400x400 and 100^4 tensors of
rank R=50, plus a noise sweep).  This module builds such inputs from a
seed; it holds none of the decomposition's arithmetic and is the only
module that both the GPU path's tests and the CPU oracle's tests share.

Every tensor is a dense C-order float32 array

    X = sum_r  w_r * a1_r o a2_r o ... o aN_r   +   sigma * E

where the factor columns are drawn as described per workload, E is iid
N(0,1) and sigma = noise * rms(X_clean) (amplitude signal-to-noise ratio
1/noise; the paper never defines SNR, this is the reading used here).
Random numbers come from numpy's PCG64 generator seeded with ``seed``:
factors first (mode 0, 1, ...), then the noise, drawn slice by slice
along mode 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np


@dataclass
class Workload:
    """A synthetic tensor plus the ground truth it was built from."""
    X: np.ndarray                      # float32, C-order
    factors: List[np.ndarray]          # float64, I_n x R (true factor columns)
    weights: np.ndarray                # float64, R (true column weights)
    sigma: float                       # absolute noise standard deviation
    meta: dict = field(default_factory=dict)


def _gaussian_factors(rng, dims, R):
    return [rng.standard_normal((int(I), R)) for I in dims]


def _collinear_factors(rng, dims, R, cos):
    """Unit-norm columns with pairwise cosine ``cos`` in every mode.

    Each mode takes an orthonormal I_n x R basis (QR of a Gaussian matrix)
    and mixes it with the transposed Cholesky factor of the target Gram
    C = (1-cos) I + cos 11^T, so A^T A = C exactly.
    """
    C = (1.0 - cos) * np.eye(R) + cos * np.ones((R, R))
    L = np.linalg.cholesky(C)
    out = []
    for I in dims:
        G = rng.standard_normal((int(I), R))
        Qb, Rb = np.linalg.qr(G)
        Qb = Qb * np.sign(np.diag(Rb))
        out.append(Qb @ L.T)
    return out


def _assemble(dims, factors, weights, noise, rng, slab=None, dtype=np.float32):
    """Dense low-rank tensor plus white noise, built slab by slab on mode 0."""
    dims = tuple(int(d) for d in dims)
    X = np.empty(dims, dtype=dtype)
    rest = dims[1:]
    R = len(weights)
    # Column r of the trailing factor product, as a (prod(rest), R) matrix,
    # in C order over modes 1..N-1.
    tail = np.ones((1, R))
    for A in factors[1:]:
        tail = (tail[:, None, :] * A[None, :, :]).reshape(-1, R)
    head = factors[0] * weights[None, :]
    if slab is None:
        slab = max(1, int(2 ** 24 // max(1, tail.shape[0])))
    sumsq = 0.0
    for i0 in range(0, dims[0], slab):
        i1 = min(dims[0], i0 + slab)
        block = head[i0:i1] @ tail.T
        sumsq += float(np.dot(block.ravel(), block.ravel()))
        X[i0:i1] = block.reshape((i1 - i0,) + rest)
    count = float(np.prod(dims))
    rms = np.sqrt(sumsq / count) if count > 0 else 0.0
    sigma = float(noise) * rms
    if sigma > 0.0:
        for i0 in range(0, dims[0], slab):
            i1 = min(dims[0], i0 + slab)
            E = rng.standard_normal((i1 - i0,) + rest)
            X[i0:i1] = (X[i0:i1].astype(np.float64) + sigma * E).astype(dtype)
    return X, sigma, rms


def low_rank(dims: Sequence[int], R: int, noise: float, seed: int,
             kind: str = "gaussian", cos: float = 0.8, dtype=np.float32) -> Workload:
    """Random rank-R tensor plus noise.

    kind:
      "gaussian"    every factor entry iid N(0,1), unit weights;
      "logweights"  as "gaussian", but the mode-0 columns are rescaled to
                    norms 10**(2 u_r), u_r ~ U(0,1) (log-uniform in [1,100]);
      "collinear"   unit-norm columns with pairwise cosine ``cos`` in every
                    mode, unit weights.
    dtype is the storage type of X (float32 for every workload; float64
    only for exact-arithmetic checks of the oracle).
    """
    rng = np.random.default_rng(seed)
    dims = [int(d) for d in dims]
    if kind == "gaussian":
        factors = _gaussian_factors(rng, dims, R)
        weights = np.ones(R)
    elif kind == "logweights":
        factors = _gaussian_factors(rng, dims, R)
        u = rng.uniform(0.0, 1.0, R)
        norms = 10.0 ** (2.0 * u)
        A0 = factors[0]
        A0 = A0 / np.linalg.norm(A0, axis=0, keepdims=True) * norms[None, :]
        factors[0] = A0
        weights = np.ones(R)
    elif kind == "collinear":
        factors = _collinear_factors(rng, dims, R, cos)
        weights = np.ones(R)
    else:
        raise ValueError(f"unknown factor kind {kind!r}")
    X, sigma, rms = _assemble(dims, factors, weights, noise, rng, dtype=dtype)
    return Workload(X=X, factors=factors, weights=weights, sigma=sigma,
                    meta=dict(dims=dims, R=R, noise=noise, seed=seed, kind=kind,
                              rms_clean=rms))


# ---------------------------------------------------------------------------
# The workloads, by name.  Data seed 20170327 + index; test-matrix seed
# 1000 + index.

WORKLOADS = {
    # 100^3, R=5, factors N(0,1), noise 0.01 rms; k=5 p=10 q=2, 50 sweeps.
    "rcp100": dict(dims=(100, 100, 100), R=5, noise=0.01, kind="gaussian",
                   k=5, p=10, q=2, iters=50, data_seed=20170327, seed=1000),
    # 400^3, R=20, mode-0 norms log-uniform in [1,100], noise 0.05 rms;
    # k=20 p=10 q=2, 100 sweeps.
    "rcp400": dict(dims=(400, 400, 400), R=20, noise=0.05, kind="logweights",
                   k=20, p=10, q=2, iters=100, data_seed=20170328, seed=1001),
    # 2048x2048x512, R=50, noise 0.1 rms; k=50 p=10 q=2, 100 sweeps.
    "rcp2048": dict(dims=(2048, 2048, 512), R=50, noise=0.1, kind="gaussian",
                    k=50, p=10, q=2, iters=100, data_seed=20170329, seed=1002),
    # 256x256x256x64, R=30, pairwise cosine 0.8, noise 0.05 rms;
    # k=30 p=15 q in {1,3}, 200 sweeps.
    "rcp4way": dict(dims=(256, 256, 256, 64), R=30, noise=0.05, kind="collinear",
                    k=30, p=15, q=3, iters=200, data_seed=20170330, seed=1003),
    # the same tensor with a single power iteration
    "rcp4way_q1": dict(dims=(256, 256, 256, 64), R=30, noise=0.05, kind="collinear",
                       k=30, p=15, q=1, iters=200, data_seed=20170330, seed=1003),
}


def low_rank_device(dims: Sequence[int], R: int, noise: float, seed: int,
                    kind: str = "gaussian", cos: float = 0.8, device="cuda"):
    """The same recipe as ``low_rank`` (factors drawn with numpy from ``seed``),
    assembled on the GPU with torch, for tensors too large to build on the
    host quickly.  The noise comes from torch's generator seeded with ``seed``
    (a different stream from numpy's, so the tensor differs from
    ``low_rank``'s by its noise).  Returns (X float32 on device, factors,
    weights, sigma)."""
    import torch
    rng = np.random.default_rng(seed)
    dims = [int(d) for d in dims]
    if kind == "gaussian":
        factors = _gaussian_factors(rng, dims, R)
    elif kind == "logweights":
        factors = _gaussian_factors(rng, dims, R)
        norms = 10.0 ** (2.0 * rng.uniform(0.0, 1.0, R))
        factors[0] = factors[0] / np.linalg.norm(factors[0], axis=0, keepdims=True) * norms[None, :]
    elif kind == "collinear":
        factors = _collinear_factors(rng, dims, R, cos)
    else:
        raise ValueError(f"unknown factor kind {kind!r}")
    weights = np.ones(R)
    dev = torch.device(device)
    tail = torch.ones((1, R), dtype=torch.float64, device=dev)
    for A in factors[1:]:
        At = torch.from_numpy(A).to(dev)
        tail = (tail[:, None, :] * At[None, :, :]).reshape(-1, R)
    head = torch.from_numpy(factors[0]).to(dev)
    X = torch.empty(dims, dtype=torch.float32, device=dev)
    Xf = X.view(dims[0], -1)
    slab = max(1, int(2 ** 26 // max(1, tail.shape[0])))
    sumsq = 0.0
    for i0 in range(0, dims[0], slab):
        i1 = min(dims[0], i0 + slab)
        block = head[i0:i1] @ tail.T
        sumsq += float((block * block).sum())
        Xf[i0:i1] = block.to(torch.float32)
    rms = float(np.sqrt(sumsq / float(np.prod(dims))))
    sigma = float(noise) * rms
    if sigma > 0.0:
        g = torch.Generator(device=dev)
        g.manual_seed(int(seed))
        for i0 in range(0, dims[0], slab):
            i1 = min(dims[0], i0 + slab)
            E = torch.randn((i1 - i0, Xf.shape[1]), generator=g, dtype=torch.float64, device=dev)
            Xf[i0:i1] = (Xf[i0:i1].to(torch.float64) + sigma * E).to(torch.float32)
    return X, factors, weights, sigma


def make(name: str, **overrides) -> Workload:
    cfg = dict(WORKLOADS[name])
    cfg.update(overrides)
    return low_rank(cfg["dims"], cfg["R"], cfg["noise"], cfg["data_seed"],
                    kind=cfg["kind"])


def batch_problems(count: int, seed: int, lo: int = 32, hi: int = 256,
                   rlo: int = 4, rhi: int = 16, noise: float = 0.05):
    """Shapes and ranks of a batch of independent 3-way problems.

    Each mode size is uniform on [lo, hi], each true rank uniform on
    [rlo, rhi].  Returns a list of (dims, R, data_seed).
    """
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        dims = tuple(int(x) for x in rng.integers(lo, hi + 1, size=3))
        R = int(rng.integers(rlo, rhi + 1))
        out.append((dims, R, int(seed * 1000 + b)))
    return out
