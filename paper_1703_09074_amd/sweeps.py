"""Validation sweeps of the randomized CP decomposition on the GPU, over many
independent runs at once through the batched path:

  * ``theorem1``: the empirical check of Theorem 1 (eq. theorem, Appendix A):
    the mean over Gaussian test matrices of the projection error
    ||X - X x_1 Q_1 Q_1^T ... x_N Q_N Q_N^T|| against
    sqrt(1 + k / (p - 1)) sqrt(sum_n sum_{j > k} sigma_nj^2), for a
    noise-free rank-R tensor, q = 0, the bases taken from X itself;
  * ``snr_sweep``: the relative error of rCP-ALS (q = 0 and q = 2) and of
    deterministic CP-ALS against the signal-to-noise ratio (Section 4.1, the
    SNR figure), the noise amplitude being rms(X_clean) / SNR.

The bases, cores and decompositions come from the library's kernels; what
this module adds is the bookkeeping of the experiment: the synthetic inputs,
the singular values behind the bound (float64 on the host) and the averages.
"""
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import Batch, Plan, _lib, synth


def _torch():
    import torch
    return torch


def unfolding_spectra(X: np.ndarray) -> List[np.ndarray]:
    """Squared singular values of every mode-n unfolding (descending), as the
    eigenvalues of X_(n) X_(n)^T in float64."""
    X = np.asarray(X, dtype=np.float64)
    out = []
    for n in range(X.ndim):
        Xn = np.moveaxis(X, n, 0).reshape(X.shape[n], -1)
        ev = np.linalg.eigvalsh(Xn @ Xn.T)[::-1]
        out.append(np.clip(ev, 0.0, None))
    return out


def theorem1_bound(spectra: Sequence[np.ndarray], k: int, p: int) -> float:
    """sqrt(1 + k / (p - 1)) sqrt(sum_n sum_{j > k} sigma_nj^2)."""
    tail = sum(float(np.sum(s[k:])) for s in spectra)
    return math.sqrt(1.0 + k / (p - 1.0)) * math.sqrt(tail)


def _cores(problems, X, device):
    """Decompose X once per problem and return the cores (device views)
    with the elapsed time: one batch when the batched path takes the
    problems, else one plan per problem."""
    torch = _torch()
    try:
        b = Batch(problems, device=device)
    except _lib.RcpError as e:
        if e.status != _lib.RCP_ERR_UNSUPPORTED:
            raise
        b = None
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    if b is not None:
        b.decompose([X] * len(problems))
        torch.cuda.synchronize(device)
        dt = time.perf_counter() - t0
        return [b.core(i) for i in range(len(problems))], dt, "batch", b
    cores, plans = [], []
    for pr in problems:
        pl = Plan(pr["dims"], pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0, pr["seed"],
                  scheme=pr["scheme"], device=device)
        pl.decompose(X)
        plans.append(pl)
    torch.cuda.synchronize(device)
    dt = time.perf_counter() - t0
    return [pl.core() for pl in plans], dt, "plans", plans


def theorem1(dims: Sequence[int], R: int = 25, ks: Sequence[int] = (5, 10, 15, 20),
             runs: int = 100, p: int = 2, data_seed: int = 20170401, seed0: int = 0,
             X: Optional[np.ndarray] = None, device="cuda") -> Dict:
    """Theorem 1 over ``runs`` test-matrix seeds per target rank k.  Returns
    per k the bound, the mean / max / std of the errors, the per-run errors
    and the GPU time per run."""
    torch = _torch()
    if X is None:
        X = synth.low_rank(dims, R, 0.0, data_seed).X
    X = np.ascontiguousarray(X, dtype=np.float32)
    spectra = unfolding_spectra(X)
    normX2 = float(np.sum(X.astype(np.float64) ** 2))
    Xd = torch.from_numpy(X).to(device)
    rows = []
    for k in ks:
        probs = [dict(dims=list(X.shape), k=int(k), p=int(p), q=0, max_iters=1, tol=0.0,
                      seed=seed0 + s, scheme="independent") for s in range(runs)]
        cores, dt, path, keep = _cores(probs, Xd, device)
        # the projection is orthogonal: ||X - Xhat||^2 = ||X||^2 - ||B||^2
        b2 = torch.stack([(c.double() ** 2).sum() for c in cores]).cpu().numpy()
        errs = np.sqrt(np.clip(normX2 - b2, 0.0, None))
        bound = theorem1_bound(spectra, int(k), int(p))
        rows.append(dict(k=int(k), bound=bound, mean=float(errs.mean()), max=float(errs.max()),
                         std=float(errs.std()), holds=bool(errs.mean() <= bound),
                         errors=errs.tolist(), ms_per_run=dt * 1e3 / runs, path=path))
        del keep, cores
    return dict(dims=list(X.shape), R=R, p=p, runs=runs, normX=math.sqrt(normX2), rows=rows)


def snr_sweep(dims: Sequence[int] = (100, 100, 100), R: int = 50,
              snrs: Sequence[float] = (1, 2, 4, 8, 16), runs: int = 100,
              qs: Sequence[int] = (0, 2), p: int = 10, iters: int = 50,
              deterministic: bool = True, det_q: int = 4, data_seed: int = 20170501,
              seed0: int = 0, make: Optional[Callable] = None, device="cuda") -> Dict:
    """Relative error against SNR.  Per level, ``runs`` tensors (rank R plus
    noise of amplitude rms(X_clean) / SNR; ``make(level, snr, run)`` may
    supply them as float32 CUDA tensors), each decomposed by rCP-ALS for
    every q in ``qs`` (one batch per q) and, with ``deterministic``, by
    CP-ALS on the full tensor (eigenvector start by subspace iteration with
    ``det_q`` steps).  Returns per level and method the mean / std and the
    per-run errors (rcp_als_info.rel_err, the exact fit of Section 3.3) and
    the time per run."""
    torch = _torch()
    dims = [int(d) for d in dims]
    levels = []
    for li, snr in enumerate(snrs):
        if make is not None:
            Xs = [make(li, snr, r) for r in range(runs)]
        else:
            Xs = [synth.low_rank_device(dims, R, 1.0 / snr, data_seed + 1000 * li + r,
                                        device=device)[0] for r in range(runs)]
        methods = {}
        for q in qs:
            probs = [dict(dims=dims, k=R, p=p, q=int(q), max_iters=iters, tol=0.0,
                          seed=seed0 + r) for r in range(runs)]
            b = Batch(probs, device=device)
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            b.decompose(Xs)
            torch.cuda.synchronize(device)
            dt = time.perf_counter() - t0
            errs = np.array([inf["rel_err"] for inf in b.read_info()])
            stats = [inf["status"] for inf in b.read_info()]
            methods[f"rcp_als_q{q}"] = dict(mean=float(errs.mean()), std=float(errs.std()),
                                            errors=errs.tolist(), ms_per_run=dt * 1e3 / runs,
                                            status_nonzero=int(sum(1 for s in stats if s)))
            del b
        if deterministic:
            pl = Plan(dims, R, p, det_q, iters, 0.0, seed0, device=device, solver="cp_als")
            A = [torch.empty((d, R), dtype=torch.float32, device=device) for d in dims]
            lam = torch.empty((R,), dtype=torch.float32, device=device)
            infos = [pl._info_buffer() for _ in range(runs)]
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            for X, inf in zip(Xs, infos):
                pl.decompose_into(X, A, lam, inf)
            torch.cuda.synchronize(device)
            dt = time.perf_counter() - t0
            errs = np.array([Plan.read_info(inf)["rel_err"] for inf in infos])
            methods["cp_als"] = dict(mean=float(errs.mean()), std=float(errs.std()),
                                     errors=errs.tolist(), ms_per_run=dt * 1e3 / runs)
        levels.append(dict(snr=float(snr), noise=1.0 / float(snr), methods=methods))
        del Xs
    return dict(dims=dims, R=R, p=p, iters=iters, runs=runs, levels=levels)
