"""Pins of the oracle's block coordinate descent (Section 3.2.2, Algorithm 3)
against what the paper and the mathematics fix:

  * each block update is the least-squares solution of the rank-one
    subproblem on the deflated residual: brute force builds the residual
    tensor explicitly (the residual update) and solves the subproblem with lstsq on the
    explicit Khatri-Rao column;
  * with one component the method is CP-ALS of rank one;
  * an orthogonally decomposable noise-free tensor is recovered exactly,
    largest component first;
  * the fit of the current model never decreases during a component's sweeps
    (each step is an exact block minimiser, the normalisation does not change
    the model), and the implicit fit equals the explicit residual;
  * the stopping rule ends each component once the fit stalls.
"""
import numpy as np
import pytest

import oracle.rcp as rcp
from paper_1703_09074_amd import synth


def _bcd_explicit(B, R, iters, init):
    """Algorithm 3 with the residual formed explicitly and every block update
    solved by lstsq on the unfolded residual (tiny tensors only)."""
    N = B.ndim
    A = [np.array(a, dtype=np.float64) for a in init]
    lam = np.zeros(R)
    for r in range(R):
        Y = B.copy()
        for s in range(r):
            t = A[0][:, s]
            for m in range(1, N):
                t = np.multiply.outer(t, A[m][:, s])
            Y = Y - lam[s] * t
        for _ in range(iters):
            for n in range(N):
                others = [A[m][:, r:r + 1] for m in range(N) if m != n]
                kr = rcp.khatri_rao(others)[:, 0]               # column of the explicit KR
                Yn = rcp.unfold(Y, n)
                # argmin_a || Y_(n) - a kr^T ||  <=>  kr a^T ~ Y_(n)^T
                sol, *_ = np.linalg.lstsq(kr[:, None], Yn.T, rcond=None)
                v = sol[0]
                nu = np.linalg.norm(v)
                A[n][:, r] = v / nu if nu > 0 else v
                if n == N - 1:
                    lam[r] = nu
    return A, lam


@pytest.mark.parametrize("shape,R", [((4, 5, 6), 3), ((3, 4, 5, 3), 2)])
def test_bcd_updates_are_explicit_residual_least_squares(shape, R):
    rng = np.random.default_rng(sum(shape))
    B = rng.standard_normal(shape)
    # a non-normalised start exercises the scalar Gram product of the update
    init = [rng.standard_normal((d, R)) * (1.0 + m) for m, d in enumerate(shape)]
    got = rcp.bcd(B, R, 4, init=[a.copy() for a in init])
    A, lam = _bcd_explicit(B, R, 4, init)
    np.testing.assert_allclose(got.lam, lam, rtol=1e-11)
    for a, b in zip(got.factors, A):
        np.testing.assert_allclose(a, b, atol=1e-11)


def test_bcd_with_one_component_is_rank_one_als():
    w = synth.low_rank((12, 10, 9), 3, 0.1, 7, dtype=np.float64)
    a = rcp.als(w.X, 1, 6)
    b = rcp.bcd(w.X, 1, 6)
    assert abs(a.rho - b.rho) < 1e-13
    np.testing.assert_allclose(a.lam, b.lam, rtol=1e-12)
    for x, y in zip(a.factors, b.factors):
        np.testing.assert_allclose(x, y, atol=1e-12)


def _orthogonal_tensor(shape, weights, seed):
    rng = np.random.default_rng(seed)
    R = len(weights)
    fac = [np.linalg.qr(rng.standard_normal((d, R)))[0] for d in shape]
    X = rcp.kruskal_full(np.asarray(weights, dtype=np.float64), fac)
    return X, fac


def test_bcd_recovers_orthogonal_components_largest_first():
    weights = [5.0, 3.0, 2.0, 1.0]
    X, fac = _orthogonal_tensor((14, 12, 10), weights, 3)
    res = rcp.bcd(X, 4, 60, tol=1e-15)
    np.testing.assert_allclose(res.lam, weights, rtol=1e-10)
    err = np.linalg.norm(rcp.kruskal_full(res.lam, res.factors) - X) / np.linalg.norm(X)
    assert err < 1e-10
    assert 1.0 - res.rho < 1e-20 + 1e-10
    for A, F in zip(res.factors, fac):
        np.testing.assert_allclose(np.abs(np.sum(A * F, axis=0)), 1.0, atol=1e-10)


def test_bcd_fit_never_decreases_within_a_component():
    w = synth.low_rank((20, 18, 16), 4, 0.2, 11, dtype=np.float64)
    iters = 12
    res = rcp.bcd(w.X, 4, iters)
    h = np.array(res.rho_history).reshape(4, iters)
    assert np.all(np.diff(h, axis=1) >= -1e-12)
    # later components add to the model: the fit after each component grows
    assert np.all(np.diff(h[:, -1]) > 0)


def test_bcd_fit_matches_explicit_residual():
    w = synth.low_rank((9, 8, 7), 3, 0.1, 13, dtype=np.float64)
    res = rcp.bcd(w.X, 3, 5)
    Xhat = rcp.kruskal_full(res.lam, res.factors)
    rho = 1.0 - np.sum((w.X - Xhat) ** 2) / np.sum(w.X ** 2)
    assert abs(rho - res.rho) < 1e-12


def test_bcd_stopping_rule():
    w = synth.low_rank((16, 15, 14), 3, 0.05, 17, dtype=np.float64)
    res = rcp.bcd(w.X, 3, 500, tol=1e-9)
    assert len(res.component_iters) == 3 and res.iters == sum(res.component_iters)
    start = 0
    for it in res.component_iters:
        assert 2 <= it < 500
        h = res.rho_history[start:start + it]
        assert abs(h[-1] - h[-2]) < 1e-9
        assert all(abs(h[j] - h[j - 1]) >= 1e-9 for j in range(1, it - 1))
        start += it


def test_rcp_bcd_full_width_equals_deterministic_bcd():
    """With l_n = I_n the bases are orthogonal and BCD is equivariant to
    them: randomized and deterministic BCD give the same model."""
    w = synth.low_rank((10, 9, 8), 3, 0.05, 19, dtype=np.float64)
    r = rcp.rcp_bcd(w.X, 3, 10, 0, 20, 0.0, 5)
    lam, A, res = rcp.cp_bcd(w.X, 3, 20)
    assert abs(r.rho - res.rho) < 1e-10
    np.testing.assert_allclose(r.lam, lam, rtol=1e-8)
