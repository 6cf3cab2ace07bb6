"""End-to-end pins of the oracle's randomized CP (Algorithms 1 and 2,
Theorem 1, Section 3.3 fit, eq. qbs back-projection).  Expected values come
from what the mathematics fixes: exact recovery of noise-free low-rank
tensors, orthonormality, invariances, brute-force evaluation, the paper's
error bound and the paper's printed numbers."""
import os

import numpy as np
import pytest

from oracle import evaluate, philox, rcp
from paper_1703_09074_amd import synth


def _exact(dims, R, seed, kind="gaussian"):
    return synth.low_rank(dims, R, 0.0, seed, kind=kind, dtype=np.float64)


def test_range_capture_exact_for_low_rank():
    """Noise-free rank-R tensor, l >= R: the bases capture X exactly."""
    for dims, R in [((40, 30, 20), 4), ((12, 10, 9, 8), 3)]:
        w = _exact(dims, R, 1)
        for scheme in ("sequential", "independent"):
            comp = rcp.compress(w.X, R, p=3, q=1, seed=2, scheme=scheme)
            for Q in comp.Q:
                np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-13)
            P = comp.core
            for n, Q in enumerate(comp.Q):
                P = rcp.mode_product(P, Q, n)
            err = np.linalg.norm(P - w.X) / np.linalg.norm(w.X)
            assert err < 1e-12, (scheme, err)


def test_matrix_special_case_is_halko_range_finder():
    """For N = 2 and q = 0 mode 0 of Algorithm 1 is the randomized range
    finder of Section 2.3: Q spans A Omega, and for rank(A) <= l it spans
    range(A) (projection error ~ 0)."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((70, 6)) @ rng.standard_normal((6, 50))
    comp = rcp.compress(A, 6, p=4, q=0, seed=4)
    Q = comp.Q[0]
    err = np.linalg.norm(A - Q @ (Q.T @ A)) / np.linalg.norm(A)
    assert err < 1e-13
    # span(Q) contains the sketch A Omega, Omega the mode-0 test matrix
    Om = philox.omega(4, 0, 0, 0, 50, 10)
    Y = A @ Om
    assert Q.shape == (70, 10)
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) / np.linalg.norm(Y) < 1e-13
    # full-rank case: span(Q) equals span(A Omega) exactly
    B = rng.standard_normal((70, 50))
    QB = rcp.compress(B, 6, p=4, q=0, seed=4).Q[0]
    YB = B @ Om
    s = np.linalg.svd(QB.T @ np.linalg.qr(YB)[0], compute_uv=False)
    assert np.min(s) > 1.0 - 1e-12


def test_power_iterations_increase_captured_energy():
    """q normalised power iterations (eq. IMPsampleMatrix) sharpen the basis
    on a slowly decaying spectrum: captured energy is non-decreasing in q."""
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(rng.standard_normal((120, 120)))
    V, _ = np.linalg.qr(rng.standard_normal((300, 120)))
    A = (U * (1.0 / np.arange(1, 121) ** 0.5)) @ V.T
    prev = -1.0
    for q in range(4):
        Q = rcp.compress(A, 8, p=2, q=q, seed=1).Q[0]
        cap = np.linalg.norm(Q.T @ A) ** 2
        assert cap >= prev - 1e-12
        prev = cap


def test_lu_and_qr_normalisers_give_same_basis():
    """Algorithm 1 normalises with pivoted LU (Remark 2); the QR reading
    spans the same subspace in exact arithmetic."""
    w = synth.low_rank((30, 25, 20), 4, 0.05, 5, dtype=np.float64)
    a = rcp.compress(w.X, 4, p=4, q=2, seed=6, normalizer="qr", scheme="independent")
    b = rcp.compress(w.X, 4, p=4, q=2, seed=6, normalizer="lu", scheme="independent")
    for Qa, Qb in zip(a.Q, b.Q):
        s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
        assert np.min(s) > 1.0 - 1e-8


def test_full_width_bases_reduce_to_deterministic_cp_als():
    """With l_n = I_n every Q_n is square orthogonal; ALS is equivariant under
    an orthogonal change of basis per mode (including the eigenvector
    initialisation up to sign), so rCP equals deterministic CP-ALS."""
    w = synth.low_rank((9, 8, 7), 3, 0.2, 11, dtype=np.float64)
    r = rcp.rcp_als(w.X, 3, p=20, q=1, max_iters=30, seed=12)
    for Q, I in zip(r.compression.Q, w.X.shape):
        assert Q.shape == (I, I)
    lam, A, res = rcp.cp_als(w.X, 3, max_iters=30)
    np.testing.assert_allclose(r.lam, lam, rtol=1e-8)
    for a, b in zip(r.factors, A):
        np.testing.assert_allclose(a, b, atol=1e-7)
    assert abs(r.rho - res.rho) < 1e-12


def test_exact_recovery_noise_free():
    """Noise-free rank-5 100^3 tensor (the rcp100 shape), k = R = 5, p = 10,
    q = 2: relative error < 1e-10 and congruence to the true factors
    > 1 - 1e-8."""
    w = _exact((100, 100, 100), 5, 20170327)
    r = rcp.rcp_als(w.X, 5, p=10, q=2, max_iters=150, tol=0.0, seed=1000)
    rel = evaluate.relative_error(w.X, r.lam, r.factors)
    assert rel < 1e-10, rel
    mean, mn, _ = evaluate.congruence(r.factors, w.factors)
    assert mn > 1.0 - 1e-8


def test_fit_identity_matches_brute_force():
    """Section 3.3 fit via the projection identity == 1 - ||X - Xhat||^2/||X||^2
    from the dense reconstruction."""
    for dims, R, scheme in [((12, 11, 10), 3, "sequential"), ((8, 7, 6, 5), 2, "independent")]:
        w = synth.low_rank(dims, R, 0.3, 13, dtype=np.float64)
        r = rcp.rcp_als(w.X, R, p=2, q=1, max_iters=7, seed=14, scheme=scheme)
        Xh = rcp.kruskal_full(r.lam, r.factors)
        direct = 1.0 - np.sum((w.X - Xh) ** 2) / np.sum(w.X ** 2)
        assert abs(direct - r.rho) < 1e-12
        assert abs(evaluate.relative_error(w.X, r.lam, r.factors) - r.rel_err) < 1e-9


def test_als_residual_monotone():
    """Every least-squares update is exact, so the core residual cannot grow
    from sweep to sweep (rho non-decreasing)."""
    w = synth.low_rank((15, 14, 13), 4, 0.5, 15, dtype=np.float64)
    res = rcp.als(w.X, 4, max_iters=25)
    h = np.array(res.rho_history)
    assert np.all(np.diff(h) >= -1e-13)


def test_back_projection_preserves_norms():
    w = synth.low_rank((40, 35, 30), 4, 0.05, 16, dtype=np.float64)
    comp = rcp.compress(w.X, 4, p=5, q=1, seed=17)
    res = rcp.als(comp.core, 4, 10)
    for Q, At in zip(comp.Q, res.factors):
        np.testing.assert_allclose(np.linalg.norm(Q @ At, axis=0), np.linalg.norm(At, axis=0), rtol=1e-13)


def test_finalize_order_and_signs():
    rng = np.random.default_rng(18)
    F = [rng.standard_normal((6, 3)) for _ in range(3)]
    lam0 = np.array([0.5, 2.0, 1.0])
    lam, A = rcp.finalize(lam0, F)
    assert np.all(np.diff(lam) <= 0)
    for n in range(2):
        for r in range(3):
            i = np.argmax(np.abs(A[n][:, r]))
            assert A[n][i, r] > 0
    for a in A:
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 1.0, rtol=1e-14)
    # the model is unchanged
    np.testing.assert_allclose(rcp.kruskal_full(lam, A), rcp.kruskal_full(lam0, F), atol=1e-12)


def test_stopping_rule():
    w = synth.low_rank((20, 18, 16), 3, 0.1, 19, dtype=np.float64)
    fixed = rcp.als(w.X, 3, max_iters=12, tol=0.0)
    assert fixed.iters == 12 and len(fixed.rho_history) == 12
    early = rcp.als(w.X, 3, max_iters=500, tol=1e-6)
    assert early.iters < 500
    h = early.rho_history
    assert abs(h[-1] - h[-2]) < 1e-6
    assert all(abs(h[i] - h[i - 1]) >= 1e-6 for i in range(1, len(h) - 1))


@pytest.mark.parametrize("order", [3, 4])
def test_theorem1_bound(order):
    """Theorem 1 (eq. theorem): mean over seeds of
    ||X - X x_1 Q_1Q_1^T ... x_N Q_NQ_N^T|| is below
    sqrt(1 + k/(p-1)) sqrt(sum_n sum_{j>k} sigma_nj^2) for Gaussian test
    matrices, q = 0, p = 2 (the paper's own check uses 50^3 / 50^4, rank 25)."""
    dims = (20,) * order if order == 4 else (50, 50, 50)
    R = 12 if order == 4 else 25
    w = synth.low_rank(dims, R, 0.0, 21, dtype=np.float64)
    X = w.X
    sig = [np.linalg.svd(rcp.unfold(X, n), compute_uv=False) for n in range(order)]
    p = 2
    for k in ([4, 8] if order == 4 else [5, 10, 20]):
        tail = np.sqrt(sum(np.sum(s[k:] ** 2) for s in sig))
        bound = np.sqrt(1.0 + k / (p - 1.0)) * tail
        errs = []
        for s in range(8):
            comp = rcp.compress(X, k, p=p, q=0, seed=100 + s, scheme="independent")
            P = comp.core
            for n, Q in enumerate(comp.Q):
                P = rcp.mode_product(P, Q, n)
            errs.append(np.linalg.norm(X - P))
        assert np.mean(errs) <= bound, (k, np.mean(errs), bound)


def test_compression_ratios_match_paper(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "compression_ratios.txt"))
    for I, J, K, R, c_svd, c_cp in rows:
        a, b = evaluate.compression_ratios(int(I), int(J), int(K), int(R))
        assert abs(a - c_svd) < 0.006 and abs(b - c_cp) < 0.006


def test_power_iterations_help_under_noise():
    """Section 4.1: without power iterations the randomized result is poor at
    high noise; q = 2 comes close to deterministic CP-ALS."""
    w = synth.low_rank((60, 60, 60), 10, 0.4, 22)
    lam, A, res = rcp.cp_als(w.X, 10, max_iters=30)
    det = evaluate.relative_error(w.X, lam, A)
    e = {}
    for q in (0, 2):
        r = rcp.rcp_als(w.X, 10, p=10, q=q, max_iters=30, seed=23)
        e[q] = evaluate.relative_error(w.X, r.lam, r.factors)
    assert e[0] > 1.2 * e[2]
    assert e[2] < det * 1.01


def test_congruence_invariances():
    rng = np.random.default_rng(24)
    F = [rng.standard_normal((7, 4)) for _ in range(3)]
    perm = [2, 0, 3, 1]
    G = [f[:, perm] * np.array([1.0, -2.0, 0.5, 3.0]) for f in F]
    mean, mn, p = evaluate.congruence(F, G)
    assert abs(mean - 1.0) < 1e-14 and abs(mn - 1.0) < 1e-14
    assert list(p) == [1, 3, 0, 2]


def test_warm_start_continues_the_sweeps():
    """CP-ALS started from given factors (the warm start / resume of the
    boundary): a sweep updates mode 1 first from the factors of modes 2..N,
    so continuing from the factors after j sweeps reproduces sweeps j+1..
    of the uninterrupted run exactly, and starting from the true factors of
    a noise-free low-rank tensor fits it in one sweep."""
    w = synth.low_rank((14, 12, 11), 3, 0.2, 25, dtype=np.float64)
    full = rcp.als(w.X, 3, max_iters=7)
    head = rcp.als(w.X, 3, max_iters=3)
    tail = rcp.als(w.X, 3, max_iters=4, init=head.factors)
    np.testing.assert_allclose(tail.rho_history, full.rho_history[3:], rtol=0, atol=1e-13)
    np.testing.assert_allclose(tail.lam, full.lam, rtol=1e-11)
    for a, b in zip(tail.factors, full.factors):
        np.testing.assert_allclose(a, b, atol=1e-10)
    e = _exact((10, 9, 8), 3, 26)
    true = [f / np.linalg.norm(f, axis=0) for f in e.factors]
    one = rcp.als(e.X, 3, max_iters=1, init=true)
    assert abs(one.rho - 1.0) < 1e-13, one.rho
