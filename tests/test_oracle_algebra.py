"""Brute-force pins of the oracle's tensor algebra (Section 2.1 notation,
Definition 1 n-mode product, the matricized CP model and the Khatri-Rao
pseudo-inverse of Section 3.2.1, and the QR / LU normalisers of
Algorithm 1).  Expected values come from explicit index loops written here,
never from the oracle's own formulas."""
import itertools

import numpy as np
import pytest

from oracle import philox, rcp

SHAPES = [(3, 4, 5), (4, 5, 6, 3), (2, 3, 2, 2, 3)]


def _rand(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def _col_index(shape, n, idx):
    """C-order position of idx among the elements with the same mode-n index."""
    j = 0
    for m, (s, i) in enumerate(zip(shape, idx)):
        if m == n:
            continue
        j = j * s + i
    return j


@pytest.mark.parametrize("shape", SHAPES)
def test_unfold_and_fold(shape):
    T = _rand(shape)
    for n in range(len(shape)):
        U = rcp.unfold(T, n)
        for idx in itertools.product(*[range(s) for s in shape]):
            assert U[idx[n], _col_index(shape, n, idx)] == T[idx]
        np.testing.assert_array_equal(rcp.fold(U, n, shape), T)


@pytest.mark.parametrize("shape", SHAPES)
def test_mode_product_loops(shape):
    T = _rand(shape, 1)
    for n in range(len(shape)):
        M = _rand((2, shape[n]), 2 + n)
        got = rcp.mode_product(T, M, n)
        want_shape = list(shape)
        want_shape[n] = 2
        want = np.zeros(want_shape)
        for idx in itertools.product(*[range(s) for s in shape]):
            for j in range(2):
                out = list(idx)
                out[n] = j
                want[tuple(out)] += M[j, idx[n]] * T[idx]
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_khatri_rao_loops():
    A, B, C = _rand((3, 4), 3), _rand((2, 4), 4), _rand((5, 4), 5)
    K = rcp.khatri_rao([A, B, C])
    assert K.shape == (30, 4)
    for i in range(3):
        for j in range(2):
            for k in range(5):
                np.testing.assert_allclose(K[(i * 2 + j) * 5 + k], A[i] * B[j] * C[k], rtol=1e-14)


@pytest.mark.parametrize("shape", SHAPES)
def test_mttkrp_loops(shape):
    R = 3
    T = _rand(shape, 6)
    F = [_rand((s, R), 10 + m) for m, s in enumerate(shape)]
    for n in range(len(shape)):
        got = rcp.mttkrp(T, F, n)
        want = np.zeros((shape[n], R))
        for idx in itertools.product(*[range(s) for s in shape]):
            for r in range(R):
                w = T[idx]
                for m in range(len(shape)):
                    if m != n:
                        w *= F[m][idx[m], r]
                want[idx[n], r] += w
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
def test_kruskal_full_loops(shape):
    R = 2
    F = [_rand((s, R), 20 + m) for m, s in enumerate(shape)]
    lam = np.array([1.5, -0.25])
    X = rcp.kruskal_full(lam, F)
    for idx in itertools.product(*[range(s) for s in shape]):
        want = 0.0
        for r in range(R):
            t = lam[r]
            for m in range(len(shape)):
                t *= F[m][idx[m], r]
            want += t
        assert abs(X[idx] - want) < 1e-13


@pytest.mark.parametrize("shape", SHAPES)
def test_sketch_row_order(shape):
    """Y = T_(n) Omega with Omega's row j = C-order position over the other
    modes, checked by an index loop."""
    T = _rand(shape, 30)
    for n in range(len(shape)):
        J = int(np.prod(shape)) // shape[n]
        Om = philox.omega(9, n, 0, 0, J, 3)
        got = rcp.unfold(T, n) @ Om
        want = np.zeros((shape[n], 3))
        for idx in itertools.product(*[range(s) for s in shape]):
            want[idx[n]] += T[idx] * Om[_col_index(shape, n, idx)]
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m,n", [(50, 7), (7, 7), (200, 30), (5, 9)])
def test_qr_pos(m, n):
    Y = _rand((m, n), m * n)
    Q = rcp.qr_pos(Y)
    k = min(m, n)
    assert Q.shape == (m, k)
    np.testing.assert_allclose(Q.T @ Q, np.eye(k), atol=1e-14)
    R = Q.T @ Y
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(np.tril(R, -1), 0.0, atol=1e-12)
    np.testing.assert_allclose(Q @ R, Y, atol=1e-12)


def test_qr_pos_rank_deficient_still_orthonormal():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((60, 4)) @ rng.standard_normal((4, 10))
    Q = rcp.qr_pos(Y)
    np.testing.assert_allclose(Q.T @ Q, np.eye(10), atol=1e-13)
    np.testing.assert_allclose(Q @ (Q.T @ Y), Y, atol=1e-11)


def test_lu_factor_and_span():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((80, 12))
    L = rcp.lu_factor_l(Y)
    # permuted unit lower trapezoid: one row per column carries the unit pivot
    # and, in pivot order, rows are zero beyond their step
    U = np.linalg.lstsq(L, Y, rcond=None)[0]
    np.testing.assert_allclose(L @ U, Y, atol=1e-12)
    np.testing.assert_allclose(np.tril(U, -1), 0.0, atol=1e-12)
    assert np.max(np.abs(L)) <= 1.0 + 1e-15        # partial pivoting bound
    # same column space as the QR basis (principal angles ~ 0)
    Q1 = rcp.qr_pos(Y)
    Q2 = rcp.qr_pos(L)
    s = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    assert np.min(s) > 1.0 - 1e-12


def test_kr_pseudo_inverse_identity():
    """(A (.) B)^+ = (A^T A * B^T B)^+ (A (.) B)^T (Definition 2), against a
    library pseudo-inverse of the explicit Khatri-Rao product."""
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((6, 4)), rng.standard_normal((5, 4))
    K = rcp.khatri_rao([A, B])
    lhs = np.linalg.pinv(K)
    V = rcp.gram_hadamard([A, B], skip=None)
    rhs = np.linalg.pinv(V) @ K.T
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("shape", SHAPES)
def test_ls_update_equals_lstsq(shape):
    """Each ALS update solves min ||T_(n) - A KR^T|| (eqs. Astar ff.); compare
    the normal-equation form with a library least-squares solve on the
    explicit Khatri-Rao matrix."""
    R = 2
    T = _rand(shape, 40)
    F = [_rand((s, R), 50 + m) for m, s in enumerate(shape)]
    for n in range(len(shape)):
        got = rcp.solve_gram(rcp.mttkrp(T, F, n), rcp.gram_hadamard(F, skip=n))
        K = np.ones((1, R))
        for m in range(len(shape)):
            if m != n:
                K = np.einsum("jr,kr->jkr", K, F[m]).reshape(-1, R)
        want = np.linalg.lstsq(K, rcp.unfold(T, n).T, rcond=None)[0].T
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_solve_gram_singular_falls_back_to_pinv():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((5, 3))
    V = A.T @ A
    V[:, 2] = V[:, 1]
    V[2, :] = V[1, :]          # exactly singular, not positive definite
    M = rng.standard_normal((4, 3))
    got = rcp.solve_gram(M, V)
    np.testing.assert_allclose(got, M @ np.linalg.pinv(V), atol=1e-10)


def test_eig_init_spans_leading_singular_subspace():
    """Algorithm 2's initialisation: the initial factor of mode n spans the leading R
    left singular vectors of B_(n) (checked against a library SVD on a core
    with a known, well separated spectrum), with the sign rule applied."""
    rng = np.random.default_rng(31)
    U, _ = np.linalg.qr(rng.standard_normal((9, 9)))
    V, _ = np.linalg.qr(rng.standard_normal((40, 9)))
    s = 2.0 ** -np.arange(9)
    B = ((U * s) @ V.T).reshape(9, 5, 8)            # mode 0 has spectrum s
    Bp = np.moveaxis(B, 0, 1).copy()                # same core, as mode 1
    for T, n in ((B, 0), (Bp, 1)):
        A = rcp.eig_init(T, 3, n)
        Ul = np.linalg.svd(rcp.unfold(T, n))[0][:, :3]
        for r in range(3):
            assert abs(abs(Ul[:, r] @ A[:, r]) - 1.0) < 1e-10
            i = np.argmax(np.abs(A[:, r]))
            assert A[i, r] > 0
