"""Exact pins of two parts of Algorithm 1 that inequality checks cannot hold.

Power iterations (eq. IMPsampleMatrix, Algorithm 1's power iterations).  The q
normalised power iterations compute, in exact arithmetic, an orthonormal
basis of span((T_(n) T_(n)^T)^q T_(n) Omega_n); every normalisation between
the steps is an invertible right factor and leaves the span unchanged.  With
the SVD T_(n) = U S V^T that span is span(U S^(2q+1) V^T Omega_n), which is
computed here from a library SVD, not from the loop.  On a matrix whose
singular values lie in [1, 2] this matrix is well conditioned for q <= 3, so
the oracle's basis must agree with it to principal angles of ~1e-12, while
the span for q - 1 iterations is measurably different.

Sequential scheme (Algorithm 1's projection: the tensor is replaced by its
compressed form before the next mode).  Mode n is sketched on the tensor
already compressed in modes 0..n-1: its input has dims
(l_0, .., l_{n-1}, I_n, .., I_{N-1}), its test matrix has J_n = product of
those dims except I_n rows, and its first sketch y0 equals a brute-force
sum over the partly compressed tensor built here by explicit loops from the
returned bases.
"""
import itertools

import numpy as np
import pytest

from oracle import philox, rcp


def _max_angle(A, B):
    """Sine of the largest principal angle between span(A) and span(B), of
    equal dimension: the 2-norm of (I - Qa Qa^T) Qb (accurate near zero,
    unlike the arccos of the cosines)."""
    qa = np.linalg.qr(A)[0]
    qb = np.linalg.qr(B)[0]
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))


def _well_conditioned(m, n, seed):
    rng = np.random.default_rng(seed)
    r = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = np.linspace(2.0, 1.0, r)
    return (U * s[None, :]) @ V.T


def _closed_form_span(A, Om, q):
    """U S^(2q+1) V^T Omega from the SVD of A."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    return (U * s[None, :] ** (2 * q + 1)) @ (Vt @ Om)


@pytest.mark.parametrize("q", [1, 2, 3])
@pytest.mark.parametrize("normalizer", ["qr", "lu"])
def test_power_iterations_span_closed_form(q, normalizer):
    m, J, l, seed = 40, 90, 7, 31
    A = _well_conditioned(m, J, 5)
    Om = philox.omega(seed, 0, 0, 0, J, l)
    st = rcp.range_finder(A, 0, l, q, seed, normalizer=normalizer)
    np.testing.assert_array_equal(st.omega, Om)
    want = _closed_form_span(A, Om, q)
    assert _max_angle(st.Q, want) <= 1e-8, (q, _max_angle(st.Q, want))
    # q - 1 iterations give a different subspace (the pin is not blind to q)
    prev = _closed_form_span(A, Om, q - 1)
    assert _max_angle(st.Q, prev) >= 1e-2, (q, _max_angle(st.Q, prev))
    # the first sketch is T_(n) Omega itself, q = 0 of the closed form
    np.testing.assert_allclose(st.y0, A @ Om, rtol=1e-13, atol=1e-13)


def test_power_iterations_span_through_compress():
    """The same pin on mode 1 of a 3-way tensor, through the scheme driver
    (the independent scheme sketches X itself, so the closed form applies)."""
    rng = np.random.default_rng(8)
    dims = (9, 30, 8)
    X = rng.standard_normal(dims)
    for q in (1, 2):
        comp = rcp.compress(X, 4, p=3, q=q, seed=77, scheme="independent")
        Tn = rcp.unfold(X, 1)
        Om = philox.omega(77, 1, 0, 0, Tn.shape[1], 7)
        want = _closed_form_span(Tn, Om, q)
        assert _max_angle(comp.Q[1], want) <= 1e-7, (q, _max_angle(comp.Q[1], want))
        assert _max_angle(comp.Q[1], _closed_form_span(Tn, Om, q - 1)) >= 1e-3


def _brute_partial(X, Qs, n):
    """X x_0 Q_0^T .. x_{n-1} Q_{n-1}^T by explicit loops over every index."""
    dims = X.shape
    N = X.ndim
    out_dims = tuple(Qs[m].shape[1] for m in range(n)) + dims[n:]
    out = np.zeros(out_dims)
    for o in itertools.product(*[range(d) for d in out_dims]):
        s = 0.0
        for i in itertools.product(*[range(dims[m]) for m in range(n)]):
            w = 1.0
            for m in range(n):
                w *= Qs[m][i[m], o[m]]
            s += w * X[i + o[n:]]
        out[o] = s
    return out


def _brute_sketch(T, n, Om):
    """y0[i, c] = sum over the other indices in C order of T * Omega."""
    dims = T.shape
    others = [m for m in range(T.ndim) if m != n]
    y = np.zeros((dims[n], Om.shape[1]))
    for i in range(dims[n]):
        for j, rest in enumerate(itertools.product(*[range(dims[m]) for m in others])):
            idx = list(rest)
            idx.insert(n, i)
            y[i] += T[tuple(idx)] * Om[j]
    return y


@pytest.mark.parametrize("dims,k,p", [((6, 5, 4), 2, 1), ((5, 4, 3, 3), 1, 1)])
def test_sequential_scheme_sketches_partly_compressed_tensor(dims, k, p):
    X = np.random.default_rng(sum(dims)).standard_normal(dims)
    seed = 4242
    comp = rcp.compress(X, k, p=p, q=1, seed=seed, scheme="sequential")
    N = len(dims)
    for n, st in enumerate(comp.stages):
        ls = [rcp.sketch_width(k, p, dims[m]) for m in range(n)]
        assert tuple(st.shape_in) == tuple(ls) + tuple(dims[n:]), (n, st.shape_in)
        T = _brute_partial(X, comp.Q, n)
        J = int(np.prod([d for m, d in enumerate(T.shape) if m != n]))
        l = rcp.sketch_width(k, p, dims[n])
        Om = philox.omega(seed, n, 0, 0, J, l)
        assert st.omega.shape == (J, l)
        np.testing.assert_allclose(st.y0, _brute_sketch(T, n, Om), rtol=1e-12, atol=1e-12)
    # the core is the full chain of mode products
    np.testing.assert_allclose(comp.core, _brute_partial(X, comp.Q, N), rtol=1e-12, atol=1e-12)


def test_sequential_and_independent_schemes_differ():
    """After mode 0 the two schemes sketch different tensors, so their later
    bases differ even though both capture a noise-free low-rank range."""
    X = np.random.default_rng(3).standard_normal((7, 6, 5))
    a = rcp.compress(X, 2, p=1, q=0, seed=9, scheme="sequential")
    b = rcp.compress(X, 2, p=1, q=0, seed=9, scheme="independent")
    np.testing.assert_allclose(a.Q[0], b.Q[0], rtol=1e-13, atol=1e-13)
    assert _max_angle(a.Q[1], b.Q[1]) > 1e-3
