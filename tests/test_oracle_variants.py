"""Pins of the oracle's test-matrix and parameter variants (the note on
quasi-random numbers in Section 3.1, Algorithm 1's rand and the
remarks after Algorithm 1: uniform test matrices, randomly selected
columns, a chosen subset of modes and per-mode oversampling)."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import oracle.philox as philox
import oracle.rcp as rcp
from paper_1703_09074_amd import synth


def test_halton_matches_published_first_points(golden_dir):
    for line in open(f"{golden_dir}/halton_first_points.txt"):
        if line.startswith("#") or not line.strip():
            continue
        base, vals = line.split(":")
        b = int(base)
        want = [float(Fraction(v)) for v in vals.split()]
        c = philox.PRIMES.index(b)
        got = philox.omega_halton(0, len(want), c + 1)[:, c]
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("b,m", [(2, 6), (3, 4), (5, 3)])
def test_halton_stratifies(b, m):
    """The radical inverse maps 1..b^m - 1 one to one onto the grid
    k / b^m, k = 1..b^m - 1: rows 0..b^m - 2 (the points of 1..b^m - 1) fall
    one into each cell [k / b^m, (k + 1) / b^m), k >= 1."""
    c = philox.PRIMES.index(b)
    n = b ** m
    pts = philox.omega_halton(0, n - 1, c + 1)[:, c]
    cells = np.floor(pts * n).astype(int)
    assert sorted(cells.tolist()) == list(range(1, n))


def test_uniform_test_matrix_distribution_and_words():
    u = philox.omega_uniform(7, 1, 0, 1000, 200_000, 6)
    assert u.shape == (200_000, 6)
    assert np.all(u > 0.0) and np.all(u <= 1.0)
    for c in range(6):
        assert abs(u[:, c].mean() - 0.5) < 5e-3
        assert abs(u[:, c].var() - 1.0 / 12.0) < 2e-3
        assert stats.kstest(u[:, c], "uniform").pvalue > 1e-4
    # the same counter words as the Gaussian matrix: Box-Muller of a group's
    # uniforms gives that group's Gaussian entries
    g = philox.omega(7, 1, 0, 1000, 5, 4)
    uu = philox.omega_uniform(7, 1, 0, 1000, 5, 4)
    np.testing.assert_allclose(g[:, 0], np.sqrt(-2 * np.log(uu[:, 0])) * np.cos(2 * np.pi * uu[:, 1]),
                               rtol=1e-15)


@pytest.mark.parametrize("J,l", [(1000, 10), (37, 37), (5, 1), (2 ** 33 + 7, 12)])
def test_column_selection_distinct_sorted_in_range(J, l):
    sel = philox.select_columns(11, 2, 0, J, l)
    assert len(sel) == l and len(set(sel.tolist())) == l
    assert np.all(np.diff(sel) > 0) and sel[0] >= 0 and sel[-1] < J
    if J == l:
        np.testing.assert_array_equal(sel, np.arange(J))


def test_column_selection_is_uniform():
    J, l, runs = 40, 6, 4000
    counts = np.zeros(J)
    for s in range(runs):
        counts[philox.select_columns(s, 0, 0, J, l)] += 1
    expect = runs * l / J
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert stats.chi2.sf(chi2, J - 1) > 1e-4, chi2


@pytest.mark.parametrize("test", ["uniform", "halton", "columns"])
def test_range_capture_exact_with_each_test_matrix(test):
    w = synth.low_rank((30, 25, 20), 4, 0.0, 21, dtype=np.float64)
    comp = rcp.compress(w.X, 4, 4, 1, seed=3, test=test)
    P = comp.core
    for n, Q in enumerate(comp.Q):
        P = rcp.mode_product(P, Q, n)
    assert np.linalg.norm(P - w.X) / np.linalg.norm(w.X) < 1e-11


def test_columns_sketch_is_the_selected_columns():
    T = np.random.default_rng(2).standard_normal((12, 9, 7))
    st = rcp.range_finder(T, 1, 5, 0, 17, test="columns")
    sel = philox.select_columns(17, 1, 0, 12 * 7, 5)
    np.testing.assert_array_equal(st.y0, rcp.unfold(T, 1)[:, sel])


def test_mode_subset_keeps_identity_bases():
    w = synth.low_rank((30, 8, 20), 3, 0.0, 23, dtype=np.float64)
    comp = rcp.compress(w.X, 3, 4, 1, seed=5, modes=[0, 2])
    assert comp.core.shape == (7, 8, 7)
    np.testing.assert_array_equal(comp.Q[1], np.eye(8))
    P = comp.core
    for n, Q in enumerate(comp.Q):
        P = rcp.mode_product(P, Q, n)
    assert np.linalg.norm(P - w.X) / np.linalg.norm(w.X) < 1e-11
    # no mode compressed: the core is X and rCP-ALS is deterministic CP-ALS
    none = rcp.compress(w.X, 3, 4, 1, seed=5, modes=[])
    np.testing.assert_array_equal(none.core, w.X)
    r = rcp.rcp_als(w.X, 3, 4, 1, 15, seed=5, modes=[])
    lam, A, ref = rcp.cp_als(w.X, 3, 15)
    assert abs(r.rho - ref.rho) < 1e-12


def test_per_mode_oversampling_sets_sketch_widths():
    w = synth.low_rank((30, 25, 20), 3, 0.01, 25, dtype=np.float64)
    comp = rcp.compress(w.X, 3, 10, 1, seed=7, p_modes=[2, 9, 30])
    assert comp.core.shape == (5, 12, 20)
    assert [q.shape[1] for q in comp.Q] == [5, 12, 20]
