"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in the oracle (on the CPU, via monkeypatch) and checks that the pin
written for that part of the paper fails."""
import numpy as np
import pytest

import oracle.philox as philox
import oracle.rcp as rcp
from tests import test_oracle_algebra as alg
from tests import test_oracle_bcd as tbcd
from tests import test_oracle_philox as tph
from tests import test_oracle_rcp as trcp


def test_reversed_khatri_rao_order_is_caught(monkeypatch):
    def kr_reversed(mats):
        R = mats[0].shape[1]
        out = np.ones((1, R))
        for A in reversed(mats):
            out = (out[:, None, :] * A[None, :, :]).reshape(-1, R)
        return out
    monkeypatch.setattr(rcp, "khatri_rao", kr_reversed)
    with pytest.raises(AssertionError):
        alg.test_mttkrp_loops((3, 4, 5))


def test_wrong_fold_in_mode_product_is_caught(monkeypatch):
    def mp_bad(T, M, n):
        shape = list(T.shape)
        shape[n] = M.shape[0]
        return (M @ rcp.unfold(T, n)).reshape(shape)   # axis not moved back
    monkeypatch.setattr(rcp, "mode_product", mp_bad)
    with pytest.raises(AssertionError):
        alg.test_mode_product_loops((3, 4, 5))
    with pytest.raises(AssertionError):
        trcp.test_range_capture_exact_for_low_rank()


def test_missing_qr_sign_fix_is_caught(monkeypatch):
    monkeypatch.setattr(rcp, "qr_pos", lambda Y: np.linalg.qr(Y, mode="reduced")[0])
    with pytest.raises(AssertionError):
        for m, n in [(50, 7), (200, 30)]:
            alg.test_qr_pos(m, n)


def test_dropped_fit_term_is_caught(monkeypatch):
    orig = rcp.gram_hadamard

    def gh(factors, skip):
        V = orig(factors, skip)
        return V * 0.0 if skip is None else V     # drops lam^T(*A^TA)lam
    monkeypatch.setattr(rcp, "gram_hadamard", gh)
    with pytest.raises(AssertionError):
        trcp.test_fit_identity_matches_brute_force()


def test_wrong_gram_solve_is_caught(monkeypatch):
    monkeypatch.setattr(rcp, "solve_gram", lambda M, V: M @ V)
    with pytest.raises(AssertionError):
        alg.test_ls_update_equals_lstsq((3, 4, 5))


def test_wrong_philox_constant_is_caught(monkeypatch, golden_dir):
    monkeypatch.setattr(philox, "_M1", np.uint64(0xCD9E8D55))
    with pytest.raises(AssertionError):
        tph.test_known_answer_vectors(golden_dir)


def test_skewed_gaussian_transform_is_caught(monkeypatch):
    orig = philox.omega

    def om(seed, mode, batch, row0, nrows, l):
        z = orig(seed, mode, batch, row0, nrows, l)
        return z * 1.01                              # wrong radius scale
    monkeypatch.setattr(philox, "omega", om)
    with pytest.raises(AssertionError):
        tph.test_gaussian_moments_and_ks()


def test_smallest_eigenvectors_init_is_caught(monkeypatch):
    def eig_small(B, R, n):
        Bn = rcp.unfold(B, n)
        w, V = np.linalg.eigh(Bn @ Bn.T)
        return V[:, :R].copy()
    monkeypatch.setattr(rcp, "eig_init", eig_small)
    with pytest.raises(AssertionError):
        alg.test_eig_init_spans_leading_singular_subspace()


def test_lost_sign_compensation_is_caught(monkeypatch):
    def fin(lam, factors):
        A = [np.array(f, dtype=np.float64) for f in factors]
        lam = np.array(lam, dtype=np.float64)
        for n in range(len(A)):
            nu = rcp.col_norms(A[n])
            A[n] = A[n] / nu
            lam = lam * nu
        order = np.argsort(-lam, kind="stable")
        lam, A = lam[order], [a[:, order] for a in A]
        for r in range(lam.shape[0]):
            for n in range(len(A) - 1):
                i = int(np.argmax(np.abs(A[n][:, r])))
                if A[n][i, r] < 0:
                    A[n][:, r] = -A[n][:, r]       # sign not pushed to mode N
        return lam, A
    monkeypatch.setattr(rcp, "finalize", fin)
    with pytest.raises(AssertionError):
        trcp.test_finalize_order_and_signs()


def test_dropped_power_iteration_is_caught(monkeypatch):
    """range_finder running q - 1 normalised power iterations instead of q."""
    from tests import test_oracle_power_sequential as tps

    def rf_short(T, n, l, q, seed, batch=0, normalizer="qr", test="gaussian"):
        Tn = rcp.unfold(T, n)
        Om = rcp.test_matrix(test, seed, n, batch, Tn.shape[1], l)
        Y = Tn @ Om
        y0 = Y.copy()
        for _ in range(max(0, int(q) - 1)):
            Qt = rcp._normalize(Y, normalizer)
            Z = rcp._normalize(Tn.T @ Qt, normalizer)
            Y = Tn @ Z
        return rcp.ModeStage(mode=n, shape_in=T.shape, omega=Om, y0=y0, y_final=Y,
                             Q=rcp.qr_pos(Y))
    monkeypatch.setattr(rcp, "range_finder", rf_short)
    with pytest.raises(AssertionError):
        tps.test_power_iterations_span_closed_form(2, "qr")
    with pytest.raises(AssertionError):
        tps.test_power_iterations_span_through_compress()


def test_sequential_scheme_sketching_x_is_caught(monkeypatch):
    """The sequential scheme taking every sketch from X instead of the tensor
    already compressed in the earlier modes (Algorithm 1's projection)."""
    from tests import test_oracle_power_sequential as tps
    orig = rcp.compress

    def compress_bad(X, k, p=10, q=2, seed=0, batch=0, scheme="sequential", normalizer="qr",
                     test="gaussian", modes=None, p_modes=None):
        if scheme != "sequential":
            return orig(X, k, p, q, seed, batch, scheme, normalizer, test, modes, p_modes)
        X = np.asarray(X, dtype=np.float64)
        T, Qs, stages = X, [], []
        for n in range(X.ndim):
            st = rcp.range_finder(X, n, rcp.sketch_width(k, p, X.shape[n]), q, seed, batch,
                                  normalizer)
            stages.append(st)
            Qs.append(st.Q)
            T = rcp.mode_product(T, st.Q.T, n)
        return rcp.Compression(core=T, Q=Qs, stages=stages)
    monkeypatch.setattr(rcp, "compress", compress_bad)
    with pytest.raises(AssertionError):
        tps.test_sequential_scheme_sketches_partly_compressed_tensor((6, 5, 4), 2, 1)
    with pytest.raises(AssertionError):
        tps.test_sequential_and_independent_schemes_differ()


def test_missing_column_normalisation_is_caught(monkeypatch):
    """ALS and the renormalisation leaving the factor columns unscaled
    (Algorithm 2's normalisations and final renormalisation)."""
    monkeypatch.setattr(rcp, "_scale_columns", lambda A, nu: A)
    with pytest.raises(AssertionError):
        trcp.test_exact_recovery_noise_free()


def test_wrong_fit_sign_is_caught(monkeypatch):
    """The model term of the Section 3.3 fit entering with the wrong sign."""
    orig = rcp.gram_hadamard

    def gh(factors, skip):
        V = orig(factors, skip)
        return -V if skip is None else V
    monkeypatch.setattr(rcp, "gram_hadamard", gh)
    with pytest.raises(AssertionError):
        trcp.test_fit_identity_matches_brute_force()


def _bcd_variant(drop_deflation=False, wrong_vector=False):
    """A copy of the oracle's bcd with one planted mistake."""
    def bcd(B, R, max_iters, tol=0.0, normX2=None, init=None):
        B = np.asarray(B, dtype=np.float64)
        N = B.ndim
        nx = float(np.dot(B.ravel(), B.ravel())) if normX2 is None else normX2
        A = ([np.zeros((B.shape[0], R))] + [rcp.eig_init(B, R, n) for n in range(1, N)]
             if init is None else [np.array(a, dtype=np.float64) for a in init])
        lam = np.zeros(R)
        hist, comp_iters = [], []
        rho = 0.0
        for r in range(R):
            it = 0
            for it in range(1, int(max_iters) + 1):
                for n in range(N):
                    v = rcp.mttkrp(B, [A[m][:, r:r + 1] for m in range(N)], n)[:, 0]
                    if not drop_deflation:
                        for s in range(r):
                            w = np.prod([A[m][:, s] @ A[m][:, r] for m in range(N) if m != n])
                            v = v - lam[s] * w * A[n][:, r if wrong_vector else s]
                    d = np.prod([A[m][:, r] @ A[m][:, r] for m in range(N) if m != n])
                    v = v / d
                    nu = float(np.linalg.norm(v))
                    A[n][:, r] = v / nu if nu > 0 else v
                    if n == N - 1:
                        lam[r] = nu
                rho = rcp.bcd_fit(B, A, lam, r, nx)
                hist.append(rho)
            comp_iters.append(it)
        return rcp.BCDResult(factors=A, lam=lam, rho=rho, iters=sum(comp_iters),
                             component_iters=comp_iters, rho_history=hist)
    return bcd


def test_bcd_without_deflation_is_caught(monkeypatch):
    monkeypatch.setattr(rcp, "bcd", _bcd_variant(drop_deflation=True))
    with pytest.raises(AssertionError):
        tbcd.test_bcd_updates_are_explicit_residual_least_squares((4, 5, 6), 3)
    with pytest.raises(AssertionError):
        tbcd.test_bcd_fit_never_decreases_within_a_component()


def test_bcd_deflating_with_the_wrong_vector_is_caught(monkeypatch):
    monkeypatch.setattr(rcp, "bcd", _bcd_variant(wrong_vector=True))
    with pytest.raises(AssertionError):
        tbcd.test_bcd_updates_are_explicit_residual_least_squares((4, 5, 6), 3)

