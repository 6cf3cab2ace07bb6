"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake in the oracle (on the CPU, via monkeypatch) and checks that the pin
written for that part of the paper fails."""
import numpy as np
import pytest

import oracle.philox as philox
import oracle.rcp as rcp
from tests import test_oracle_algebra as alg
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
