"""Randomized CP decomposition, float64 reference (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows the paper step by step:

  Section 3.1 / Algorithm 1   randomized tensor compression: per mode a
                              sketch Y = T_(n) Omega, q normalized power
                              iterations, an orthonormal basis Q_n = qr(Y),
                              then the projection T <- T x_n Q_n^T.
  Section 3.2.1 / Algorithm 2 CP-ALS on the compressed tensor, with the
                              Khatri-Rao pseudo-inverse (Definition 2) and
                              column normalisation, eigenvector
                              initialisation, back-projection A_n = Q_n Ã_n
                              (eq. qbs) and a final renormalisation.
  Section 3.2.2 / Algorithm 3 block coordinate descent on the compressed
                              tensor: rank-one components found one after
                              another on the implicitly deflated residual.
  Section 3.3                 the fit rho used for the stopping rule.

Conventions (readings where the paper is silent; all listed with reasons in
the design notes):
  * tensors are C-order; the mode-n unfolding is
    ``moveaxis(T, n, 0).reshape(I_n, -1)`` so its column index is the C-order
    position over the other modes; Khatri-Rao products use the matching
    ("first factor slowest") row order;
  * l_n = min(k + p, I_n) columns per mode; the core is l_1 x ... x l_N;
  * every QR is Householder with the signs fixed so that diag(R) > 0;
  * the default normaliser inside the power iterations is QR; the paper's
    pivoted LU (the normalisers of Algorithm 1's power iterations) is available as ``normalizer="lu"``;
  * "norm" in Algorithm 2's normalisations is the column 2-norm; lambda comes
    from the last mode;
  * fit: rho = 1 - ||X - Xhat||^2 / ||X||^2 (the Section 3.3 formula); the
    sweep loop stops after sweep j >= 2 once |rho_j - rho_{j-1}| < tol, and
    runs exactly ``max_iters`` sweeps when tol == 0;
  * output: components sorted by lambda (descending); each column of modes
    1..N-1 has its largest-magnitude entry positive (first index on ties),
    the compensating sign goes to mode N.

Parity: every function here is pinned by the oracle self-tests (brute-force
loops on tiny tensors, exact recovery of noise-free low-rank tensors,
orthonormality, the Halko matrix special case, equivalence with
deterministic CP-ALS when l_n = I_n, the Khatri-Rao pseudo-inverse identity,
monotone ALS residuals and the fit identity).  The q power iterations are
pinned exactly: span(Q_n) equals span(U S^(2q+1) V^T Omega_n) from an SVD
of T_(n) (eq. IMPsampleMatrix) and differs from the q - 1 span.  The
sequential scheme is pinned by a brute-force loop: mode n sketches the tensor
compressed in modes < n, with J_n rows of Omega_n (Algorithm 1: the tensor is replaced by its
projection after each mode).
The warm start of ``als`` is pinned by continuing an interrupted run.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg

from . import philox


# ---------------------------------------------------------------------------
# Tensor algebra (Section 2.1 notation; Definition 1 of the n-mode product)

def unfold(T: np.ndarray, n: int) -> np.ndarray:
    """Mode-n unfolding T_(n): I_n x prod_{m != n} I_m, C-order columns."""
    return np.moveaxis(T, n, 0).reshape(T.shape[n], -1)


def fold(M: np.ndarray, n: int, shape: Sequence[int]) -> np.ndarray:
    """Inverse of ``unfold`` for a tensor of the given shape."""
    shape = list(shape)
    lead = [shape[n]] + shape[:n] + shape[n + 1:]
    return np.moveaxis(M.reshape(lead), 0, n)


def mode_product(T: np.ndarray, M: np.ndarray, n: int) -> np.ndarray:
    """T x_n M (Definition 1): every mode-n fibre is multiplied by M.

    M has shape (J, I_n); the result has mode n of size J and satisfies
    (T x_n M)_(n) = M T_(n).
    """
    shape = list(T.shape)
    out = M @ unfold(T, n)
    shape[n] = M.shape[0]
    return fold(out, n, shape)


def khatri_rao(mats: Sequence[np.ndarray]) -> np.ndarray:
    """Column-wise Kronecker product of matrices with R columns each.

    Row index runs in C order over the matrices (first matrix slowest), which
    matches the column order of ``unfold``.  The paper writes the reversed
    order (C (.) B for the mode-1 unfolding), which goes with the
    column-major unfolding of the Tensor Toolbox.
    """
    R = mats[0].shape[1]
    out = np.ones((1, R))
    for A in mats:
        out = (out[:, None, :] * A[None, :, :]).reshape(-1, R)
    return out


def kruskal_full(lam: np.ndarray, factors: Sequence[np.ndarray]) -> np.ndarray:
    """Dense tensor sum_r lam_r a1_r o ... o aN_r (eq. CPlamb2)."""
    shape = [A.shape[0] for A in factors]
    M = (factors[0] * lam[None, :]) @ khatri_rao(factors[1:]).T
    return M.reshape(shape)


# ---------------------------------------------------------------------------
# Orthonormalisation (Algorithm 1: the power iterations' normalisers and the
# final QR)

def qr_pos(Y: np.ndarray) -> np.ndarray:
    """Economic Householder QR with diag(R) >= 0; returns Q (m x min(m, n))."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def lu_factor_l(Y: np.ndarray) -> np.ndarray:
    """The permuted unit-lower factor of a partially pivoted LU, i.e. the
    first output of ``[L, U] = lu(Y)`` in Algorithm 1's power iterations (Remark 2:
    pivoted LU for the normalised power iterations)."""
    PL, _ = scipy.linalg.lu(Y, permute_l=True)
    return PL


def _normalize(Y: np.ndarray, normalizer: str) -> np.ndarray:
    if normalizer == "qr":
        return qr_pos(Y)
    if normalizer == "lu":
        return lu_factor_l(Y)
    raise ValueError(normalizer)


# ---------------------------------------------------------------------------
# Randomized range finder and compression (Section 3.1, Algorithm 1)

def sketch_width(k: int, p: int, I: int) -> int:
    """l_n = min(k + p, I_n) (Algorithm 1's oversampled width, clamped to the mode size)."""
    return min(int(k) + int(p), int(I))


@dataclass
class ModeStage:
    """Intermediates of one mode of Algorithm 1."""
    mode: int
    shape_in: tuple
    omega: np.ndarray       # J x l
    y0: np.ndarray          # I_n x l, the first sketch T_(n) Omega
    y_final: np.ndarray     # I_n x l, the sketch after q power iterations
    Q: np.ndarray           # I_n x l


TEST_MATRICES = ("gaussian", "uniform", "halton", "columns")


def test_matrix(kind: str, seed: int, n: int, batch: int, J: int, l: int) -> np.ndarray:
    """The J x l test matrix Omega of mode n (Algorithm 1's test-matrix draw): Gaussian
    (Section 3.1), uniform (the rand of that draw and the remark after
    Algorithm 1), quasi-random Halton (the note in Section 3.1), or the
    selection of l random columns (the remark after Algorithm 1), as the
    0/1 matrix picking them."""
    if kind == "gaussian":
        return philox.omega(seed, n, batch, 0, J, l)
    if kind == "uniform":
        return philox.omega_uniform(seed, n, batch, 0, J, l)
    if kind == "halton":
        return philox.omega_halton(0, J, l)
    if kind == "columns":
        sel = philox.select_columns(seed, n, batch, J, l)
        Om = np.zeros((J, l))
        Om[sel, np.arange(l)] = 1.0
        return Om
    raise ValueError(kind)


def range_finder(T: np.ndarray, n: int, l: int, q: int, seed: int,
                 batch: int = 0, normalizer: str = "qr", test: str = "gaussian"):
    """Basis Q_n of the mode-n range of T (Algorithm 1, from the sketch to the final QR).

    Omega is the J x l test matrix of mode n (Gaussian unless ``test`` says
    otherwise); the sketch Y = T_(n) Omega (eq. sampleMatrix) goes through q
    normalised power iterations  Q~ = nrm(Y),  Z = nrm(T_(n)^T Q~),
    Y = T_(n) Z  (eq. IMPsampleMatrix, Algorithm 1's power iterations), then
    Q_n = qr(Y).
    """
    Tn = unfold(T, n)
    J = Tn.shape[1]
    Om = test_matrix(test, seed, n, batch, J, l)
    Y = Tn @ Om
    y0 = Y.copy()
    for _ in range(int(q)):
        Qt = _normalize(Y, normalizer)
        Z = _normalize(Tn.T @ Qt, normalizer)
        Y = Tn @ Z
    Q = qr_pos(Y)
    return ModeStage(mode=n, shape_in=T.shape, omega=Om, y0=y0, y_final=Y, Q=Q)


@dataclass
class Compression:
    core: np.ndarray
    Q: List[np.ndarray]
    stages: List[ModeStage]


def compress(X: np.ndarray, k: int, p: int = 10, q: int = 2, seed: int = 0,
             batch: int = 0, scheme: str = "sequential",
             normalizer: str = "qr", test: str = "gaussian",
             modes: Optional[Sequence[int]] = None,
             p_modes: Optional[Sequence[int]] = None) -> Compression:
    """Randomized tensor compression (Algorithm 1).

    scheme="sequential": the paper's loop, in which mode n is sketched on the
    tensor already compressed in modes < n (the algorithm sets X <- B_n after
    each mode).  scheme="independent": every Q_n is taken from X itself and
    B = X x_1 Q_1^T ... x_N Q_N^T is formed afterwards.
    modes / p_modes (the remark after Algorithm 1: the user chooses the modes
    to compress and their oversampling): a mode left out keeps Q_n = I
    (its full size in the core); p_modes[n] replaces p for mode n.
    """
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    T = X
    Qs, stages = [], []
    chosen = set(range(N)) if modes is None else set(int(m) for m in modes)
    for n in range(N):
        src = T if scheme == "sequential" else X
        if n not in chosen:
            Qs.append(np.eye(src.shape[n]))
            stages.append(None)
            continue
        pn = p if p_modes is None else int(p_modes[n])
        l = sketch_width(k, pn, src.shape[n])
        st = range_finder(src, n, l, q, seed, batch, normalizer, test)
        stages.append(st)
        Qs.append(st.Q)
        if scheme == "sequential":
            T = mode_product(T, st.Q.T, n)
    if scheme == "independent":
        T = X
        for n in range(N):
            if n in chosen:
                T = mode_product(T, Qs[n].T, n)
    elif scheme != "sequential":
        raise ValueError(scheme)
    return Compression(core=T, Q=Qs, stages=stages)


# ---------------------------------------------------------------------------
# CP-ALS on the core (Section 3.2.1, Algorithm 2)

def eig_init(B: np.ndarray, R: int, n: int) -> np.ndarray:
    """Leading R eigenvectors of B_(n) B_(n)^T (Algorithm 2's initialisation),
    ordered by decreasing eigenvalue; each column's largest-magnitude entry
    (first index on ties) is made positive."""
    Bn = unfold(B, n)
    w, V = np.linalg.eigh(Bn @ Bn.T)
    V = V[:, ::-1][:, :R].copy()
    for r in range(V.shape[1]):
        i = int(np.argmax(np.abs(V[:, r])))
        if V[i, r] < 0:
            V[:, r] = -V[:, r]
    return V


def mttkrp(B: np.ndarray, factors: Sequence[np.ndarray], n: int) -> np.ndarray:
    """B_(n) times the Khatri-Rao product of all factors except n
    (the first factor of the least-squares updates of Algorithm 2)."""
    others = [factors[m] for m in range(B.ndim) if m != n]
    return unfold(B, n) @ khatri_rao(others)


def gram_hadamard(factors: Sequence[np.ndarray], skip: Optional[int]) -> np.ndarray:
    """Hadamard product of the Grams A_m^T A_m over m != skip
    (the matrix inside the Khatri-Rao pseudo-inverse, Definition 2)."""
    R = factors[0].shape[1]
    V = np.ones((R, R))
    for m, A in enumerate(factors):
        if m != skip:
            V = V * (A.T @ A)
    return V


PIVOT_RTOL = 1e-13


def solve_gram(M: np.ndarray, V: np.ndarray) -> np.ndarray:
    """M V^+ for the symmetric positive semi-definite R x R matrix V
    (Definition 2).  Cholesky solve when V is numerically positive definite;
    V counts as singular, and the Moore-Penrose pseudo-inverse is used,
    when the factorisation fails or a squared Cholesky pivot falls below
    PIVOT_RTOL times the largest diagonal entry of V."""
    try:
        c = scipy.linalg.cho_factor(V, lower=True, check_finite=True)
        piv = np.diag(c[0]) ** 2
        if np.min(piv) > PIVOT_RTOL * np.max(np.diag(V)):
            return scipy.linalg.cho_solve(c, M.T).T
    except (np.linalg.LinAlgError, scipy.linalg.LinAlgError):
        pass
    return M @ np.linalg.pinv(V, rcond=PIVOT_RTOL, hermitian=True)


def col_norms(A: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(A * A, axis=0))


def _scale_columns(A: np.ndarray, nu: np.ndarray) -> np.ndarray:
    safe = np.where(nu > 0, nu, 1.0)
    return A / safe[None, :]


@dataclass
class ALSResult:
    factors: List[np.ndarray]
    lam: np.ndarray
    rho: float
    iters: int
    rho_history: List[float] = field(default_factory=list)


def als(B: np.ndarray, R: int, max_iters: int, tol: float = 0.0,
        normX2: Optional[float] = None, init: Optional[Sequence[np.ndarray]] = None) -> ALSResult:
    """CP-ALS on B (Algorithm 2: initialisation and sweeps).

    Sweep: for n = 1..N, Ã_n = B_(n) KR(Ã_{m != n}) (*_{m != n} Ã_m^T Ã_m)^+,
    then column-normalise (modes 1..N-1) or split off lambda (mode N).

    normX2 is ||X||^2 of the uncompressed tensor (defaults to ||B||^2).
    Because X x_1 Q_1 ... x_N Q_N is an orthogonal projection of X onto a
    subspace that contains Xhat,
      ||X - Xhat||^2 = ||X||^2 - ||B||^2 + ||B - Bhat||^2,
      ||B - Bhat||^2 = ||B||^2 - 2 sum_r lam_r <M_N[:, r], Ã_N[:, r]>
                       + lam^T (*_m Ã_m^T Ã_m) lam,
    with M_N the mode-N product B_(N) KR(...) of the same sweep.
    """
    B = np.asarray(B, dtype=np.float64)
    N = B.ndim
    normB2 = float(np.dot(B.ravel(), B.ravel()))
    if normX2 is None:
        normX2 = normB2
    if init is None:
        A = [None] + [eig_init(B, R, n) for n in range(1, N)]
        A[0] = np.zeros((B.shape[0], R))
    else:
        A = [np.array(a, dtype=np.float64) for a in init]
    lam = np.ones(R)
    rho_prev = None
    rho = 0.0
    hist = []
    it = 0
    for it in range(1, int(max_iters) + 1):
        MN = None
        for n in range(N):
            M = mttkrp(B, A, n)
            V = gram_hadamard(A, skip=n)
            An = solve_gram(M, V)
            nu = col_norms(An)
            An = _scale_columns(An, nu)
            A[n] = An
            if n == N - 1:
                lam = nu
                MN = M
        inner = float(np.sum(lam * np.sum(MN * A[N - 1], axis=0)))
        model2 = float(lam @ gram_hadamard(A, skip=None) @ lam)
        resid2 = normB2 - 2.0 * inner + model2
        err2 = normX2 - normB2 + resid2
        rho = 1.0 - err2 / normX2 if normX2 > 0 else 0.0
        hist.append(rho)
        if tol > 0 and rho_prev is not None and abs(rho - rho_prev) < tol:
            break
        rho_prev = rho
    return ALSResult(factors=A, lam=lam, rho=rho, iters=it, rho_history=hist)


# ---------------------------------------------------------------------------
# Block coordinate descent on the core (Section 3.2.2, Algorithm 3)

@dataclass
class BCDResult:
    factors: List[np.ndarray]
    lam: np.ndarray
    rho: float
    iters: int                      # sweeps summed over the R components
    component_iters: List[int] = field(default_factory=list)
    rho_history: List[float] = field(default_factory=list)


def bcd_fit(B: np.ndarray, factors: Sequence[np.ndarray], lam: np.ndarray, r: int,
            normX2: float) -> float:
    """rho = 1 - ||X - Xhat||^2 / ||X||^2 (Section 3.3) for the model made of
    components 0..r, evaluated on the core as in ``als``:
    ||X - Xhat||^2 = ||X||^2 - 2 <B, Bhat> + ||Bhat||^2."""
    N = B.ndim
    idx = list(range(r + 1))
    Fs = [f[:, idx] for f in factors]
    lr = np.asarray(lam, dtype=np.float64)[idx]
    M = mttkrp(B, Fs, N - 1)
    inner = float(np.sum(lr * np.sum(M * Fs[N - 1], axis=0)))
    model = float(lr @ gram_hadamard(Fs, skip=None) @ lr)
    err2 = normX2 - 2.0 * inner + model
    return 1.0 - err2 / normX2 if normX2 > 0 else 0.0


def bcd(B: np.ndarray, R: int, max_iters: int, tol: float = 0.0,
        normX2: Optional[float] = None, init: Optional[Sequence[np.ndarray]] = None) -> BCDResult:
    """Rank-one block coordinate descent on B (Algorithm 3: initialisation and rank-one sweeps).

    The components are found one after another.  For component r the
    residual is Y = B - sum_{s<r} lam_s a_s^(0) o ... o a_s^(N-1) (the residual update),
    and the sweeps update its blocks in mode order:
        a_r^(n) = Y_(n) (KR_{m != n} a_r^(m)) / prod_{m != n} <a_r^(m), a_r^(m)>
    (the rank-one updates: the least-squares update of one block, the
    pseudo-inverse of the scalar Gram product), scaled to unit norm for
    n < N-1 and split into lam_r and a unit vector for n = N-1 (the normalisations
    11, 12).  Y is never formed (the remark before Algorithm 3): by
    multilinearity
        Y_(n) (KR a_r) = B_(n) (KR a_r)
                         - sum_{s<r} lam_s a_s^(n) prod_{m != n} <a_s^(m), a_r^(m)>.
    Starting vectors (the initialisation): column r of the leading eigenvectors of
    B_(n) B_(n)^T for modes 1..N-1; mode 0 is updated first.
    Stopping (the per-component convergence test): after sweep j >= 2 of a component once the fit
    (``bcd_fit`` of components 0..r) changes by less than tol; tol = 0 runs
    exactly max_iters sweeps per component.
    """
    B = np.asarray(B, dtype=np.float64)
    N = B.ndim
    normB2 = float(np.dot(B.ravel(), B.ravel()))
    if normX2 is None:
        normX2 = normB2
    if init is None:
        A = [np.zeros((B.shape[0], R))] + [eig_init(B, R, n) for n in range(1, N)]
    else:
        A = [np.array(a, dtype=np.float64) for a in init]
    lam = np.zeros(R)
    hist, comp_iters = [], []
    rho = 0.0
    total = 0
    for r in range(R):
        rho_prev = None
        it = 0
        for it in range(1, int(max_iters) + 1):
            for n in range(N):
                cols = [A[m][:, r:r + 1] for m in range(N)]
                v = mttkrp(B, cols, n)[:, 0]
                for s in range(r):
                    w = 1.0
                    for m in range(N):
                        if m != n:
                            w *= float(A[m][:, s] @ A[m][:, r])
                    v = v - lam[s] * w * A[n][:, s]
                d = 1.0
                for m in range(N):
                    if m != n:
                        d *= float(A[m][:, r] @ A[m][:, r])
                v = v / d if d > 0 else np.zeros_like(v)
                nu = float(np.sqrt(v @ v))
                A[n][:, r] = v / nu if nu > 0 else v
                if n == N - 1:
                    lam[r] = nu
            rho = bcd_fit(B, A, lam, r, normX2)
            hist.append(rho)
            if tol > 0 and rho_prev is not None and abs(rho - rho_prev) < tol:
                break
            rho_prev = rho
        comp_iters.append(it)
        total += it
    return BCDResult(factors=A, lam=lam, rho=rho, iters=total, component_iters=comp_iters,
                     rho_history=hist)


def finalize(lam: np.ndarray, factors: Sequence[np.ndarray]):
    """Algorithm 2's final renormalisation: re-normalise the columns, fold the norms into
    lambda, sort by lambda (descending) and fix signs (largest-magnitude
    entry positive in modes 1..N-1, sign pushed into mode N)."""
    A = [np.array(f, dtype=np.float64) for f in factors]
    lam = np.array(lam, dtype=np.float64)
    for n in range(len(A)):
        nu = col_norms(A[n])
        A[n] = _scale_columns(A[n], nu)
        lam = lam * np.where(nu > 0, nu, 1.0)
    order = np.argsort(-lam, kind="stable")
    lam = lam[order]
    A = [a[:, order] for a in A]
    N = len(A)
    for r in range(lam.shape[0]):
        for n in range(N - 1):
            i = int(np.argmax(np.abs(A[n][:, r])))
            if A[n][i, r] < 0:
                A[n][:, r] = -A[n][:, r]
                A[N - 1][:, r] = -A[N - 1][:, r]
    return lam, A


def expand(Q: Sequence[np.ndarray], factors: Sequence[np.ndarray], lam: np.ndarray):
    """Back-projection A_n = Q_n Ã_n (eq. qbs, Algorithm 2's factor recovery)
    followed by the final renormalisation."""
    return finalize(lam, [Qn @ An for Qn, An in zip(Q, factors)])


@dataclass
class RCPResult:
    lam: np.ndarray
    factors: List[np.ndarray]
    rho: float
    rel_err: float
    iters: int
    compression: Compression
    als: ALSResult


def rcp_als(X: np.ndarray, R: int, p: int = 10, q: int = 2, max_iters: int = 50,
            tol: float = 0.0, seed: int = 0, scheme: str = "sequential",
            normalizer: str = "qr", batch: int = 0, test: str = "gaussian",
            modes: Optional[Sequence[int]] = None,
            p_modes: Optional[Sequence[int]] = None) -> RCPResult:
    """Randomized CP via ALS (Algorithm 2): compress with target rank k = R,
    fit CP-ALS on the core, back-project and renormalise."""
    X = np.asarray(X, dtype=np.float64)
    normX2 = float(np.dot(X.ravel(), X.ravel()))
    comp = compress(X, R, p, q, seed, batch, scheme, normalizer, test, modes, p_modes)
    res = als(comp.core, R, max_iters, tol, normX2=normX2)
    lam, A = expand(comp.Q, res.factors, res.lam)
    rel = float(np.sqrt(max(0.0, 1.0 - res.rho)))
    return RCPResult(lam=lam, factors=A, rho=res.rho, rel_err=rel, iters=res.iters,
                     compression=comp, als=res)


def rcp_bcd(X: np.ndarray, R: int, p: int = 10, q: int = 2, max_iters: int = 50,
            tol: float = 0.0, seed: int = 0, scheme: str = "sequential",
            normalizer: str = "qr", batch: int = 0) -> RCPResult:
    """Randomized CP via block coordinate descent (Algorithm 3): the same
    compression as ``rcp_als``, ``bcd`` on the core (the rank-one sweeps),
    back-projection and renormalisation (Algorithm 3's factor recovery)."""
    X = np.asarray(X, dtype=np.float64)
    normX2 = float(np.dot(X.ravel(), X.ravel()))
    comp = compress(X, R, p, q, seed, batch, scheme, normalizer)
    res = bcd(comp.core, R, max_iters, tol, normX2=normX2)
    lam, A = expand(comp.Q, res.factors, res.lam)
    rel = float(np.sqrt(max(0.0, 1.0 - res.rho)))
    return RCPResult(lam=lam, factors=A, rho=res.rho, rel_err=rel, iters=res.iters,
                     compression=comp, als=res)


def cp_bcd(X: np.ndarray, R: int, max_iters: int = 50, tol: float = 0.0):
    """Deterministic CP via block coordinate descent on the full tensor (the
    solver of Algorithm 3 with Q_n = I)."""
    X = np.asarray(X, dtype=np.float64)
    res = bcd(X, R, max_iters, tol)
    lam, A = finalize(res.lam, res.factors)
    return lam, A, res


def cp_als(X: np.ndarray, R: int, max_iters: int = 50, tol: float = 0.0):
    """Deterministic CP-ALS on the full tensor: the same solver with Q_n = I
    (the baseline that the paper's implementation follows, Section 3.3)."""
    X = np.asarray(X, dtype=np.float64)
    res = als(X, R, max_iters, tol)
    lam, A = finalize(res.lam, res.factors)
    return lam, A, res
