"""Parity of the HIP path (through the C interface) with the float64 oracle.

Stage-level checks compare each entry point with the oracle on the same
seeded input; end-to-end checks compare the decomposition by what is
unique about it (relative reconstruction error and factor congruence),
since CP factors are defined only up to permutation, scale and sign and
the randomized path agrees with the oracle only up to rounding.

Tolerances (float32 path vs float64 oracle):
  * Omega: the uint32 stream is identical, log/sqrt/sincos in float32 ->
    a few float32 ulps of |z| <= 5.8: |diff| <= 4e-6.
  * bases Q_n on well-conditioned inputs: float32 accumulation of
    contractions of length J ~ 1e3..1e5 with orthonormalisation in
    float64; entries are O(1/sqrt(I)); |diff| <= 2e-4 absolute.
  * mode products with a given Q: relative error <= 1e-5 of the max.
  * end to end: |rel_err_gpu - rel_err_oracle| <= 1e-4 and congruence >= 0.999.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from oracle import evaluate, philox, rcp  # noqa: E402
from paper_1703_09074_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    yield
    torch.cuda.synchronize()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


# ---------------------------------------------------------------------------
def test_omega_bits_match_oracle():
    seed = (123 << 32) | 456
    plan = rcpgpu.Plan((64, 64, 64), 5, 5, 0, 1, 0.0, seed)
    for mode, row0, nrows, l in [(0, 0, 5000, 30), (2, 12345, 777, 13), (1, (1 << 32) + 5, 300, 64)]:
        got = _np(plan.omega(mode, row0, nrows, l))
        want = philox.omega(seed, mode, 0, row0, nrows, l)
        assert np.max(np.abs(got - want)) <= 4e-6, (mode, row0, np.max(np.abs(got - want)))


def test_philox_words_match_oracle_bitwise():
    """The uint32 Philox4x32-10 stream behind Omega is the oracle's, bit for bit
    (rows past 2^32 included, so the counter's high word is exercised)."""
    seed = (0xDEADBEEF << 32) | 0x12345678
    plan = rcpgpu.Plan((64, 64, 64), 5, 5, 0, 1, 0.0, seed)
    for mode, row0, nrows, ng in [(0, 0, 4096, 16), (1, 77777, 1000, 3), (2, (1 << 32) - 10, 20, 8)]:
        got = plan.philox_words(mode, row0, nrows, ng).cpu().numpy().view(np.uint32)
        want = philox.omega_bits(seed, mode, 0, row0, nrows, ng).astype(np.uint32)
        np.testing.assert_array_equal(got.reshape(nrows, 4 * ng), want)


SKETCH_CASES = [
    # shape, mode, k, p, q
    ((37, 50, 41), 0, 5, 5, 0),        # ragged, case A (Rr = 2050)
    ((37, 50, 41), 1, 5, 5, 1),        # middle mode, Rr = 41 (case A, ragged tile)
    ((37, 50, 41), 2, 5, 5, 2),        # last mode, Rr = 1 (case B)
    ((64, 48, 5), 1, 4, 6, 1),         # small Rr (case B, 6 slabs per tile)
    ((120, 90, 70), 0, 10, 10, 2),     # several row blocks of 64, many tiles
    ((30, 11, 3, 7), 2, 3, 4, 1),      # 4-way, Rr = 7
    ((45, 33), 0, 6, 4, 2),            # matrix (N = 2)
    ((16, 16, 16), 1, 10, 10, 1),      # l = I: square basis
    ((600, 20, 9), 0, 8, 8, 1),        # I > 512: two row blocks, two-pass power step
    ((3, 530, 70), 1, 3, 9, 2),        # tall middle mode: 3 a-slabs, unaligned rows
    ((1500, 30, 20), 0, 6, 4, 2),      # basis too tall for one workgroup's LDS: row-block QR
    ((1300, 50, 40), 0, 20, 20, 1),    # the same with 40 columns (the 1024-thread Cholesky)
]


@pytest.mark.parametrize("shape,mode,k,p,q", SKETCH_CASES)
def test_sketch_matches_oracle(shape, mode, k, p, q):
    T = _rand(shape, sum(shape) + mode)
    seed = 99 + mode
    plan = rcpgpu.Plan(shape, k, p, q, 1, 0.0, seed)
    Q = _np(plan.sketch(_dev(T), mode))
    l = rcp.sketch_width(k, p, shape[mode])
    want = rcp.range_finder(T.astype(np.float64), mode, l, q, seed).Q
    assert Q.shape == want.shape
    np.testing.assert_allclose(Q.T @ Q, np.eye(l), atol=2e-6)
    err = np.max(np.abs(Q - want))
    assert err <= 2e-4, err


@pytest.mark.parametrize("shape,mode", [((37, 50, 41), 0), ((37, 50, 41), 1), ((37, 50, 41), 2),
                                        ((64, 48, 5), 1), ((30, 11, 3, 7), 3), ((700, 9, 40), 0),
                                        ((45, 33), 1), ((3, 530, 70), 1), ((520, 300), 0)])
def test_compress_matches_oracle(shape, mode):
    T = _rand(shape, 7 + mode)
    I = shape[mode]
    l = min(8, I)
    Qn = np.linalg.qr(np.random.default_rng(mode).standard_normal((I, l)))[0].astype(np.float32)
    k = min(2, min(shape))
    plan = rcpgpu.Plan(shape, k, 8 - k, 0, 1, 0.0, 1)
    out = _np(plan.compress(_dev(T), mode, _dev(Qn)))
    want = rcp.mode_product(T.astype(np.float64), Qn.astype(np.float64).T, mode)
    assert out.shape == want.shape
    assert np.max(np.abs(out - want)) <= 1e-5 * np.max(np.abs(want))


def test_norm2():
    X = _rand((33, 17, 9), 5)
    plan = rcpgpu.Plan(X.shape, 3, 2, 0, 1, 0.0, 1)
    got = float(_np(plan.norm2(_dev(X)))[0])
    want = float(np.sum(X.astype(np.float64) ** 2))
    assert abs(got - want) <= 1e-12 * want


def _core_problem(dims, R, noise, seed, k, p, q):
    w = synth.low_rank(dims, R, noise, seed)
    comp = rcp.compress(w.X.astype(np.float64), k, p, q, seed=seed)
    return w, comp


@pytest.mark.parametrize("dims,R,iters", [((40, 35, 30), 4, 30), ((20, 18, 16, 14), 3, 25),
                                          ((60, 50), 5, 20)])
def test_als_matches_oracle(dims, R, iters):
    w, comp = _core_problem(dims, R, 0.05, 11, R, 5, 1)
    core = comp.core.astype(np.float32)
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    plan = rcpgpu.Plan(dims, R, 5, 1, iters, 0.0, 11)
    nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
    At, lam, info = plan.als(_dev(core), nx)
    info = rcpgpu.Plan.read_info(info)
    ref = rcp.als(core.astype(np.float64), R, iters, normX2=normX2)
    assert info["iters"] == iters
    assert abs(info["rho"] - ref.rho) <= 1e-7
    gl = _np(lam)
    cong, cmin, perm = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.9999
    np.testing.assert_allclose(gl, ref.lam[perm], rtol=1e-4)


# The stopping rule of Section 3.3 in the one-workgroup kernel (core in LDS):
# after sweep j >= 2 the run ends once the fit changes by less than tol.
@pytest.mark.parametrize("dims,R,tol", [((40, 35, 30), 4, 1e-6), ((20, 18, 16, 14), 3, 1e-7),
                                        ((30, 28, 26), 6, 1e-5)])
def test_als_stopping_rule_in_lds(dims, R, tol):
    w, comp = _core_problem(dims, R, 0.05, 17, R, 5, 1)
    core = comp.core.astype(np.float32)
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    plan = rcpgpu.Plan(dims, R, 5, 1, 500, tol, 17)
    nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
    At, lam, info = plan.als(_dev(core), nx)
    info = rcpgpu.Plan.read_info(info)
    ref = rcp.als(core.astype(np.float64), R, 500, tol=tol, normX2=normX2)
    assert 2 <= ref.iters < 500
    assert info["iters"] == ref.iters, (info["iters"], ref.iters)
    assert abs(info["rho"] - ref.rho) <= 1e-7, (info["rho"], ref.rho)
    cong, cmin, perm = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.9999, cmin


# Warm start (rcp_als with given factors): the sweeps continue from the
# caller's factors instead of the eigenvector start, in both the in-LDS and
# the grid-wide form; the oracle continues from the same factors.
@pytest.mark.parametrize("dims,R", [((40, 35, 30), 4), ((20, 18, 16, 14), 3), ((60, 55, 50), 40)])
def test_als_warm_start_matches_oracle(dims, R):
    w, comp = _core_problem(dims, R, 0.05, 23, R, 5, 1)
    core = comp.core.astype(np.float32)
    c64 = core.astype(np.float64)
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    first = rcp.als(c64, R, 4, normX2=normX2)
    start = [f.astype(np.float32) for f in first.factors]
    ref = rcp.als(c64, R, 3, normX2=normX2, init=[s.astype(np.float64) for s in start])
    plan = rcpgpu.Plan(dims, R, 5, 1, 3, 0.0, 23)
    nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
    At, lam, info = plan.als(_dev(core), nx, init=[_dev(s) for s in start])
    info = rcpgpu.Plan.read_info(info)
    assert info["iters"] == 3
    assert abs(info["rho"] - ref.rho) <= 1e-7, (info["rho"], ref.rho)
    cong, cmin, perm = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.9999, cmin
    np.testing.assert_allclose(_np(lam), ref.lam[perm], rtol=1e-4)
    # three sweeps from the eigenvector start end elsewhere than three more
    # sweeps after the first four: the given factors were used
    At_c, lam_c, info_c = plan.als(_dev(core), nx)
    cold = rcpgpu.Plan.read_info(info_c)
    assert abs(cold["rho"] - info["rho"]) > 1e-9, (cold["rho"], info["rho"])


def test_status_word_collects_numeric_outcomes():
    """rcp_read_status: a noise-free rank-3 tensor with l = 13 > 3 makes the
    sketches exactly rank deficient (Householder QR fallback); an all-zero
    core makes the Gram singular (pseudo-inverse).  The word is cleared by
    each read."""
    w = synth.low_rank((60, 50, 40), 3, 0.0, 41)
    plan = rcpgpu.Plan(w.X.shape, 3, 10, 1, 5, 0.0, 3)
    assert plan.read_status() == 0
    plan.decompose(_dev(w.X))
    st = plan.read_status()
    assert st & rcpgpu._lib.RCP_INFO_QR_HOUSEHOLDER, st
    assert plan.read_status() == 0
    zp = rcpgpu.Plan((9, 8, 7), 3, 4, 0, 3, 0.0, 11)
    zp.als(_dev(np.zeros((7, 7, 7), np.float32)), torch.tensor([1.0], dtype=torch.float64,
                                                                 device="cuda"))
    st = zp.read_status()
    assert st & rcpgpu._lib.RCP_INFO_PINV_FALLBACK, st
    # a well-conditioned problem raises nothing
    w2 = synth.low_rank((50, 40, 30), 4, 0.05, 43)
    p2 = rcpgpu.Plan(w2.X.shape, 4, 6, 1, 10, 0.0, 5)
    p2.decompose(_dev(w2.X))
    assert p2.read_status() == 0


# An all-zero core: the first update makes A_0 zero, so every later V is the
# zero matrix, the elimination meets zero pivots and the pseudo-inverse (of
# zero) takes over (Definition 2), as in the oracle.  Three solver paths: one
# wavefront (R = 3), blocked elimination (R = 36 > 32 rows) and the grid-wide
# form (a 45^3 core exceeds one workgroup's LDS).
@pytest.mark.parametrize("dims,R", [((9, 8, 7), 3), ((60, 50), 36), ((45, 45, 45), 4)])
def test_als_zero_core_takes_pseudo_inverse(dims, R):
    iters = 3
    core = np.zeros(dims, dtype=np.float32)
    plan = rcpgpu.Plan(dims, R, max(dims) - R, 0, iters, 0.0, 11)
    nx = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    At, lam, info = plan.als(_dev(core), nx)
    info = rcpgpu.Plan.read_info(info)
    ref = rcp.als(core.astype(np.float64), R, iters, normX2=1.0)
    assert info["status"] & 1, info
    assert info["iters"] == iters
    assert info["rho"] == ref.rho == 0.0
    assert np.all(_np(lam) == 0.0) and np.all(ref.lam == 0.0)
    for a, b in zip(At, ref.factors):
        assert np.all(_np(a) == 0.0) and np.all(b == 0.0)


# Cores larger than one workgroup's LDS take the grid-wide form (mode
# products over the whole GPU, one-workgroup solves): 45^3 and 15^4 floats.
@pytest.mark.parametrize("dims,R,iters,tol", [((60, 55, 50), 40, 15, 0.0),
                                              ((30, 28, 26, 24), 10, 20, 0.0),
                                              ((30, 28, 26, 24), 10, 200, 1e-6)])
def test_als_grid_wide_matches_oracle(dims, R, iters, tol):
    w, comp = _core_problem(dims, R, 0.05, 13, R, 5, 1)
    core = comp.core.astype(np.float32)
    assert core.size * 4 > 160 * 1024
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    plan = rcpgpu.Plan(dims, R, 5, 1, iters, tol, 13)
    nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
    At, lam, info = plan.als(_dev(core), nx)
    info = rcpgpu.Plan.read_info(info)
    ref = rcp.als(core.astype(np.float64), R, iters, tol=tol, normX2=normX2)
    assert info["status"] == 0, info
    assert info["iters"] == ref.iters, (info, ref.iters)
    assert abs(info["rho"] - ref.rho) <= 1e-7, (info["rho"], ref.rho)
    cong, cmin, perm = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.999, cmin
    np.testing.assert_allclose(_np(lam), ref.lam[perm], rtol=1e-4)
    # without ||X||^2 the fit is taken against ||core||^2
    At2, lam2, info2 = plan.als(_dev(core))
    info2 = rcpgpu.Plan.read_info(info2)
    ref2 = rcp.als(core.astype(np.float64), R, iters, tol=tol)
    assert abs(info2["rho"] - ref2.rho) <= 1e-6, (info2["rho"], ref2.rho)


def test_als_grid_wide_under_graph_capture():
    """The grid-wide ALS (mode products over the whole GPU, float64
    reductions, one-workgroup solves, a device-side stop flag) recorded into a
    HIP graph: three replays (with eager work in between) each reproduce the
    eager run exactly (the reductions have a fixed order) and match the
    oracle.  Eight sweeps from the eigenvector start stop this core mid-descent
    (the fit still moves by 1e-2 a sweep), where the float32 rounding of the
    mode products is amplified to a few 1e-7 in the fit (1.9e-7 and 5.2e-7
    for two summation orders of the products), hence 1e-6 against the
    oracle."""
    dims, R, iters = (60, 55, 50), 40, 8
    w, comp = _core_problem(dims, R, 0.05, 29, R, 5, 1)
    core = _dev(comp.core.astype(np.float32))
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    ref = rcp.als(comp.core.astype(np.float32).astype(np.float64), R, iters, normX2=normX2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan = rcpgpu.Plan(dims, R, 5, 1, iters, 0.0, 29)
        nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
        At_e, lam_e, info_e = plan.als(core, nx)             # eager
    torch.cuda.synchronize()
    eager = rcpgpu.Plan.read_info(info_e)
    assert abs(eager["rho"] - ref.rho) <= 1e-6, (eager["rho"], ref.rho)
    lam_eager = _np(lam_e)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        At_g, lam_g, info_g = plan.als(core, nx)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = rcpgpu.Plan.read_info(info_g)
        assert got["iters"] == iters and got["status"] == 0, got
        assert got["rho"] == eager["rho"], (rep, got["rho"], eager["rho"])
        np.testing.assert_array_equal(_np(lam_g), lam_eager)
        assert abs(got["rho"] - ref.rho) <= 1e-6, (rep, got["rho"], ref.rho)
        cong, cmin, perm = evaluate.congruence([_np(a) for a in At_g], ref.factors)
        assert cmin >= 0.999, cmin
        np.testing.assert_allclose(_np(lam_g), ref.lam[perm], rtol=1e-4)
        lam_g.zero_()
        info_g.zero_()
        torch.cuda.synchronize()


def test_expand_matches_oracle():
    dims, R = (50, 40, 30), 4
    w, comp = _core_problem(dims, R, 0.05, 12, R, 6, 1)
    res = rcp.als(comp.core, R, 10)
    plan = rcpgpu.Plan(dims, R, 6, 1, 10, 0.0, 12)
    Q = [_dev(q) for q in comp.Q]
    At = [_dev(a) for a in res.factors]
    A, lam = plan.expand(Q, At, _dev(res.lam))
    lam_ref, A_ref = rcp.expand([q.astype(np.float32).astype(np.float64) for q in comp.Q],
                                [a.astype(np.float32).astype(np.float64) for a in res.factors],
                                res.lam.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(_np(lam), lam_ref, rtol=2e-6)
    for a, b in zip(A, A_ref):
        np.testing.assert_allclose(_np(a), b, atol=2e-6)


# ---------------------------------------------------------------------------
def _decompose_and_compare(X, k, p, q, iters, seed, scheme="sequential", truth=None,
                           tol_err=1e-4, min_cong=0.999):
    lam, A, info = rcpgpu.decompose(_dev(X), k, p, q, iters, 0.0, seed, scheme)
    lam = _np(lam)
    A = [_np(a) for a in A]
    ref = rcp.rcp_als(X.astype(np.float64), k, p, q, iters, 0.0, seed, scheme)
    e_gpu = evaluate.relative_error(X, lam, A)
    e_ref = evaluate.relative_error(X, ref.lam, ref.factors)
    assert abs(e_gpu - e_ref) <= tol_err, (e_gpu, e_ref)
    assert abs(info["rel_err"] - e_gpu) <= max(1e-4, 1e-3 * e_gpu), (info, e_gpu)
    assert info["iters"] == iters
    cong, cmin, perm = evaluate.congruence(A, ref.factors)
    assert cong >= min_cong, cong
    assert np.all(np.diff(lam) <= 0)
    for a in A:
        np.testing.assert_allclose(np.linalg.norm(a, axis=0), 1.0, atol=1e-5)
    return e_gpu, e_ref, cong, info


def test_decompose_rcp100():
    cfg = synth.WORKLOADS["rcp100"]
    w = synth.make("rcp100")
    _decompose_and_compare(w.X, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], cfg["seed"])


@pytest.mark.parametrize("dims,R,noise,k,p,q,iters,scheme", [
    ((70, 60, 50), 6, 0.05, 6, 10, 1, 25, "sequential"),
    ((70, 60, 50), 6, 0.05, 6, 10, 2, 25, "independent"),
    ((24, 22, 20, 18), 4, 0.05, 4, 6, 1, 30, "sequential"),
    ((90, 80, 70), 5, 0.02, 5, 10, 0, 30, "sequential"),
    ((150, 40), 5, 0.05, 5, 5, 2, 20, "sequential"),
])
def test_decompose_variants(dims, R, noise, k, p, q, iters, scheme):
    w = synth.low_rank(dims, R, noise, 31 + len(dims))
    _decompose_and_compare(w.X, k, p, q, iters, 5, scheme)


def test_decompose_noise_free_rank_deficient_sketch():
    """l > R on an exactly rank-R tensor: the sketches are rank deficient,
    the Householder QR still returns orthonormal bases."""
    w = synth.low_rank((60, 50, 40), 3, 0.0, 41)
    lam, A, info = rcpgpu.decompose(_dev(w.X), 3, 10, 1, 40, 0.0, 3)
    e = evaluate.relative_error(w.X, _np(lam), [_np(a) for a in A])
    assert e < 1e-5
    cong = evaluate.congruence([_np(a) for a in A], w.factors)[0]
    assert cong > 0.99999


# (dims, k, p): sketch widths 10 (the one-wavefront Cholesky), 40 and 60 (the
# 2 x 2 block Cholesky over 32-row register eliminations); 1200 rows take the
# row-block QR, 400 rows the one-workgroup QR
QR_WIDTH_CASES = [((1200, 20, 16), 4, 6), ((1200, 64, 40), 30, 10), ((1200, 64, 64), 50, 10),
                  ((400, 64, 40), 30, 10), ((400, 64, 64), 50, 10)]


@pytest.mark.parametrize("dims,k,p", QR_WIDTH_CASES)
def test_tall_rank_deficient_sketch(dims, k, p):
    """A rank-2 noise-free tensor sketched 10 to 60 wide: an orthonormal basis
    whose span holds the mode's range."""
    w = synth.low_rank(dims, 2, 0.0, 43)
    plan = rcpgpu.Plan(dims, k, p, 1, 5, 0.0, 3)
    Q = _np(plan.sketch(_dev(w.X), 0))
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-5)
    X0 = rcp.unfold(w.X.astype(np.float64), 0)
    resid = np.linalg.norm(X0 - Q @ (Q.T @ X0)) / np.linalg.norm(X0)
    assert resid < 1e-5, resid


@pytest.mark.parametrize("dims,k,p", QR_WIDTH_CASES)
def test_tall_zero_sketch_falls_back_to_householder(dims, k, p):
    """An all-zero tensor: every Cholesky pivot is zero, the Householder
    fallback runs on the (unchanged) sketch and returns an orthonormal basis,
    raising its bit."""
    plan = rcpgpu.Plan(dims, k, p, 1, 5, 0.0, 3)
    assert plan.read_status() == 0
    Q = _np(plan.sketch(_dev(np.zeros(dims)), 0))
    np.testing.assert_allclose(Q.T @ Q, np.eye(Q.shape[1]), atol=1e-6)
    assert plan.read_status() & rcpgpu._lib.RCP_INFO_QR_HOUSEHOLDER


def test_decompose_rcp400_full_size():
    cfg = synth.WORKLOADS["rcp400"]
    w = synth.make("rcp400")
    _decompose_and_compare(w.X, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], cfg["seed"])


def test_deterministic_bits():
    w = synth.low_rank((80, 70, 60), 5, 0.05, 51)
    X = _dev(w.X)
    plan = rcpgpu.Plan(w.X.shape, 5, 10, 2, 20, 0.0, 9)
    lam1, A1, _ = plan.decompose(X)
    lam2, A2, _ = plan.decompose(X)
    torch.cuda.synchronize()
    assert torch.equal(lam1, lam2)
    for a, b in zip(A1, A2):
        assert torch.equal(a, b)


def test_stage_entry_points_compose_to_decompose():
    """rcp_sketch / rcp_compress / rcp_als / rcp_expand called one by one give
    the same result as rcp_decompose (sequential scheme)."""
    w = synth.low_rank((50, 45, 40), 4, 0.05, 61)
    X = _dev(w.X)
    plan = rcpgpu.Plan(w.X.shape, 4, 6, 1, 15, 0.0, 21)
    lam_d, A_d, info_d = plan.decompose(X)
    Q_d = [q.clone() for q in plan.bases()]
    core_d = plan.core().clone()
    T = X
    Qs = []
    for n in range(3):
        Q = plan.sketch(T, n)
        Qs.append(Q)
        T = plan.compress(T, n, Q)
    torch.cuda.synchronize()
    for a, b in zip(Qs, Q_d):
        assert torch.equal(a, b)
    assert torch.equal(T, core_d)
    nx = plan.norm2(X)
    At, lam, info = plan.als(T, nx)
    A, lam2 = plan.expand(Qs, At, lam)
    torch.cuda.synchronize()
    assert torch.equal(lam2, lam_d)
    for a, b in zip(A, A_d):
        assert torch.equal(a, b)


def test_python_api_rejects_bad_arguments():
    plan = rcpgpu.Plan((20, 20, 20), 4, 4, 1, 5, 0.0, 1)
    X = _dev(_rand((20, 20, 20), 1))
    with pytest.raises(ValueError):
        plan.decompose(_dev(_rand((20, 20, 21), 1)))
    with pytest.raises(TypeError):
        plan.decompose(X.double())
    Q = plan.sketch(X, 0)
    st = plan.lib.rcp_compress(plan.handle, X.data_ptr(), rcpgpu._lib.dims_array((20, 20, 20)), 0,
                               Q.data_ptr(), X.data_ptr())
    assert st == rcpgpu._lib.RCP_ERR_INVALID_ARG          # output aliases the input
    st = plan.lib.rcp_sketch(plan.handle, X.data_ptr(), rcpgpu._lib.dims_array((20, 21, 20)), 0,
                             Q.data_ptr())
    assert st == rcpgpu._lib.RCP_ERR_INVALID_ARG          # dims beyond the plan's
