"""Block coordinate descent (Section 3.2.2, Algorithm 3) on the GPU against
the float64 oracle's ``bcd`` / ``rcp_bcd`` on the same inputs.

Tolerances (float32 core and contractions, float64 factors and sums, against
float64 throughout):
  * on a given core: fit within 1e-7, congruence >= 0.9999, lambda to 1e-4,
    the same number of sweeps (also with the per-component stopping rule);
  * end to end: |rel_err_gpu - rel_err_oracle| <= 1e-4, congruence >= 0.999.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from oracle import evaluate, rcp  # noqa: E402
from paper_1703_09074_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _core(dims, R, p, seed):
    w = synth.low_rank(dims, R, 0.05, seed)
    comp = rcp.compress(w.X.astype(np.float64), R, p, 1, seed=seed)
    return w, comp.core.astype(np.float32)


@pytest.mark.parametrize("dims,R,p,iters,tol", [
    ((40, 35, 30), 4, 5, 15, 0.0),          # core in LDS
    ((20, 18, 16, 14), 3, 5, 12, 0.0),      # 4-way
    ((60, 50), 5, 8, 10, 0.0),              # matrix
    ((60, 55, 50), 10, 35, 6, 0.0),         # 45^3 core: read from global memory
    ((40, 35, 30), 4, 5, 400, 1e-8),        # stopping rule per component
])
def test_bcd_on_core_matches_oracle(dims, R, p, iters, tol):
    w, core = _core(dims, R, p, 31)
    normX2 = float(np.sum(w.X.astype(np.float64) ** 2))
    ref = rcp.bcd(core.astype(np.float64), R, iters, tol=tol, normX2=normX2)
    plan = rcpgpu.Plan(dims, R, p, 1, iters, tol, 31, solver="bcd")
    nx = torch.tensor([normX2], dtype=torch.float64, device="cuda")
    At, lam, info = plan.bcd(_dev(core), nx)
    info = rcpgpu.Plan.read_info(info)
    print(f"[bcd] {dims} R={R}: rho gpu {info['rho']:.12f} oracle {ref.rho:.12f} "
          f"iters {info['iters']} / {ref.iters}", flush=True)
    assert info["status"] == 0, info
    assert info["iters"] == ref.iters, (info["iters"], ref.iters)
    assert abs(info["rho"] - ref.rho) <= 1e-7, (info["rho"], ref.rho)
    cong, cmin, perm = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.9999, cmin
    np.testing.assert_allclose(_np(lam), ref.lam[perm], rtol=1e-4)
    # the fit against ||core||^2 when ||X||^2 is not given
    At2, lam2, info2 = plan.bcd(_dev(core))
    ref2 = rcp.bcd(core.astype(np.float64), R, iters, tol=tol)
    assert abs(rcpgpu.Plan.read_info(info2)["rho"] - ref2.rho) <= 1e-6


def test_bcd_warm_start_matches_oracle():
    dims, R, p = (40, 35, 30), 4, 5
    w, core = _core(dims, R, p, 37)
    c64 = core.astype(np.float64)
    rng = np.random.default_rng(3)
    start = [rng.standard_normal((l, R)).astype(np.float32) for l in core.shape]
    ref = rcp.bcd(c64, R, 5, init=[s.astype(np.float64) for s in start])
    plan = rcpgpu.Plan(dims, R, p, 1, 5, 0.0, 37, solver="bcd")
    At, lam, info = plan.bcd(_dev(core), init=[_dev(s) for s in start])
    info = rcpgpu.Plan.read_info(info)
    assert abs(info["rho"] - ref.rho) <= 1e-7, (info["rho"], ref.rho)
    cong, cmin, _ = evaluate.congruence([_np(a) for a in At], ref.factors)
    assert cmin >= 0.9999, cmin


def test_bcd_recovers_orthogonal_components():
    """A noise-free orthogonally decomposable tensor: the components come back
    exactly, largest first."""
    rng = np.random.default_rng(5)
    dims, weights = (30, 28, 26), np.array([9.0, 6.0, 4.0, 2.5, 1.0])
    fac = [np.linalg.qr(rng.standard_normal((d, 5)))[0] for d in dims]
    X = rcp.kruskal_full(weights, fac).astype(np.float32)
    lam, A, info = rcpgpu.decompose(_dev(X), 5, 10, 1, 40, 0.0, 3, solver="bcd")
    lam = _np(lam)
    np.testing.assert_allclose(lam, weights, rtol=1e-5)
    e = evaluate.relative_error(X, lam, [_np(a) for a in A])
    assert e < 1e-5, e
    cong = evaluate.congruence([_np(a) for a in A], fac)[0]
    assert cong > 0.99999, cong


@pytest.mark.parametrize("dims,R,noise,k,p,q,iters", [
    ((100, 100, 100), 5, 0.01, 5, 10, 2, 30),
    ((24, 22, 20, 18), 4, 0.05, 4, 6, 1, 20),
    ((120, 90, 70), 6, 0.1, 6, 10, 2, 25),
])
def test_decompose_bcd_matches_oracle(dims, R, noise, k, p, q, iters):
    w = synth.low_rank(dims, R, noise, 41 + len(dims))
    lam, A, info = rcpgpu.decompose(_dev(w.X), k, p, q, iters, 0.0, 7, solver="bcd")
    lam = _np(lam)
    A = [_np(a) for a in A]
    ref = rcp.rcp_bcd(w.X.astype(np.float64), k, p, q, iters, 0.0, 7)
    e_gpu = evaluate.relative_error(w.X, lam, A)
    e_ref = evaluate.relative_error(w.X, ref.lam, ref.factors)
    cong = evaluate.congruence(A, ref.factors)[0]
    print(f"[bcd] decompose {dims}: rel_err gpu {e_gpu:.7f} oracle {e_ref:.7f} congruence {cong:.6f}",
          flush=True)
    assert abs(e_gpu - e_ref) <= 1e-4, (e_gpu, e_ref)
    assert abs(info["rel_err"] - e_gpu) <= max(1e-4, 1e-3 * e_gpu), (info, e_gpu)
    assert info["iters"] == k * iters
    assert cong >= 0.999, cong
    assert np.all(np.diff(lam) <= 0)
