"""rcp_decompose_noalloc (the entry point for callers that cannot allocate)
against rcp_decompose on the same inputs, through the C interface: two
calls in a row, the second on a smaller problem, each equal to the planned
entry point's result; a problem whose workspace exceeds the library's
scratch array is refused with RCP_ERR_WORKSPACE."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from paper_1703_09074_amd import _lib, synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _noalloc(lib, dims, k, p, q, iters, seed, X):
    prob = _lib.make_problem(dims, k, p, q, iters, 0.0, seed)
    A = [torch.full((d, k), float("nan"), dtype=torch.float32, device="cuda") for d in dims]
    lam = torch.full((k,), float("nan"), dtype=torch.float32, device="cuda")
    info = torch.zeros(ctypes.sizeof(_lib.AlsInfo), dtype=torch.uint8, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.rcp_decompose_noalloc(ctypes.byref(prob), ctypes.c_void_p(X.data_ptr()),
                                   _lib.ptr_array([a.data_ptr() for a in A]),
                                   ctypes.c_void_p(lam.data_ptr()),
                                   ctypes.c_void_p(info.data_ptr()), stream)
    return st, A, lam, info


def test_noalloc_matches_planned_decompose_twice():
    lib = _lib.load()
    cases = [((120, 100, 80), 6, 10, 2, 30, 5, 71),      # larger first
             ((60, 50, 40), 4, 6, 1, 20, 9, 72)]         # then smaller: stale scratch contents
    for dims, k, p, q, iters, seed, dseed in cases:
        w = synth.low_rank(dims, k, 0.05, dseed)
        X = torch.from_numpy(w.X).cuda()
        st, A, lam, info = _noalloc(lib, dims, k, p, q, iters, seed, X)
        assert st == _lib.RCP_OK, _lib.load().rcp_status_string(st)
        torch.cuda.synchronize()
        plan = rcpgpu.Plan(dims, k, p, q, iters, 0.0, seed)
        lam_r, A_r, info_r = plan.decompose(X)
        torch.cuda.synchronize()
        got = rcpgpu.Plan.read_info(info)
        ref = rcpgpu.Plan.read_info(info_r)
        print(f"[noalloc] {dims}: rel_err {got['rel_err']:.9f} planned {ref['rel_err']:.9f}",
              flush=True)
        assert got["iters"] == ref["iters"] == iters
        assert got["status"] == ref["status"]
        assert abs(got["rel_err"] - ref["rel_err"]) <= 1e-7
        np.testing.assert_allclose(lam.cpu().numpy(), lam_r.cpu().numpy(), rtol=1e-6)
        for a, b in zip(A, A_r):
            np.testing.assert_allclose(a.cpu().numpy(), b.cpu().numpy(), atol=1e-6)


def test_noalloc_refuses_problems_beyond_the_scratch_array():
    lib = _lib.load()
    dims = (400, 400, 400)
    prob = _lib.make_problem(dims, 20, 10, 2, 10, 0.0, 1)
    need = ctypes.c_size_t(0)
    assert lib.rcp_workspace_size(ctypes.byref(prob), ctypes.byref(need)) == _lib.RCP_OK
    assert need.value > _lib.RCP_NOALLOC_SCRATCH_BYTES
    X = torch.zeros(dims, dtype=torch.float32, device="cuda")
    st, _, _, _ = _noalloc(lib, dims, 20, 10, 2, 10, 1, X)
    assert st == _lib.RCP_ERR_WORKSPACE
