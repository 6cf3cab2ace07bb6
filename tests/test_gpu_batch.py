"""Batches of independent problems (rcp_batch_*): uneven shapes, ranks and
seeds in one unit of work, CP-ALS and the back-projection in one launch each.

  * every problem of a batch gets exactly what rcp_decompose gives it alone
    (the same kernels and arithmetic);
  * every problem matches the float64 oracle (relative error within 1e-4,
    congruence >= 0.999);
  * on a non-default stream the batch is recorded in a HIP graph: three
    replays, with eager PyTorch work and synchronisations between them, each
    equal the directly enqueued batch.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from oracle import evaluate, rcp  # noqa: E402
from paper_1703_09074_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _problems(count, seed, lo, hi, iters):
    probs, tensors = [], []
    for dims, R, dseed in synth.batch_problems(count, seed, lo=lo, hi=hi, rlo=3, rhi=8):
        w = synth.low_rank(dims, R, 0.05, dseed)
        probs.append(dict(dims=dims, k=R, p=10, q=2, max_iters=iters, seed=dseed % 9973))
        tensors.append(w.X)
    return probs, tensors


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def test_batch_equals_single_and_oracle():
    probs, tensors = _problems(10, 5, 24, 60, 30)
    Xs = [torch.from_numpy(x).cuda() for x in tensors]
    b = rcpgpu.Batch(probs)
    b.decompose(Xs)
    torch.cuda.synchronize()
    infos = b.read_info()
    for i, (pr, x) in enumerate(zip(probs, tensors)):
        plan = rcpgpu.Plan(pr["dims"], pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0, pr["seed"])
        lam, A, info = plan.decompose(Xs[i])
        torch.cuda.synchronize()
        single = rcpgpu.Plan.read_info(info)
        assert infos[i]["iters"] == pr["max_iters"] and infos[i]["status"] == single["status"]
        assert infos[i]["rho"] == single["rho"], (i, infos[i]["rho"], single["rho"])
        np.testing.assert_array_equal(_np(b.lam[i]), _np(lam))
        for n in range(len(pr["dims"])):
            np.testing.assert_array_equal(_np(b.A[i][n]), _np(A[n]))
        ref = rcp.rcp_als(x.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0,
                          pr["seed"])
        e_ref = evaluate.relative_error(x, ref.lam, ref.factors)
        e_gpu = evaluate.relative_error(x, _np(b.lam[i]), [_np(a) for a in b.A[i]])
        cong = evaluate.congruence([_np(a) for a in b.A[i]], ref.factors)[0]
        assert abs(e_gpu - e_ref) <= 1e-4, (i, e_gpu, e_ref)
        assert cong >= 0.999, (i, cong)


def test_batch_graph_replays():
    probs, tensors = _problems(6, 9, 20, 48, 20)
    Xs = [torch.from_numpy(x).cuda() for x in tensors]
    eager = rcpgpu.Batch(probs)                 # default stream: no graph
    eager.decompose(Xs)
    torch.cuda.synchronize()
    want_lam = [_np(t) for t in eager.lam]
    want_A = [[_np(a) for a in As] for As in eager.A]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = rcpgpu.Batch(probs)
    for rep in range(3):
        with torch.cuda.stream(s):
            g.decompose(Xs)                     # first call records, then replays
        torch.cuda.synchronize()
        for i in range(len(probs)):
            np.testing.assert_array_equal(_np(g.lam[i]), want_lam[i])
            for n in range(len(probs[i]["dims"])):
                np.testing.assert_array_equal(_np(g.A[i][n]), want_A[i][n])
        # eager work of the program between replays
        for t in g.lam:
            t.zero_()
        for As in g.A:
            for a in As:
                a.fill_(3.0)
        torch.cuda.synchronize()


def test_batch_autotune_keeps_a_valid_shape():
    """The autotuner's chosen launch shape is one of its candidates, and the
    batch solved with it still matches the oracle (graph replays included)."""
    probs, tensors = _problems(8, 13, 24, 64, 25)
    Xs = [torch.from_numpy(x).cuda() for x in tensors]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = rcpgpu.Batch(probs)
        shape = b.autotune(Xs)
    assert shape["streams"] in (4, 8, 16)
    assert shape["workgroups"] >= 64
    assert shape["row_block_rows"] in (64, 128, 256, 512)
    assert shape["ms_per_batch"] > 0.0
    got = []
    for rep in range(2):
        with torch.cuda.stream(s):
            b.decompose(Xs)
        torch.cuda.synchronize()
        got.append([_np(t) for t in b.lam])
    for i, (pr, x) in enumerate(zip(probs, tensors)):
        np.testing.assert_array_equal(got[0][i], got[1][i])
        ref = rcp.rcp_als(x.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0,
                          pr["seed"])
        e_ref = evaluate.relative_error(x, ref.lam, ref.factors)
        e_gpu = evaluate.relative_error(x, _np(b.lam[i]), [_np(a) for a in b.A[i]])
        cong = evaluate.congruence([_np(a) for a in b.A[i]], ref.factors)[0]
        assert abs(e_gpu - e_ref) <= 1e-4, (i, e_gpu, e_ref)
        assert cong >= 0.999, (i, cong)


def test_batch_bf16_subset_of_the_large_batch_matches_oracle():
    """A seeded subset of the 512-problem workload (modes U{32..256}, R
    U{4..16}, noise 0.05, k = R, p = 10, q = 2, 50 sweeps, bfloat16 range
    finder): every problem within 1e-4 of the float64 oracle's relative
    error, congruence >= 0.999; the error difference is printed per problem."""
    shapes = synth.batch_problems(512, 20170331, lo=32, hi=256, rlo=4, rhi=16)
    pick = [shapes[i] for i in range(0, 512, 43)]                # 12 problems
    probs, tensors = [], []
    for dims, R, dseed in pick:
        w = synth.low_rank(dims, R, 0.05, dseed)
        probs.append(dict(dims=list(dims), k=R, p=10, q=2, max_iters=50, seed=dseed % 100003,
                          precision="bf16"))
        tensors.append(w.X)
    Xs = [torch.from_numpy(x).cuda() for x in tensors]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b = rcpgpu.Batch(probs)
        b.decompose(Xs)
    torch.cuda.synchronize()
    infos = b.read_info()
    worst = 0.0
    for i, (pr, x) in enumerate(zip(probs, tensors)):
        assert infos[i]["status"] == 0 and infos[i]["iters"] == 50, infos[i]
        assert b.read_status(i) == 0
        ref = rcp.rcp_als(x.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0,
                          pr["seed"])
        e_ref = evaluate.relative_error(x, ref.lam, ref.factors)
        e_gpu = evaluate.relative_error(x, _np(b.lam[i]), [_np(a) for a in b.A[i]])
        cong = evaluate.congruence([_np(a) for a in b.A[i]], ref.factors)[0]
        print(f"[batch-bf16] {pr['dims']} R={pr['k']}: rel_err gpu {e_gpu:.7f} oracle {e_ref:.7f} "
              f"diff {e_gpu - e_ref:+.2e} congruence {cong:.6f}", flush=True)
        worst = max(worst, abs(e_gpu - e_ref))
        assert abs(e_gpu - e_ref) <= 1e-4, (i, e_gpu, e_ref)
        assert cong >= 0.999, (i, cong)
    print(f"[batch-bf16] max |rel_err diff| {worst:.2e}", flush=True)
