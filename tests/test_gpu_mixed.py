"""16-bit operand precisions of the range finder's contractions (bfloat16,
float16; float32 accumulation) against the float64 oracle.  The kernels'
16-bit paths are exercised directly through the two-pass mode product (the
Z = T_(n)^T Q product of the power iteration), and through the sketch;
rcp_compress itself keeps float32 operands in every precision.

Tolerances come from the rounding of both operands to the 16-bit format
(relative error u16 = 2^-9 for bfloat16, 2^-12 for float16, each):
  * rcp_compress in a 16-bit plan equals the float32 result (<= 1e-5 of the
    max), since the core keeps float32 operands;
  * bases: the oracle's signal directions lie in span(Q) (residual of the
    projection <= 40 u16), Q orthonormal to 1e-5 (the QR is float64);
  * end to end: relative error within 1e-4 of the oracle's and congruence
    >= 0.999, the acceptance rule for mixed against float32.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from oracle import evaluate, rcp  # noqa: E402
from paper_1703_09074_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

U16 = {"bf16": 2.0 ** -9, "fp16": 2.0 ** -12}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("shape,mode", [((37, 50, 41), 0), ((37, 50, 41), 2), ((64, 48, 5), 1),
                                        ((700, 9, 40), 0), ((30, 11, 3, 7), 3)])
def test_mixed_plan_compress_is_fp32(prec, shape, mode):
    T = np.random.default_rng(3 + mode).standard_normal(shape).astype(np.float32)
    I = shape[mode]
    l = min(8, I)
    Qn = np.linalg.qr(np.random.default_rng(mode).standard_normal((I, l)))[0].astype(np.float32)
    k = min(2, min(shape))
    plan = rcpgpu.Plan(shape, k, 8 - k, 0, 1, 0.0, 1, precision=prec)
    out = _np(plan.compress(_dev(T), mode, _dev(Qn)))
    want = rcp.mode_product(T.astype(np.float64), Qn.astype(np.float64).T, mode)
    assert np.max(np.abs(out - want)) <= 1e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("dims,mode,q", [((120, 90, 70), 0, 1), ((120, 90, 70), 2, 2),
                                         ((600, 20, 30), 0, 1)])
def test_mixed_sketch_captures_signal(prec, dims, mode, q):
    R = 6
    w = synth.low_rank(dims, R, 0.01, 21 + mode)
    plan = rcpgpu.Plan(dims, R, 6, q, 1, 0.0, 5, precision=prec)
    Q = _np(plan.sketch(_dev(w.X), mode))
    l = rcp.sketch_width(R, 6, dims[mode])
    np.testing.assert_allclose(Q.T @ Q, np.eye(l), atol=1e-5)
    ref = rcp.range_finder(w.X.astype(np.float64), mode, l, q, 5).Q
    S = ref[:, :R]
    resid = np.max(np.abs(S - Q @ (Q.T @ S)))
    assert resid <= 40.0 * U16[prec], resid


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("name", ["rcp100", "rcp400"])
def test_mixed_end_to_end(prec, name):
    cfg = synth.WORKLOADS[name]
    w = synth.make(name)
    X = _dev(w.X)
    lam, A, info = rcpgpu.decompose(X, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0,
                                    cfg["seed"], precision=prec)
    ref = rcp.rcp_als(w.X.astype(np.float64), cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0,
                      cfg["seed"])
    e_ref = evaluate.relative_error(w.X, ref.lam, ref.factors)
    e_gpu = evaluate.relative_error(w.X, _np(lam), [_np(a) for a in A])
    cong = evaluate.congruence([_np(a) for a in A], ref.factors)[0]
    print(f"[mixed] {name} {prec}: rel_err gpu {e_gpu:.7f} oracle {e_ref:.7f} congruence {cong:.6f}")
    assert abs(e_gpu - e_ref) <= 1e-4, (e_gpu, e_ref)
    assert cong >= 0.999, cong
