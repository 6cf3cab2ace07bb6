"""The full-size workloads on the GPU against the float64 oracle, end to end:

  * 2048 x 2048 x 512, R = 50, noise 0.1 rms, k = 50, p = 10, q = 2, 100 sweeps,
    float32 and bfloat16 range-finder operands;
  * 256 x 256 x 256 x 64, R = 30, pairwise factor cosine 0.8, noise 0.05 rms,
    k = 30, p = 15, q = 3 (float32 and float16 range finder) and q = 1
    (float32), 200 sweeps.

The tensors are assembled on the GPU from the seeded recipe and copied back;
the oracle's unmodified ``rcp_als`` decomposes the host copy of the same
buffer (float64, about 3.5x the tensor's float32 size of host memory at its
peak: the float32 copy, its float64 upcast and one unfolding-sized
temporary).  Both results go through the same float64 evaluator
(relative error ||X - Xhat|| / ||X|| computed slab by slab from X) and the
congruence of their factors:

  * |rel_err_gpu - rel_err_oracle| <= 1e-4 and congruence >= 0.999, for
    every precision (a 16-bit range finder only perturbs the bases, which the
    float64 QR re-orthonormalises, so the bar is the float32 one); each
    result's difference from the oracle is printed;
  * every basis is orthonormal to 1e-5.

For 2048 x 2048 x 512 with R = 50, 100 sweeps from the eigenvector start end
at a relative error of about 0.18, above the noise floor of about 0.1, on the
oracle as on the GPU: the parity bar still applies to the stalled fit.
"""
import resource

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1703_09074_amd as rcpgpu  # noqa: E402
from oracle import evaluate, rcp  # noqa: E402
from paper_1703_09074_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

_X = {}        # data seed -> (device tensor, host copy)
_REF = {}      # workload name -> oracle result and its relative error


def _tensor(cfg):
    key = (cfg["data_seed"], tuple(cfg["dims"]))
    if key not in _X:
        _X.clear()
        torch.cuda.empty_cache()
        X, _, _, _ = synth.low_rank_device(list(cfg["dims"]), cfg["R"], cfg["noise"],
                                           cfg["data_seed"], kind=cfg["kind"])
        torch.cuda.synchronize()
        _X[key] = (X, X.cpu().numpy())
    return _X[key]


def _oracle(name, cfg, X_host):
    if name not in _REF:
        print(f"[fullsize] oracle rcp_als on {name} ...", flush=True)
        ref = rcp.rcp_als(X_host, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"])
        e_ref = evaluate.relative_error(X_host, ref.lam, ref.factors)
        rss_gib = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 2 ** 20
        print(f"[fullsize] oracle {name}: rel_err {e_ref:.7f} (fit form {ref.rel_err:.7f}), "
              f"host peak RSS {rss_gib:.1f} GiB", flush=True)
        _REF.clear()
        _REF[name] = (ref, e_ref)
    return _REF[name]


@pytest.mark.parametrize("name,prec", [("rcp2048", "fp32"), ("rcp2048", "bf16"),
                                       ("rcp4way", "fp32"), ("rcp4way", "fp16"),
                                       ("rcp4way_q1", "fp32")])
def test_full_size_matches_oracle(name, prec):
    cfg = synth.WORKLOADS[name]
    dims = list(cfg["dims"])
    k = cfg["k"]
    print(f"[fullsize] {name} {prec} dims {dims} q {cfg['q']}", flush=True)
    X, X_host = _tensor(cfg)
    plan = rcpgpu.Plan(dims, k, cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"], precision=prec)
    A = [torch.empty((d, k), dtype=torch.float32, device="cuda") for d in dims]
    lam = torch.empty((k,), dtype=torch.float32, device="cuda")
    info = plan._info_buffer()
    plan.decompose_into(X, A, lam, info)
    torch.cuda.synchronize()
    res = rcpgpu.Plan.read_info(info)
    assert res["status"] == 0 and res["iters"] == cfg["iters"], res
    for n, b in enumerate(plan.bases()):
        Q = b.cpu().numpy().astype(np.float64)
        err = np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1])))
        assert err <= 1e-5, (n, err)
    lam_h = lam.cpu().numpy().astype(np.float64)
    A_h = [a.cpu().numpy().astype(np.float64) for a in A]
    del plan
    ref, e_ref = _oracle(name, cfg, X_host)
    e_gpu = evaluate.relative_error(X_host, lam_h, A_h)
    cong, cmin, _ = evaluate.congruence(A_h, ref.factors)
    print(f"[fullsize] {name} {prec}: rel_err gpu {e_gpu:.7f} oracle {e_ref:.7f} "
          f"diff {e_gpu - e_ref:+.2e}; congruence mean {cong:.6f} min {cmin:.6f}", flush=True)
    assert abs(e_gpu - e_ref) <= 1e-4, (e_gpu, e_ref)
    assert cong >= 0.999, cong
    # the device-side fit agrees with the evaluator
    assert abs(res["rel_err"] - e_gpu) <= 1e-4, (res["rel_err"], e_gpu)


def teardown_module(module):
    _X.clear()
    _REF.clear()
    torch.cuda.empty_cache()
