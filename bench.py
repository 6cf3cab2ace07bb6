"""Benchmark: randomized CP solves per second on one MI355X.

One step = one whole decomposition (rcp_decompose): the randomized range
finder on every mode with in-kernel Gaussian test matrices, q power
iterations, the chained mode products down to the core, CP-ALS on the core
and the back-projection, from X resident in HBM to (lambda, A_n) in HBM.

Default workload (rcp2048, the largest single-GPU configuration): a dense
2048 x 2048 x 512 float32 tensor (8 GiB), rank 50 with factors N(0,1), noise
0.1 rms; k = 50, p = 10, q = 2, 100 ALS sweeps.  Secondary lines: the
400 x 400 x 400 workload (rank 20, log-uniform weights, noise 0.05, k = 20,
p = 10, q = 2, 100 sweeps), the bfloat16 range finder on the same tensor,
the 4-way float16 configuration and the batch of 512 small problems.

Prints one JSON line.  Besides the throughput it reports, for the kernel
class that takes the most time, the achieved algorithmic rate against the
MI355X peak (HIP events around that kernel's launches on the plan's stream),
every kernel class's totals, and the CPU oracle timed on this host on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_MFMA_TFLOPS = 78.6
N_CU = 256

STREAMING = ("sketch", "power", "contract_in", "contract_out")

# kernel class -> (binding roofline, peak, unit, counted quantity, kernel symbol,
# workgroups per launch: None = grid-wide)
ROOFLINES = {
    "sketch": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_contract_out (generated Omega)", None),
    "power": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_power_fused", None),
    "contract_in": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_power_fused (resident-Q mode product)", None),
    "contract_out": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_contract_out", None),
    "reduce": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_reduce", None),
    "qr": ("mfma", PEAK_FP64_MFMA_TFLOPS, "TFLOP/s", "flops", "k_qr", 1),
    "als": ("mfma", PEAK_FP32_MFMA_TFLOPS, "TFLOP/s", "flops", "k_als", 1),
    "expand": ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", "k_expand_raw/finish", None),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rcp2048")
    ap.add_argument("--secondary", default="rcp400",
                    help="a second workload timed after the headline one ('' skips)")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--concurrent", type=int, default=6, metavar="S",
                    help="also time independent solves on S streams (0 skips)")
    ap.add_argument("--batch", type=int, default=512, metavar="COUNT",
                    help="also time a batch of COUNT independent small problems (0 skips)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-autotune", type=int, default=1,
                    help="time the batch again with the launch shape rcp_batch_autotune picks")
    ap.add_argument("--mixed-steps", type=int, default=10,
                    help="timed solves with bfloat16 and float16 operands (0 skips the comparison)")
    ap.add_argument("--mixed-large-steps", type=int, default=2,
                    help="timed solves per precision of the large mixed-precision workloads (0 skips)")
    ap.add_argument("--validation-runs", type=int, default=100,
                    help="runs per point of the Theorem 1 and SNR sweeps (0: skip)")
    ap.add_argument("--det-steps", type=int, default=2,
                    help="timed runs of deterministic CP-ALS on the secondary workload (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="CPU oracle sample budget (0 disables the cpu_baseline leg)")
    ap.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "traffic.json"),
                    help="HBM traffic per launch measured with rocprofv3 counters")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (reference "
                         "reading for the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "launches": 3}),
          flush=True)


def _cores():
    threads = os.environ.get("OMP_NUM_THREADS") or os.environ.get("OPENBLAS_NUM_THREADS")
    cores = len(os.sched_getaffinity(0))
    return int(threads) if threads and threads.isdigit() else cores


def cpu_baseline(X, cfg, budget_s):
    """The float64 oracle, unmodified, on this host: whole solves of the same
    workload until the budget is spent (at least one)."""
    from oracle import rcp
    X64 = X.astype(np.float64)
    n = 0
    rel_err = None
    t0 = time.perf_counter()
    while True:
        r = rcp.rcp_als(X64, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"])
        if rel_err is None:
            rel_err = float(np.sqrt(max(0.0, 1.0 - r.rho)))
        n += 1
        if time.perf_counter() - t0 >= budget_s or n >= 20:
            break
    dt = time.perf_counter() - t0
    return ({"value": n / dt, "unit": "solves/s", "cores": _cores(), "kind": "oracle",
             "sample": f"{n} whole solve(s) of the same workload in float64 NumPy/SciPy ({dt:.1f} s)"},
            rel_err)


def cpu_baseline_sampled(X_dev, cfg, slices):
    """The float64 oracle, unmodified, on a bounded sample of a tensor too
    large to solve on the host within the bench: the sub-tensor of the first
    ``slices`` indices of the last mode (same leading modes, same k, p, q,
    sweeps and seed).  Its compression (Algorithm 1) is timed and scaled by
    the element-count ratio to the whole tensor, since every pass streams the
    tensor once; CP-ALS on its core (the same core size as the whole tensor's
    while slices >= k + p) is timed as it is."""
    from oracle import rcp
    sub = X_dev[..., :slices].contiguous().cpu().numpy()
    S_full = float(np.prod(cfg["dims"]))
    S_sub = float(sub.size)
    t0 = time.perf_counter()
    X64 = sub.astype(np.float64)
    normX2 = float(np.dot(X64.ravel(), X64.ravel()))
    comp = rcp.compress(X64, cfg["k"], cfg["p"], cfg["q"], cfg["seed"])
    t_comp = time.perf_counter() - t0
    del X64
    t1 = time.perf_counter()
    res = rcp.als(comp.core, cfg["k"], cfg["iters"], 0.0, normX2=normX2)
    rcp.expand(comp.Q, res.factors, res.lam)
    t_als = time.perf_counter() - t1
    t_solve = t_comp * S_full / S_sub + t_als
    dims = list(cfg["dims"])
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": _cores(), "kind": "oracle",
            "sample": (f"oracle rcp_als stages on the sub-tensor {dims[:-1] + [slices]} "
                       f"(first {slices} of {dims[-1]} last-mode slices): compression "
                       f"{t_comp:.2f} s scaled by {S_full / S_sub:.0f} (element ratio) + ALS and "
                       f"expand on its core {t_als:.2f} s = {t_solve:.1f} s per solve")}


def batch_workload(count, seed=20170331):
    """The batched workload: `count` independent 3-way tensors, every mode size
    uniform on [32, 256], true rank R uniform on [4, 16], factors N(0,1),
    noise 0.05 rms; k = R, p = 10, q = 2, 50 sweeps, bfloat16 range finder."""
    from paper_1703_09074_amd import synth
    probs = []
    for dims, R, dseed in synth.batch_problems(count, seed, lo=32, hi=256, rlo=4, rhi=16):
        probs.append(dict(dims=list(dims), k=R, p=10, q=2, max_iters=50, seed=dseed % 100003,
                          precision="bf16", R=R, data_seed=dseed))
    return probs


def run_batch(args, torch, rcpgpu, dev):
    from paper_1703_09074_amd import synth
    probs = batch_workload(args.batch)
    Xs = []
    for pr in probs:
        X, _, _, _ = synth.low_rank_device(pr["dims"], pr["R"], 0.05, pr["data_seed"], device=dev)
        Xs.append(X)
    elems = sum(int(np.prod(pr["dims"])) for pr in probs)
    s = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        b = rcpgpu.Batch([{k: v for k, v in pr.items() if k not in ("R", "data_seed")} for pr in probs],
                         device=dev)
        t0 = time.perf_counter()
        b.decompose(Xs)                       # records the graph and runs it once
    torch.cuda.synchronize()
    first = time.perf_counter() - t0
    def timed_batches():
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(s):
            e0.record(s)
            for _ in range(args.batch_steps):
                b.decompose(Xs)
            e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.batch_steps

    ms_default = timed_batches()
    tune = None
    if args.batch_autotune:
        # the launch shape chosen by the library's autotuner, then timed again
        with torch.cuda.stream(s):
            tune = b.autotune(Xs)
            b.decompose(Xs)                   # records the graph with the chosen shape
        torch.cuda.synchronize()
        ms = timed_batches()
    else:
        ms = ms_default
    infos = b.read_info()
    errs = [i["rel_err"] for i in infos]
    out = {"problems": args.batch, "elements": elems, "ms_per_batch": ms,
           "solves_per_s": args.batch * 1000.0 / ms, "first_call_s_with_graph_recording": first,
           "ms_per_batch_default_shape": ms_default, "autotuned_shape": tune,
           "rel_err_mean": float(np.mean(errs)), "rel_err_max": float(np.max(errs)),
           "status_nonzero": int(sum(1 for i in infos if i["status"] != 0)),
           "workload": "3-way tensors, modes U{32..256}, R U{4..16}, noise 0.05, k=R, p=10, q=2, "
                       "50 sweeps, bf16 range finder"}
    if args.cpu_seconds > 0:
        # the oracle on a bounded sample of the same problems
        from oracle import rcp
        n, t0, diffs = 0, time.perf_counter(), []
        for i, pr in enumerate(probs):
            x = Xs[i].cpu().numpy().astype(np.float64)
            r = rcp.rcp_als(x, pr["k"], pr["p"], pr["q"], pr["max_iters"], 0.0, pr["seed"])
            diffs.append(abs(float(np.sqrt(max(0.0, 1.0 - r.rho))) - errs[i]))
            n += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / dt, "unit": "solves/s",
                               "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"the first {n} problems of the batch in float64 ({dt:.1f} s)",
                               "max_abs_rel_err_diff_vs_gpu": float(max(diffs))}
    return out


# The mixed-precision configurations: 2048 x 2048 x 512 with a bfloat16 range
# finder, 256 x 256 x 256 x 64 with a float16 one, each against float32 on the
# same tensor (built on the GPU from the seeded recipe).
MIXED_LARGE = (("rcp2048", "bf16"), ("rcp4way", "fp16"))


def mixed_large(args, torch, rcpgpu, dev, skip=None):
    from paper_1703_09074_amd import synth
    out = {}
    for name, prec in MIXED_LARGE:
        if name == skip:
            continue
        cfg = dict(synth.WORKLOADS[name])
        dims = list(cfg["dims"])
        X, _, _, _ = synth.low_rank_device(dims, cfg["R"], cfg["noise"], cfg["data_seed"],
                                           kind=cfg["kind"], device=dev)
        res = {}
        for p in ("fp32", prec):
            plan = rcpgpu.Plan(dims, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"],
                               device=dev, precision=p)
            A = [torch.empty((d, cfg["k"]), dtype=torch.float32, device=dev) for d in dims]
            lam = torch.empty((cfg["k"],), dtype=torch.float32, device=dev)
            info = plan._info_buffer()
            plan.decompose_into(X, A, lam, info)
            torch.cuda.synchronize()
            stream = torch.cuda.current_stream(dev)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.mixed_large_steps):
                plan.decompose_into(X, A, lam, info)
            e1.record(stream)
            torch.cuda.synchronize()
            res[p] = (e0.elapsed_time(e1) / args.mixed_large_steps, rcpgpu.Plan.read_info(info)["rel_err"])
            del plan, A, lam, info
        (t32, e32), (tlp, elp) = res["fp32"], res[prec]
        out[name] = {"precision": prec, "ms_per_solve_fp32": t32, "ms_per_solve_mixed": tlp,
                     "speedup_vs_fp32": t32 / tlp, "rel_err_fp32": e32, "rel_err_mixed": elp,
                     "equal_error": abs(elp - e32) <= 1e-4,
                     "note": "float32 run's parity with the oracle: tests/test_gpu_fullsize.py"}
        del X
        torch.cuda.empty_cache()
    return out


def measure(torch, rcpgpu, dev, name, X, precision, steps, warmup, profile_steps, traffic_json):
    """Timed solves of one workload: throughput, per-kernel-class totals, the
    dominant class's roofline line and the streaming passes' rates."""
    from paper_1703_09074_amd import synth
    cfg = dict(synth.WORKLOADS[name])
    dims = list(cfg["dims"])
    plan = rcpgpu.Plan(dims, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"],
                       device=dev, precision=precision)
    A = [torch.empty((d, cfg["k"]), dtype=torch.float32, device=dev) for d in dims]
    lam = torch.empty((cfg["k"],), dtype=torch.float32, device=dev)
    info = plan._info_buffer()
    for _ in range(warmup):
        plan.decompose_into(X, A, lam, info)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.decompose_into(X, A, lam, info)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    res = rcpgpu.Plan.read_info(info)
    out = {"ms_per_step": ms, "value": 1000.0 / ms, "wall_s": wall, "rel_err": res["rel_err"],
           "status": res["status"], "iters": res["iters"]}
    if profile_steps <= 0:
        return out, plan
    # per-kernel timing (separate pass with an event pair around every launch)
    plan.profile(True)
    for _ in range(profile_steps):
        plan.decompose_into(X, A, lam, info)
    torch.cuda.synchronize()
    kern = plan.profile_read()
    plan.profile(False)
    for v in kern.values():
        v["ms_per_launch"] = v["ms"] / v["launches"]
        v["bytes_per_launch"] = v["bytes"] / v["launches"]
        v["flops_per_launch"] = v["flops"] / v["launches"]
        v["ms_per_step"] = v["ms"] / profile_steps
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    bound, peak, unit, qty, kname, wgs = ROOFLINES.get(
        dom, ("hbm", PEAK_HBM_GBS, "GB/s", "bytes", dom, None))
    if dom in STREAMING:
        # a contraction is bound by HBM or by the matrix cores, whichever its
        # arithmetic intensity (flops per byte) against the machine balance says
        ai = d["flops"] / d["bytes"]
        mpeak = PEAK_FP32_MFMA_TFLOPS if precision == "fp32" else 2500.0
        if ai > mpeak * 1e12 / (PEAK_HBM_GBS * 1e9):
            bound, peak, unit, qty = "mfma", mpeak, "TFLOP/s", "flops"
    scale = 1e9 if unit == "GB/s" else 1e12
    per_launch = d[qty] / d["launches"]
    ach = per_launch / (d["ms_per_launch"] * 1e-3) / scale
    roof = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "kernel_class": dom, "kernel": kname, "ms_per_launch": d["ms_per_launch"],
            ("flops" if qty == "flops" else "bytes") + "_per_launch": per_launch}
    if wgs == 1:
        # a single-workgroup kernel can use one compute unit's share of the peak
        roof["frac_of_one_cu"] = ach / (peak / N_CU)
    roof["traffic"] = None
    if traffic_json and os.path.exists(traffic_json):
        try:
            tj = json.load(open(traffic_json))
            ent = tj.get(name, {}).get(dom)
            if ent and ent.get("source_hash") == _source_hash(dom):
                roof["traffic"] = ent["bytes_per_launch"]
        except (ValueError, OSError):
            pass
    sb = sum(kern[k]["bytes"] for k in STREAMING if k in kern)
    sf = sum(kern[k]["flops"] for k in STREAMING if k in kern)
    sm = sum(kern[k]["ms"] for k in STREAMING if k in kern)
    mpeak = PEAK_FP32_MFMA_TFLOPS if precision == "fp32" else 2500.0
    out["roofline"] = roof
    out["sketch_ttm"] = {"gbps": sb / (sm * 1e-3) / 1e9, "tflops": sf / (sm * 1e-3) / 1e12,
                         "frac_hbm": sb / (sm * 1e-3) / 1e9 / PEAK_HBM_GBS,
                         "frac_mfma": sf / (sm * 1e-3) / 1e12 / mpeak,
                         "mfma_peak_tflops": mpeak,
                         "ms_per_step": sm / profile_steps} if sm > 0 else None
    out["kernels"] = kern
    return out, plan


def make_input(torch, name, dev):
    from paper_1703_09074_amd import synth
    cfg = dict(synth.WORKLOADS[name])
    dims = list(cfg["dims"])
    if int(np.prod(dims)) <= 100_000_000:
        w_X = synth.make(name).X
        return torch.from_numpy(w_X).to(dev), w_X
    # too large to build on the host quickly: the same recipe assembled on the GPU
    X, _, _, _ = synth.low_rank_device(dims, cfg["R"], cfg["noise"], cfg["data_seed"],
                                       kind=cfg["kind"], device=dev)
    return X, None


def config_of(name):
    from paper_1703_09074_amd import synth
    cfg = dict(synth.WORKLOADS[name])
    return {"workload": name, "dims": list(cfg["dims"]), "R": cfg["R"], "k": cfg["k"],
            "p": cfg["p"], "q": cfg["q"], "als_iters": cfg["iters"], "noise": cfg["noise"],
            "factors": cfg["kind"], "scheme": "sequential", "precision": "fp32"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy > 0:
        calibrate_copy(args.calibrate_copy)
        return

    import torch
    import paper_1703_09074_amd as rcpgpu
    from paper_1703_09074_amd import synth

    name = args.workload
    cfg = dict(synth.WORKLOADS[name])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    X, w_X = make_input(torch, name, dev)
    head, plan = measure(torch, rcpgpu, dev, name, X, "fp32", args.steps, args.warmup,
                         args.profile_steps, args.traffic_json)
    del plan

    # the mixed-precision form of the same workload, at equal error
    mixed = {}
    if args.mixed_steps > 0:
        precs = ("bf16", "fp16") if name in ("rcp100", "rcp400") else \
            (("fp16",) if name.startswith("rcp4way") else ("bf16",))
        for prec in precs:
            m, pl = measure(torch, rcpgpu, dev, name, X, prec, args.mixed_steps, 1,
                            args.profile_steps, None)
            del pl
            mixed[prec] = {"ms_per_step": m["ms_per_step"], "solves_per_s": m["value"],
                           "speedup_vs_fp32": head["ms_per_step"] / m["ms_per_step"],
                           "rel_err": m["rel_err"],
                           "rel_err_minus_fp32": m["rel_err"] - head["rel_err"],
                           "equal_error": abs(m["rel_err"] - head["rel_err"]) <= 1e-4,
                           "sketch_ttm": m.get("sketch_ttm")}

    cpu = None
    oracle_err = None
    if args.cpu_seconds > 0:
        if w_X is not None:
            cpu, oracle_err = cpu_baseline(w_X, cfg, args.cpu_seconds)
        else:
            # a bounded sample: 1/8 of the last mode for the 2048 x 2048 x 512 tensor
            slices = max(cfg["k"] + cfg["p"], cfg["dims"][-1] // 8)
            cpu = cpu_baseline_sampled(X, cfg, slices)
    del X
    torch.cuda.empty_cache()

    secondary = None
    if args.secondary and args.secondary != name:
        sname = args.secondary
        scfg = dict(synth.WORKLOADS[sname])
        X2, w_X2 = make_input(torch, sname, dev)
        sec, splan = measure(torch, rcpgpu, dev, sname, X2, "fp32", args.steps, args.warmup,
                             args.profile_steps, args.traffic_json)
        del splan
        sec["config"] = config_of(sname)
        if args.cpu_seconds > 0 and w_X2 is not None:
            scpu, s_oracle = cpu_baseline(w_X2, scfg, args.cpu_seconds)
            sec["cpu_baseline"] = scpu
            sec["oracle_rel_err"] = s_oracle
            sec["rel_err_minus_oracle"] = sec["rel_err"] - s_oracle
        if args.concurrent > 1:
            sec["concurrent_streams"] = concurrent(args, torch, rcpgpu, dev, sname, X2, sec)
        if args.det_steps > 0:
            sec["deterministic_cp_als"] = deterministic(args, torch, rcpgpu, dev, sname, X2, sec)
        if args.mixed_steps > 0:
            sm = {}
            for prec in ("bf16", "fp16"):
                m, pl = measure(torch, rcpgpu, dev, sname, X2, prec, args.mixed_steps, 1, 0, None)
                del pl
                sm[prec] = {"ms_per_step": m["ms_per_step"],
                            "speedup_vs_fp32": sec["ms_per_step"] / m["ms_per_step"],
                            "rel_err": m["rel_err"], "rel_err_minus_fp32": m["rel_err"] - sec["rel_err"]}
                if "oracle_rel_err" in sec:
                    sm[prec]["valid_at_equal_error"] = bool(
                        abs(sec["rel_err"] - sec["oracle_rel_err"]) <= 1e-4 and
                        abs(m["rel_err"] - sec["oracle_rel_err"]) <= 1e-4)
            sec["mixed_vs_fp32"] = sm
        secondary = {sname: sec}
        del X2
        torch.cuda.empty_cache()

    batched = run_batch(args, torch, rcpgpu, dev) if args.batch > 0 else None
    validation = run_validation(args, torch, dev) if args.validation_runs > 0 else None
    mixed_big = mixed_large(args, torch, rcpgpu, dev, skip=name) if args.mixed_large_steps > 0 else None

    out = {
        "metric": "rCP solves/sec + sketch/TTM TFLOP/s (% peak), mixed vs FP32 at equal rel. error",
        "value": head["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": config_of(name),
        "rel_err": head["rel_err"],
        "wall_s": head["wall_s"],
        "roofline": head.get("roofline"),
        "sketch_ttm": head.get("sketch_ttm"),
        "kernels": head.get("kernels"),
        "mixed_vs_fp32": mixed or None,
        "cpu_baseline": cpu,
        "secondary": secondary,
        "mixed_vs_fp32_large": mixed_big,
        "batched": batched,
        "validation": validation,
    }
    if oracle_err is not None:
        out["oracle_rel_err"] = oracle_err
        out["rel_err_minus_oracle"] = head["rel_err"] - oracle_err
    print(json.dumps(out), flush=True)


def deterministic(args, torch, rcpgpu, dev, name, X, base):
    """Deterministic CP-ALS on the full tensor (the method the paper measures
    the randomized one against) on the same input and sweep count: its time,
    error and the randomized method's speed-up over it; the full-tensor mode
    product's HBM rate from the plan's per-kernel event timing."""
    from paper_1703_09074_amd import synth
    cfg = dict(synth.WORKLOADS[name])
    dims = list(cfg["dims"])
    plan = rcpgpu.Plan(dims, cfg["k"], cfg["p"], 4, cfg["iters"], 0.0, cfg["seed"], device=dev,
                       solver="cp_als")
    A = [torch.empty((d, cfg["k"]), dtype=torch.float32, device=dev) for d in dims]
    lam = torch.empty((cfg["k"],), dtype=torch.float32, device=dev)
    info = plan._info_buffer()
    plan.decompose_into(X, A, lam, info)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.det_steps):
        plan.decompose_into(X, A, lam, info)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.det_steps
    rel = rcpgpu.Plan.read_info(info)["rel_err"]
    plan.profile(True)
    plan.decompose_into(X, A, lam, info)
    prof = plan.profile_read()
    plan.profile(False)
    mt = prof.get("mttkrp", {})
    out = {"ms_per_solve": ms, "rel_err": rel, "rel_err_minus_rcp": rel - base["rel_err"],
           "rcp_speedup": ms / base["ms_per_step"], "sweeps": cfg["iters"],
           "start": "eigenvectors by subspace iteration, q=4",
           "kernels_ms": {k: v["ms"] for k, v in prof.items()}}
    if mt.get("ms"):
        gbs = mt["bytes"] / (mt["ms"] * 1e-3) / 1e9
        out["mttkrp_full"] = {"launches": mt["launches"], "ms": mt["ms"], "GB_per_s": gbs,
                              "frac_hbm": gbs / PEAK_HBM_GBS}
    return out


def run_validation(args, torch, dev):
    """The paper's validation experiments over many runs on the GPU: the
    Theorem 1 bound (50^3 and 50^4, rank 25, p = 2, q = 0) and the error
    against SNR (100^3, rank 50, p = 10, q in {0, 2}, and deterministic
    CP-ALS).  Per point: the means, the bound, the GPU time per run."""
    from paper_1703_09074_amd import sweeps
    runs = args.validation_runs
    t0 = time.perf_counter()
    th = {}
    for dims, ks in (((50, 50, 50), (5, 10, 15, 20)), ((50, 50, 50, 50), (5, 10, 15, 20))):
        r = sweeps.theorem1(dims, 25, ks, runs=runs, p=2, device=dev)
        th["x".join(map(str, dims))] = [
            {k: row[k] for k in ("k", "bound", "mean", "max", "holds", "ms_per_run", "path")}
            for row in r["rows"]]
        torch.cuda.empty_cache()
    t1 = time.perf_counter()
    snr = sweeps.snr_sweep((100, 100, 100), 50, snrs=(1, 2, 4, 8, 16), runs=runs, qs=(0, 2),
                           p=10, iters=50, device=dev)
    torch.cuda.empty_cache()
    t2 = time.perf_counter()
    levels = [{"snr": lev["snr"],
               **{m: {"mean_rel_err": v["mean"], "std": v["std"], "ms_per_run": v["ms_per_run"]}
                  for m, v in lev["methods"].items()}} for lev in snr["levels"]]
    return {"runs": runs, "theorem1": th, "theorem1_s": t1 - t0,
            "snr": {"dims": snr["dims"], "R": snr["R"], "p": snr["p"], "sweeps": snr["iters"],
                    "levels": levels}, "snr_s": t2 - t1,
            "data": "synthetic rank-R tensors, Gaussian factors; noise amplitude rms(clean)/SNR"}


def concurrent(args, torch, rcpgpu, dev, name, X, base):
    """S independent plans, each bound to its own stream: one solve's ALS
    overlaps the next solves' grid-wide streaming passes."""
    from paper_1703_09074_amd import synth
    cfg = dict(synth.WORKLOADS[name])
    dims = list(cfg["dims"])
    S = args.concurrent
    streams = [torch.cuda.Stream(device=dev) for _ in range(S)]
    slots = []
    for st in streams:
        with torch.cuda.stream(st):
            pl = rcpgpu.Plan(dims, cfg["k"], cfg["p"], cfg["q"], cfg["iters"], 0.0, cfg["seed"],
                             device=dev)
            As = [torch.empty((d, cfg["k"]), dtype=torch.float32, device=dev) for d in dims]
            ls = torch.empty((cfg["k"],), dtype=torch.float32, device=dev)
            slots.append((pl, As, ls, pl._info_buffer()))
    torch.cuda.synchronize()
    for pl, As, ls, inf in slots:
        pl.decompose_into(X, As, ls, inf)
    torch.cuda.synchronize()
    total = S * max(2, args.steps // S)
    t0 = time.perf_counter()
    for i in range(total):
        pl, As, ls, inf = slots[i % S]
        pl.decompose_into(X, As, ls, inf)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    errs = [rcpgpu.Plan.read_info(inf)["rel_err"] for _, _, _, inf in slots]
    return {"streams": S, "solves": total, "solves_per_s": total / dt,
            "speedup_vs_one_stream": (total / dt) / base["value"],
            "rel_err_max_abs_diff": max(abs(e - base["rel_err"]) for e in errs),
            "timing": "host wall clock around the issue of all solves and a device sync"}


# the sources each kernel class is compiled from (besides the shared headers)
STREAM_SOURCES = ("stream_kernels.hip", "stream_tiles.h")
# the ALS class also runs the streaming kernels (the Khatri-Rao mode product
# and its reduction of the grid-wide form)
KERNEL_SOURCES = {"als": ("als_kernel.hip", "als_common.h") + STREAM_SOURCES,
                  "qr": ("qr_kernel.hip",), "expand": ("expand_kernel.hip",)}


def _strip_comments(src):
    """C++ source without comments and blank lines (string literals in these
    files hold no comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def _source_hash(kernel_class, read=None):
    """Hash of the code (comments stripped) a kernel class is built from (its
    sources and the shared device headers): stored traffic counts are used
    only while it matches.  ``read(name)`` returns a source's text (default:
    the working tree)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "paper_1703_09074_amd", "csrc")
    if read is None:
        read = lambda f: open(os.path.join(csrc, f), encoding="utf-8").read()  # noqa: E731
    for f in KERNEL_SOURCES.get(kernel_class, STREAM_SOURCES) + ("rcp_device.h", "rcp_kernels.h"):
        h.update(_strip_comments(read(f)).encode("utf-8"))
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
