"""Benchmark of the CHW transform on one MI355X.

Default workload: 1024 float32 signals of 2^20 elements (orthonormal), the
size the headline metric is quoted on; beside it, the BF16 ragged form (20000
signals with log2 sizes in [6, 20], 2^30 elements, one graph replay).

A step is one whole transform of the batch (every pass), inputs resident in
HBM.  Prints ONE JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CHW Gelem/s + % HBM peak, n=2^20 batch; plain FP32 vs BF16 ragged form"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(x_host, m, sample):
    """The oracle (plain C, float64) on the first `sample` signals, all cores."""
    from oracle import c_oracle
    threads = len(os.sched_getaffinity(0))
    xs = x_host[:sample].astype(np.float64)
    t0 = time.perf_counter()
    c_oracle.chw_rows(xs, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample * (1 << m) / dt / 1e9, 5), "unit": "Gelem/s",
            "cores": threads, "kind": "oracle",
            "sample": "%d of the %d signals of 2^%d, float64 plain-C cascade, %.2f s"
                      % (sample, x_host.shape[0], m, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tune", action="store_true", help="autotune the plan first")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--workload", default="plain_2p20_f32",
                    help="plain_2p20_f32 (headline) or, for profiling only: "
                         "plain_2p24_f32, precision_bf16, precision_f16, diff_f32, "
                         "plain_small_f32, ragged_f32, ragged_bf16")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also time a plain device copy of this many GiB (calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the batch shards across GPUs with no communication; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from oracle import c_oracle, metrics
    from paper_1609_06641_amd import chw

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.workload != "plain_2p20_f32":
        run_other(args, dev, stream)
        return

    # ---- headline workload: 1024 x 2^20 float32 ------------------------------
    w = workloads.CONFIGS["plain_2p20_f32"]
    m, batch = 20, w.batch
    t0 = time.perf_counter()
    x_host = workloads.float_signals(w.seed, batch, m)
    log("generated %d x 2^%d in %.1f s" % (batch, m, time.perf_counter() - t0))
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty_like(x)
    plan = chw.Plan([m] * batch, dtype="f32")
    if args.tune:
        plan.autotune(x, y, iters=2)
    fwd = lambda: plan.forward(x, out=y)  # noqa: E731
    ms = time_steps(fwd, args.steps, args.warmup, stream)
    elems = batch << m
    gelem = elems / (ms / 1e3) / 1e9
    desc = plan.describe()["plan"]
    algo_bytes = elems * 8
    achieved = algo_bytes / (ms / 1e3) / 1e9
    log("plain f32: %.3f ms/step, %.1f Gelem/s, %.1f GB/s algorithmic" % (ms, gelem, achieved))

    # parity spot check on sampled signals
    torch.cuda.synchronize()
    idx = [0, batch // 3, batch - 1]
    ref = c_oracle.chw_rows(x_host[idx].astype(np.float64), threads=8)
    got = y[idx].double().cpu().numpy()
    rel = float(np.max(metrics.rel_l2(got, ref)))

    out = {
        "metric": METRIC, "value": round(gelem, 3), "unit": "Gelem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain_2p20_f32", "batch": batch, "log2_n": m,
                   "norm": "orthonormal", "plan": desc["config"], "splits": desc["splits"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "kernel": "whole transform (all launches of one step)",
                     "algorithmic_bytes": algo_bytes},
        "parity": {"sampled_signals": idx, "max_rel_l2": rel},
    }
    del x, y
    torch.cuda.empty_cache()

    # ---- BF16 ragged form --------------------------------------------------
    if not args.no_ragged:
        ks = workloads.ragged_log2_sizes(4001)
        offs = workloads.packed_offsets(ks)
        xr = workloads.ragged_values(4002, ks, offs)
        xb = workloads.to_half_precision(xr, "bf16").to(dev)
        yb = torch.empty_like(xb)
        rp = chw.Plan(ks, dtype="bf16", offsets=offs, graph=True)
        ws = torch.empty(max(rp.workspace_size(), 16), dtype=torch.uint8, device=dev)
        rf = lambda: rp.forward(xb, out=yb, workspace=ws)  # noqa: E731
        rms = time_steps(rf, args.steps, args.warmup, stream)
        relems = int(offs[-1])
        out["bf16_ragged"] = {"value": round(relems / (rms / 1e3) / 1e9, 3), "unit": "Gelem/s",
                              "ms_per_step": round(rms, 4), "signals": len(ks),
                              "elements": relems,
                              "algorithmic_GBs": round(relems * 4 / (rms / 1e3) / 1e9, 1)}
        log("bf16 ragged: %.3f ms/step" % rms)
        del xb, yb, ws
        torch.cuda.empty_cache()

    if args.copy_gib > 0:
        out["copy_calibration"] = copy_calibration(args, dev, stream)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(x_host, m, min(args.cpu_sample, batch))
    print(json.dumps(out), flush=True)


def copy_calibration(args, dev, stream):
    """Time a plain device-to-device copy of known size (read + write bytes)."""
    import torch
    n = int(args.copy_gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    ms = time_steps(lambda: b.copy_(a), max(3, args.steps), 2, stream)
    res = {"bytes_per_copy": 8 * n, "ms": round(ms, 4),
           "GBs": round(8 * n / (ms / 1e3) / 1e9, 1)}
    del a, b
    return res


def run_other(args, dev, stream):
    """Profiling entry for the other workloads (one JSON line, no headline)."""
    import torch
    import workloads
    from paper_1609_06641_amd import chw
    w = workloads.CONFIGS[args.workload]
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
           "i32": torch.int32}[w.dtype]
    if w.name.startswith("ragged"):
        ks = workloads.ragged_log2_sizes(4001)
        offs = workloads.packed_offsets(ks)
        xv = torch.from_numpy(workloads.ragged_values(w.seed, ks, offs))
        plan = chw.Plan(ks, dtype=w.dtype, offsets=offs, graph=True)
        elems = int(offs[-1])
    else:
        m = w.log2_sizes[0]
        if w.dtype in ("bf16", "f16"):
            xv = torch.from_numpy(workloads.outlier_signals(w.seed, w.batch, m))
        elif w.dtype == "i32":
            xv = torch.from_numpy(workloads.int_signals(w.seed, w.batch, m))
        else:
            xv = torch.from_numpy(workloads.float_signals(w.seed, w.batch, m))
        plan = chw.Plan([m] * w.batch, dtype=w.dtype, norm=w.norm)
        elems = w.batch << m
    x = xv.reshape(-1).to(tdt).to(dev)
    y = torch.empty_like(x)
    ws = torch.empty(max(plan.workspace_size(), 16), dtype=torch.uint8, device=dev)
    if args.tune:
        plan.autotune(x, y, workspace=ws, iters=2)
    ms = time_steps(lambda: plan.forward(x, out=y, workspace=ws), args.steps, args.warmup, stream)
    es = x.element_size()
    out = {"workload": w.name, "ms_per_step": round(ms, 4),
           "Gelem_s": round(elems / (ms / 1e3) / 1e9, 2),
           "algorithmic_GBs": round(2 * es * elems / (ms / 1e3) / 1e9, 1),
           "plan": plan.describe()["plan"]["config"]}
    if args.copy_gib > 0:
        out["copy_calibration"] = copy_calibration(args, dev, stream)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
