"""Benchmark of the CHW transform on one MI355X (gfx950).

Headline workload: 1024 float32 signals of 2^20 elements, orthonormal
dyadic-ordered WHT (the size the metric is quoted on).  Beside it: the BF16
ragged form (20000 signals, log2 sizes in [6, 20], 2^30 elements; one launch
per pass and tile size, replayed as a HIP graph).

A step is one whole transform of the batch (every pass), inputs resident in
HBM.  The timed region is bracketed by device synchronizations; rank 0 (the
only rank) prints ONE JSON line on stdout.

Other modes (not the headline line):
  --workload NAME      profile another workload (one JSON line of its own)
  --summarize ...      turn rocprofv3 outputs into a profiles/ summary
"""

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CHW Gelem/s + % HBM peak, n=2^20 batch; plain FP32 vs BF16 ragged form"
HBM_PEAK_GBS = 8000.0
PROFILE_HEADLINE = os.path.join(ROOT, "profiles", "chw_2p20_f32.md")
# the ragged workload's summary per storage type
PROFILE_RAGGED = {dt: os.path.join(ROOT, "profiles", "chw_ragged_%s.md" % dt) for dt in ("bf16", "f32")}
# the rocprofv3 summary of each other workload's configuration line
CONFIG_PROFILES = {name: os.path.join(ROOT, "profiles", f + ".md") for name, f in (
    ("plain_small_f32", "chw_small_f32_64x2p10"), ("plain_small_i32", "chw_small_i32_64x2p10"),
    ("plain_2p24_f32", "chw_2p24_f32"), ("precision_bf16", "chw_precision_bf16_8192x2p12"),
    ("precision_f16", "chw_precision_f16_8192x2p12"), ("diff_f32", "chw_diff_f32_256x2p14"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRANSFORM_SOURCES = ("chw_engine.h", "chw_layout.h", "chw_types.h", "chw_kernels.inc")


def _code_only(text):
    """C++ source without comments and blank space (the sources hold no string
    literal with comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the code of the transform kernels (comments and layout
    ignored): a stored traffic figure is valid only for the kernels it was
    measured with (and for the same pass splits, which the profile records
    too)."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1609_06641_amd", "csrc", "*"))):
        b = os.path.basename(f)
        if b in TRANSFORM_SOURCES or (b.startswith("chw_kernels_") and b.endswith(".hip")):
            with open(f) as fh:
                h.update(os.path.basename(f).encode())
                h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def stored_profile(path, splits=None):
    """The machine-readable summary of a profiles/ file, or None when it was
    taken with other kernel sources or other pass splits."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    if d.get("source_hash") != kernel_source_hash():
        return None
    if splits is not None and d.get("splits") is not None and d["splits"] != splits:
        return None
    return d


def stored_traffic(path, splits=None):
    """PMC bytes per transform from a profiles/ summary (None when stale)."""
    d = stored_profile(path, splits)
    return None if d is None else d.get("traffic_bytes_per_transform")


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


def launch_breakdown(plan, fn, steps):
    """Per-launch durations (HIP events on the plan's stream), averaged."""
    plan.set_option("timing", 1)
    acc = None
    for _ in range(steps):
        fn()
        t = plan.launch_times()
        acc = np.array(t) if acc is None else acc + np.array(t)
    plan.set_option("timing", 0)
    return [] if acc is None else list(acc / steps)


def roofline(bytes_per_elem, launches_ms, launches, profile, total_elems):
    """Roofline of the dominant kernel (the launch with the longest average
    duration): its algorithmic bytes per launch -- bytes_per_elem (one read and
    one write of an element at the storage type) times the elements the launch
    takes through its part of the transform -- over its average duration;
    `traffic` is the PMC bytes of one dispatch of that kernel.  `transform`
    gives the same for the whole transform (all launches of one call, which
    take total_elems elements through the whole transform)."""
    total_ms = float(sum(launches_ms))
    dom = int(np.argmax(launches_ms)) if launches_ms else 0
    elems = int(total_elems)
    if len(launches) != len(launches_ms):
        # no per-launch timing: the call as one unit
        launches = [{"name": "all launches of one call", "elements": elems, "symbol": None}
                    for _ in launches_ms]
    per_kernel = (profile or {}).get("kernels_traffic_bytes", {})
    dom_l = launches[dom] if launches else {"name": None, "elements": 0, "symbol": None}
    algo_dom = dom_l["elements"] * bytes_per_elem
    achieved = algo_dom / (launches_ms[dom] / 1e3) / 1e9 if launches_ms else 0.0
    t_traffic = None if profile is None else profile.get("traffic_bytes_per_transform")
    t_achieved = elems * bytes_per_elem / (total_ms / 1e3) / 1e9 if total_ms else 0.0
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": per_kernel.get(dom_l.get("key", dom_l["symbol"])) if profile else None,
        "kernel": dom_l["name"],
        "algorithmic_bytes_per_launch": algo_dom,
        "units_per_launch": dom_l["elements"], "bytes_per_unit": bytes_per_elem,
        "launches": [{"kernel": l["name"], "ms": round(t, 4), "elements": l["elements"],
                      "GBs_algorithmic": round(l["elements"] * bytes_per_elem / (t / 1e3) / 1e9, 1)}
                     for l, t in zip(launches, launches_ms)],
        "transform": {
            "achieved": round(t_achieved, 1), "frac": round(t_achieved / HBM_PEAK_GBS, 4),
            "algorithmic_bytes": elems * bytes_per_elem, "ms": round(total_ms, 4),
            "traffic": t_traffic,
            "measured_hbm_frac": None if t_traffic is None else round(
                t_traffic / (total_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
    }


# Planner options for --plan-config-less runs that bypass the tuning file: the
# planner's own choices for the uniform batches; for the ragged form one
# launch per pass replayed as a graph with 2^5 registers.  (The ragged leg
# itself starts from TUNING_FILE, see tuned_ragged_plan.)
BENCH_CONFIG = {"plan": {},
                "ragged": {"exec": 0, "lr12": 5, "lr15": 5, "single15": 1, "split_l1": -1,
                           "stream": 1}}


def configure(plan, args, x, y, ws, key="plan"):
    """Apply --plan-config (a JSON object of planner options, or {"plan": {...},
    "ragged": {...}}), or run the autotuner with --tune, or else apply
    BENCH_CONFIG."""
    if args.tune and not args.plan_config:
        plan.autotune(x, y, workspace=ws, iters=2)
        return
    cfg = json.loads(args.plan_config) if args.plan_config else BENCH_CONFIG
    if "plan" in cfg or "ragged" in cfg:
        cfg = cfg.get(key, {})
    for k in ("exec", "lr12", "lr15", "single15", "split_l1", "chunk", "stream", "pipeline",
              "turn", "adjoint", "spread"):
        if k in cfg:
            plan.set_option(k, int(cfg[k]))


def plan_launches(plan, dt_code, direction="forward"):
    """The launches of one call in order: a readable name, the kernel's symbol
    as rocprofv3 prints it, and the elements the launch takes through its part
    of the transform."""
    d = plan.describe()["plan"]
    order = d["config"]["order"]
    out = []
    if d["tiny"]:
        out.append({"name": "chw_tiny_kernel", "elements": d["tiny_elements"], "symbol": None})
    kinds = {1: "BLOCKS", 2: "FIRST_A", 3: "FIRST_B", 4: "LAST", 5: "FIRST_C", 8: "TURN", 9: "FIRST_D"}
    adj = "true" if direction == "backward" else "false"
    for r in d[direction]:
        ca = 7 if r["K"] == 15 else 6
        if r["persistent"]:
            name = "chw_persistent_kernel<K=%d,LR=%d>" % (r["K"], r["LR"])
            sym = "void chw::chw_persistent_kernel<%d, %d, %d, %d, 3, %s>(chw::LaunchArgs)" % (
                dt_code, r["K"], r["LR"], ca, adj)
        elif r.get("stream"):
            name = "chw_stream_kernel<K=%d,LR=%d,%s>" % (r["K"], r["LR"], kinds[r["stream"]])
            sym = "void chw::chw_stream_kernel<%d, %d, %d, %d, 3, %s, %d>(chw::LaunchArgs)" % (
                dt_code, r["K"], r["LR"], ca, adj, r["stream"] - 1)
        else:
            name = "chw_items_kernel<K=%d,LR=%d>" % (r["K"], r["LR"])
            sym = "void chw::chw_items_kernel<%d, %d, %d, %d, 3, %s, %d>(chw::LaunchArgs)" % (
                dt_code, r["K"], r["LR"], ca, adj, order)
        out.append({"name": "%s items [%d,%d)" % (name, r["begin"], r["end"]),
                    "elements": r["elements"], "symbol": sym})
    for l, k in zip(out, launch_keys(out)):
        l["key"] = k
    return out


def launch_keys(launches):
    """Profile key of each launch of a call: its kernel symbol, with "#j" for
    the j-th launch of a symbol the call launches more than once (the
    summaries keep those launches apart by their order within the call)."""
    count, seen, keys = {}, {}, []
    for l in launches:
        count[l["symbol"]] = count.get(l["symbol"], 0) + 1
    for l in launches:
        s = l["symbol"]
        j = seen.get(s, 0)
        seen[s] = j + 1
        keys.append(s if s is None or count[s] == 1 else "%s#%d" % (s, j))
    return keys


def launch_names(plan, direction="forward"):
    return [l["name"] for l in plan_launches(plan, 0, direction)]


def cpu_baseline(x_host, m, sample):
    """The oracle (plain C, float64) on the first `sample` signals, all cores."""
    from oracle import c_oracle
    threads = len(os.sched_getaffinity(0))
    xs = x_host[:sample].astype(np.float64)
    t0 = time.perf_counter()
    c_oracle.chw_rows(xs, threads=threads)
    dt = time.perf_counter() - t0
    one = min(32, sample)
    t0 = time.perf_counter()
    c_oracle.chw_rows(xs[:one], threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": round(sample * (1 << m) / dt / 1e9, 5), "unit": "Gelem/s",
            "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": "%d of the %d signals of 2^%d, float64 plain-C cascade, %.2f s"
                      % (sample, x_host.shape[0], m, dt),
            "single_thread": {"value": round(one * (1 << m) / dt1 / 1e9, 5),
                              "unit": "Gelem/s", "cores": 1,
                              "sample": "%d signals of 2^%d, %.2f s" % (one, m, dt1)}}


def copy_calibration(gib, dev, stream, steps):
    """Time a plain device-to-device copy of known size (read + write bytes)."""
    import torch
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    ms = time_steps(lambda: b.copy_(a), max(3, steps), 2, stream)
    res = {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": round(ms, 4),
           "GBs": round(8 * n / (ms / 1e3) / 1e9, 1)}
    del a, b
    return res


# ---------------------------------------------------------------------------

def bench_headline(args, dev, stream, out):
    import torch
    import workloads
    from oracle import c_oracle, metrics
    from paper_1609_06641_amd import chw
    w = workloads.CONFIGS["plain_2p20_f32"]
    m, batch = 20, w.batch
    t0 = time.perf_counter()
    x_host = workloads.float_signals(w.seed, batch, m)
    log("generated %d x 2^%d in %.1f s" % (batch, m, time.perf_counter() - t0))
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty_like(x)
    plan = chw.Plan([m] * batch, dtype="f32")
    configure(plan, args, x, y, None)
    fwd = lambda: plan.forward(x, out=y)  # noqa: E731
    ms = time_steps(fwd, args.steps, args.warmup, stream)
    elems = batch << m
    gelem = elems / (ms / 1e3) / 1e9
    launches = launch_breakdown(plan, fwd, args.steps) if not args.no_launch_timing else [ms]
    names = launch_names(plan)
    calls = args.warmup + args.steps * (1 if args.no_launch_timing else 2)
    log("plain f32: %.3f ms/step, %.1f Gelem/s; launches %s" % (ms, gelem, launches))
    torch.cuda.synchronize()
    idx = [0, batch // 3, batch - 1]
    ref = c_oracle.chw_rows(x_host[idx].astype(np.float64), threads=8)
    rel = float(np.max(metrics.rel_l2(y[idx].double().cpu().numpy(), ref)))
    desc = plan.describe()["plan"]
    out.update({
        "metric": METRIC, "value": round(gelem, 3), "unit": "Gelem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain_2p20_f32: 1024 x 2^20 float32, orthonormal dyadic WHT",
                   "batch": batch, "log2_n": m, "plan": desc["config"],
                   "splits": desc["splits"], "autotuned": bool(args.tune and not args.plan_config)},
        "roofline": roofline(8, launches, plan_launches(plan, 0),
                             stored_profile(PROFILE_HEADLINE, desc["splits"]), elems),
        "parity": {"sampled_signals": idx, "max_rel_l2": rel},
        "forward_calls": calls,
    })
    if not args.no_forms:
        out["forms"] = bench_forms(args, x, y, m, batch, stream)
    del x, y
    torch.cuda.empty_cache()
    return x_host, m


def bench_forms(args, x, y, m, batch, stream):
    """The other forms on the headline batch (default planner choices, no
    tuning): the sequency and natural orders, the Haar transform alone
    (eq. 2), the Haar-Walsh transform (eq. 4) and three signed rounds.
    Algorithmic bytes: one read and one write of the data."""
    import torch
    import workloads
    from paper_1609_06641_amd import chw
    elems = batch << m
    steps = max(3, args.steps // 2)
    res = {}

    def rec(name, plan, fn, note):
        ms = time_steps(fn, steps, 2, stream)
        res[name] = {"ms": round(ms, 4), "Gelem_s": round(elems / (ms / 1e3) / 1e9, 2),
                     "roofline_frac": round(8 * elems / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "launches_per_call": len(plan.describe()["plan"]["forward"]), "note": note}

    ws = torch.empty(max(chw.Plan([m] * batch).workspace_size(), 16), dtype=torch.uint8,
                     device=x.device)
    for order in ("sequency", "natural"):
        p = chw.Plan([m] * batch, dtype="f32", order=order)
        rec(order, p, lambda: p.forward(x, out=y, workspace=ws), "exact permutation of the dyadic output")
        p.close()
    p = chw.Plan([m] * batch, dtype="f32")
    rec("haar", p, lambda: p.haar_forward(x, out=y, workspace=ws), "Psi_m x alone (eq. 2)")
    hw = chw.Plan.haar_walsh(batch, m, dtype="f32")
    rec("haar_walsh", hw, lambda: hw.forward(x, out=y, workspace=ws), "diag(1, H_0..H_{m-1}) w (eq. 4)")
    hw.close()
    k = 3
    words = workloads.pack_sign_bits(workloads.sign_rounds(2002, k, 1 << m)).reshape(-1).view(np.int32)
    signs = torch.from_numpy(words.copy()).to(x.device)
    rec("signed_3_rounds", p, lambda: p.forward_signed(x, signs, "shared", k, out=y, workspace=ws),
        "y = H D_3 H D_2 H D_1 x, one shared diagonal per round; each round's last pass and "
        "the next round's first pass run as one launch")
    res["signed_3_rounds"]["launches_per_call"] = k + 1 if p.describe()["plan"]["turn"] else 2 * k
    rec("signed_3_rounds_adjoint", p,
        lambda: p.backward_signed(x, signs, "shared", k, out=y, workspace=ws),
        "x = D_1 H D_2 H D_3 H g through the forward launches (the Paley-ordered H is "
        "symmetric): diagonals shifted by a round, D_1 at the last pass's store")
    res["signed_3_rounds_adjoint"]["launches_per_call"] = res["signed_3_rounds"]["launches_per_call"]
    # one round with a fresh per-element diagonal drawn on the device every call
    pe_words = torch.empty(p.sign_words("per_element"), dtype=torch.int32, device=x.device)
    seed = [0]

    def device_signed():
        seed[0] += 1
        p.philox_signs(seed[0], 1, "per_element", out=pe_words)
        p.forward_signed(x, pe_words, "per_element", 1, out=y, workspace=ws)
    rec("signed_device_signs", p, device_signed,
        "y = H D x with D (one bit per element) drawn by Philox4x64-10 on the device each call")
    gen_ms = time_steps(lambda: p.philox_signs(7, 1, "per_element", out=pe_words), steps, 2, stream)
    res["signed_device_signs"]["philox_ms"] = round(gen_ms, 4)
    del pe_words
    # the factor-by-factor node evaluation of Sec. 4: one launch per factor
    nws = torch.empty(p.nodes_workspace_size(), dtype=torch.uint8, device=x.device)
    for name, chunk in (("nodes", 0), ("nodes_chunked", 32)):
        rec(name, p, lambda: p.nodes_forward(x, out=y, workspace=nws, chunk=chunk),
            "eq. (3) factor by factor: %d node launches of a full read and write each%s"
            % (m, "" if chunk == 0 else ", %d signals at a time" % chunk))
        res[name]["launches_per_call"] = m + sum(1 for r in range(m) if (m if r == 0 else m - r) > 12)
    del nws
    p.close()
    return res


# Autotuner results for the ragged workloads on gfx950, written by
# `bench.py --write-tuning` (its header says how); the default run starts its
# ragged plans from it (the tuning cache), so that every run times the kernels
# the stored profiles name.  Without the file the run autotunes live.
TUNING_FILE = os.path.join(ROOT, "paper_1609_06641_amd", "tuning_gfx950.txt")


def tuned_ragged_plan(ks, offs, dtype, persistent=False):
    """The ragged workload's plan in the configuration the benchmark times:
    graph-replayed, starting from TUNING_FILE's entry (the cache is emptied
    again afterwards); raises when the file holds no entry for it."""
    from paper_1609_06641_amd import chw
    chw.tuning_clear()
    chw.tuning_load(TUNING_FILE)
    try:
        p = chw.Plan(ks, dtype=dtype, offsets=offs, graph=True, persistent=persistent)
    finally:
        chw.tuning_clear()
    if not p.describe()["tuned"]:
        raise RuntimeError("no entry for the ragged %s plan in %s" % (dtype, TUNING_FILE))
    return p


def ragged_inputs(dtype, dev):
    import torch
    import workloads
    ks = workloads.ragged_log2_sizes(4001)
    offs = workloads.packed_offsets(ks)
    xr = workloads.ragged_values(4002, ks, offs)
    if dtype == "f32":
        xb = torch.from_numpy(xr).to(dev)
    else:
        xb = workloads.to_half_precision(xr, dtype).to(dev)
    return ks, offs, xb


def write_tuning(args, dev, stream):
    """Autotune the ragged workload's plans (BF16 and FP32; every launch form,
    and the persistent form) and save the tuning cache to TUNING_FILE."""
    import torch
    from paper_1609_06641_amd import chw
    chw.tuning_clear()
    for dtype in ("bf16", "f32"):
        ks, offs, xb = ragged_inputs(dtype, dev)
        yb = torch.empty_like(xb)
        for persistent in (False, True):
            p = chw.Plan(ks, dtype=dtype, offsets=offs, graph=True, persistent=persistent)
            ws = torch.empty(max(p.workspace_size(), 16), dtype=torch.uint8, device=dev)
            p.autotune(xb, yb, workspace=ws, iters=20)
            log("tuned %s persistent=%d: %s" % (dtype, persistent, p.describe()["plan"]["config"]))
            p.close()
            del ws
        del xb, yb
        torch.cuda.empty_cache()
    comment = ("autotuner results for the ragged workload (20000 signals, 2^30 elements; BF16 "
               "and FP32; all launch forms and the persistent one), 20 timed calls per candidate\n"
               "written by: python3 bench.py --write-tuning (%s, %s)"
               % (torch.cuda.get_device_properties(0).gcnArchName, torch.cuda.get_device_name(0)))
    chw.tuning_save(TUNING_FILE, comment)
    log("wrote %s (%d entries)" % (TUNING_FILE, chw.tuning_count()))


def bench_ragged(args, dev, stream, dtype):
    """The ragged workload (20000 signals, log2 sizes in [6, 20], 2^30
    elements) in `dtype`: the configuration the autotuner picks among every
    launch form, replayed as a HIP graph (the reported value), and beside it
    the one-launch persistent form, autotuned within that form.  The tuned
    configurations come from TUNING_FILE when it holds them, else from a live
    autotuning run."""
    import torch
    import workloads
    from oracle import c_oracle, metrics
    from paper_1609_06641_amd import chw
    ks, offs, xb = ragged_inputs(dtype, dev)
    yb = torch.empty_like(xb)
    relems = int(offs[-1])
    es = xb.element_size()
    ws = torch.empty(max(chw.Plan(ks, dtype=dtype, offsets=offs).workspace_size(), 16),
                     dtype=torch.uint8, device=dev)
    tuned = not args.plan_config

    def timed(plan, key):
        if args.plan_config:
            configure(plan, args, xb, yb, ws, key=key)
        elif not plan.describe()["tuned"]:
            plan.autotune(xb, yb, workspace=ws, iters=2)  # no stored entry: tune now
        fn = lambda: plan.forward(xb, out=yb, workspace=ws)  # noqa: E731
        ms = time_steps(fn, args.steps, args.warmup, stream)
        launches = launch_breakdown(plan, fn, args.steps) if not args.no_launch_timing else [ms]
        fn()   # graph replay again after the timed launches
        return ms, launches

    rp = chw.Plan(ks, dtype=dtype, offsets=offs, graph=True)
    from_file = bool(rp.describe()["tuned"])
    rms, launches = timed(rp, "ragged")
    torch.cuda.synchronize()
    # parity: a few signals of each size class
    sel = [int(np.nonzero(ks == k)[0][0]) for k in (6, 12, 16, 20)]
    rels = []
    for i in sel:
        n = 1 << int(ks[i])
        o = int(offs[i])
        ref = c_oracle.chw_batch(xb[o:o + n].double().cpu().numpy(), [int(ks[i])])
        rels.append(float(metrics.rel_l2(yb[o:o + n].double().cpu().numpy(), ref)))
    d = rp.describe()["plan"]
    dt_code = {"f32": 0, "bf16": 1, "f16": 2}[dtype]
    profile = stored_profile(PROFILE_RAGGED[dtype], d["splits"])
    res = {"value": round(relems / (rms / 1e3) / 1e9, 3), "unit": "Gelem/s",
           "ms_per_step": round(rms, 4), "signals": len(ks), "elements": relems,
           "dtype": "%s storage, fp32 compute" % dtype if dtype != "f32" else "f32",
           "plan": d["config"], "autotuned": tuned, "graph": True,
           "tuning": ("from %s" % os.path.relpath(TUNING_FILE, ROOT)) if from_file and tuned
                     else ("live" if tuned else "fixed options"),
           "launches_per_call": len(d["forward"]),
           "roofline": roofline(2 * es, launches, plan_launches(rp, dt_code), profile, relems),
           "parity": {"log2_sizes": [int(ks[i]) for i in sel], "max_rel_l2": max(rels)}}
    rp.close()
    log("%s ragged: %.3f ms/step (%d launches)" % (dtype, rms, res["launches_per_call"]))
    # the one persistent launch per call (exec 2), autotuned within that form
    pp = chw.Plan(ks, dtype=dtype, offsets=offs, graph=True, persistent=True)
    pms, plaunch = timed(pp, "persistent")
    pd = pp.describe()["plan"]
    res["one_launch"] = {"ms_per_step": round(pms, 4),
                         "Gelem_s": round(relems / (pms / 1e3) / 1e9, 3),
                         "plan": pd["config"], "autotuned": tuned,
                         "launches_per_call": len(pd["forward"]),
                         "launch_ms": [round(t, 4) for t in plaunch]}
    pp.close()
    log("%s ragged, one launch: %.3f ms/step" % (dtype, pms))
    del xb, yb, ws
    torch.cuda.empty_cache()
    return res


def run_other(args, dev, stream):
    """Profiling entry for the other workloads (one JSON line of their own)."""
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
        # the configuration of the ragged leg of the default run: the tuning
        # file's entry when it holds one
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
    if not (plan.describe()["tuned"] and not args.plan_config and not args.tune):
        configure(plan, args, x, y, ws, key="ragged" if w.name.startswith("ragged") else "plan")
    es = x.element_size()
    k = args.signed_rounds
    if k > 0:
        # y = H D_k ... H D_1 x with one diagonal per round shared by the
        # signals, fused into the tile kernels; the unfused form (torch sign
        # flips, then the plain transform per round) is timed beside it
        m = int(plan.log2_sizes.max())
        diags = workloads.sign_rounds(w.seed + 1, k, 1 << m)
        words = workloads.pack_sign_bits(diags).reshape(-1).view(np.int32)
        signs = torch.from_numpy(words.copy()).to(dev)
        dflat = [torch.from_numpy(workloads.expand_shared_signs(
            diags[r:r + 1].astype(np.float32), plan.log2_sizes, plan.offsets)[0]).to(tdt).to(dev)
            for r in range(k)]
        fn = lambda: plan.forward_signed(x, signs, "shared", k, out=y, workspace=ws)  # noqa: E731

        def unfused():
            v = x
            for r in range(k):
                v = plan.forward(v * dflat[r], out=y, workspace=ws)
        ms_unfused = time_steps(unfused, args.steps, args.warmup, stream)
    else:
        fn = lambda: plan.forward(x, out=y, workspace=ws)  # noqa: E731
    ms = time_steps(fn, args.steps, args.warmup, stream)
    launches = launch_breakdown(plan, fn, args.steps) if not args.no_launch_timing else [ms]
    # algorithmic bytes: one read and one write of the data, plus the sign bits
    bpe = 2 * es + (k / 8.0 if k > 0 else 0.0)
    dt_code = {"f32": 0, "bf16": 1, "f16": 2, "i32": 3, "f64": 4}[plan.dtype]
    ls = plan_launches(plan, dt_code)
    if k > 1:  # several rounds: the launches of the call, in order
        ls = [{"name": "launch %d of the call" % (i + 1), "elements": elems, "symbol": None}
              for i in range(len(launches))]
    out = {"workload": w.name, "ms_per_step": round(ms, 4),
           "Gelem_s": round(elems / (ms / 1e3) / 1e9, 2),
           "roofline": roofline(bpe, launches, ls, None, elems),
           "splits": plan.describe()["plan"]["splits"],
           "plan": plan.describe()["plan"]["config"],
           "forward_calls": args.warmup + args.steps * (1 if args.no_launch_timing else 2)}
    if k > 0:
        from oracle import metrics, signed
        torch.cuda.synchronize()
        idx = [0, w.batch - 1] if not w.name.startswith("ragged") else []
        n = 1 << int(plan.log2_sizes[0])
        xh = x.double().cpu().numpy()
        yh = y.double().cpu().numpy()
        rel = max([float(metrics.rel_l2(yh[i * n:(i + 1) * n],
                                        signed.signed_forward(xh[i * n:(i + 1) * n], list(diags))))
                   for i in idx] or [0.0])
        out["signed"] = {"rounds": k, "diagonal": "shared by the signals",
                         "unfused_ms_per_step": round(ms_unfused, 4),
                         "parity": {"sampled_signals": idx, "max_rel_l2": rel}}
    if args.copy_gib > 0:
        out["copy_calibration"] = copy_calibration(args.copy_gib, dev, stream, args.steps)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# every configuration of the workload list, cold and warm

CONFIG_WORKLOADS = ("plain_small_f32", "plain_small_i32", "plain_2p24_f32", "precision_bf16",
                    "precision_f16", "diff_f32")
# A cold run cycles through copies of its buffers spanning at least this many
# bytes, so that no step finds its data in the 256 MB memory-side cache left
# there by the step before.
ROTATE_BYTES = 1 << 30


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _time_oracle(fn):
    t0 = time.perf_counter()
    r = fn()
    return r, time.perf_counter() - t0


def _uniform_inputs(w):
    import workloads
    m = w.log2_sizes[0]
    if w.dtype in ("bf16", "f16"):
        return workloads.outlier_signals(w.seed, w.batch, m)
    if w.dtype == "i32":
        return workloads.int_signals(w.seed, w.batch, m)
    return workloads.float_signals(w.seed, w.batch, m)


class Rotation:
    """`copies` device copies of an input (and room for as many outputs),
    cycled one per call, so a cold step reads data the previous steps did not
    leave in the caches."""

    def __init__(self, x, copies):
        import torch
        self.n = x.numel()
        self.copies = copies
        self.xs = torch.empty(copies * self.n, dtype=x.dtype, device=x.device)
        for r in range(copies):
            self.xs[r * self.n:(r + 1) * self.n].copy_(x)
        self.ys = torch.empty_like(self.xs)
        self.i = 0

    def next(self):
        r = self.i % self.copies
        self.i += 1
        return self.xs[r * self.n:(r + 1) * self.n], self.ys[r * self.n:(r + 1) * self.n]

    def first(self):
        return self.xs[:self.n], self.ys[:self.n]


def _copies(nbytes_per_set):
    return max(1, -(-ROTATE_BYTES // max(1, nbytes_per_set)))


def _step_figures(elems, bpe, cold_ms, warm_ms, launches, ls, profile=None):
    return {"ms_per_step": round(cold_ms, 5), "warm_ms_per_step": round(warm_ms, 5),
            "Gelem_s": round(elems / (cold_ms / 1e3) / 1e9, 2),
            "warm_Gelem_s": round(elems / (warm_ms / 1e3) / 1e9, 2),
            "roofline": roofline(bpe, launches, ls, profile, elems)}


def bench_uniform_config(args, name, dev, stream):
    """One uniform batch of the workload list: cold (rotating buffers) and warm
    step times, per-launch roofline (cold), sampled parity and the oracle on
    the host's cores."""
    import torch
    import workloads
    from oracle import c_oracle, metrics
    from paper_1609_06641_amd import chw
    w = workloads.CONFIGS[name]
    m, batch = w.log2_sizes[0], w.batch
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
           "i32": torch.int32}[w.dtype]
    xh = _uniform_inputs(w)
    if w.dtype in ("bf16", "f16"):
        xd = workloads.to_half_precision(xh, w.dtype).reshape(-1)
    else:
        xd = torch.from_numpy(xh.reshape(-1))
    x = xd.to(tdt).to(dev)
    elems = batch << m
    es = x.element_size()
    plan = chw.Plan([m] * batch, dtype=w.dtype, norm=w.norm)
    ws = torch.empty(max(plan.workspace_size(), 16), dtype=torch.uint8, device=dev)
    rot = Rotation(x, _copies(2 * elems * es))
    steps = args.steps

    def cold():
        a, b = rot.next()
        plan.forward(a, out=b, workspace=ws)
    x0, y0 = rot.first()
    cold_ms = time_steps(cold, steps, args.warmup + rot.copies, stream)
    warm_ms = time_steps(lambda: plan.forward(x0, out=y0, workspace=ws), steps, args.warmup, stream)
    launches = launch_breakdown(plan, cold, steps) if not args.no_launch_timing else [cold_ms]
    dt_code = {"f32": 0, "bf16": 1, "f16": 2, "i32": 3}[w.dtype]
    splits = plan.describe()["plan"]["splits"]
    res = {"workload": w.note, "dtype": w.dtype, "elements": elems,
           "copies_rotated": rot.copies, "splits": splits}
    res.update(_step_figures(elems, 2 * es, cold_ms, warm_ms, launches,
                             plan_launches(plan, dt_code),
                             stored_profile(CONFIG_PROFILES[name], splits)))
    res["device_ms_per_step"] = round(float(sum(launches)), 5)
    res["forward_calls"] = (args.warmup + rot.copies + steps) + (args.warmup + steps) + \
        (0 if args.no_launch_timing else steps) + 1
    # parity on sampled signals, and the oracle timed on the host
    plan.forward(x0, out=y0, workspace=ws)
    torch.cuda.synchronize()
    idx = sorted({0, batch // 2, batch - 1})
    n = 1 << m
    got = y0.reshape(batch, n)[idx]
    xin = x0.reshape(batch, n)[idx]
    threads = len(os.sched_getaffinity(0))
    if w.dtype == "i32":
        ref = c_oracle.chw_rows(xin.cpu().numpy().astype(np.int64))
        res["parity"] = {"sampled_signals": idx, "bit_exact": bool(np.array_equal(
            got.cpu().numpy().astype(np.int64), ref.astype(np.int32).astype(np.int64)))}
        full = xd.numpy().astype(np.int64).reshape(batch, n)
    else:
        ref = c_oracle.chw_rows(xin.double().cpu().numpy())
        res["parity"] = {"sampled_signals": idx, "max_rel_l2": float(np.max(
            metrics.rel_l2(got.double().cpu().numpy(), ref)))}
        full = xd.double().numpy().reshape(batch, n) if w.dtype in ("bf16", "f16") else \
            xh.astype(np.float64).reshape(batch, n)
    # the oracle on at most 2^26 elements of the batch, all cores
    take = max(1, min(batch, (1 << 26) >> m))
    _, dt = _time_oracle(lambda: c_oracle.chw_rows(full[:take], threads=threads))
    res["cpu_baseline"] = {"value": round(take * n / dt / 1e9, 5), "unit": "Gelem/s",
                           "cores": threads, "kind": "oracle", "cpu": cpu_model(),
                           "sample": "%d of the %d signals of 2^%d, %s plain-C cascade, %.2f s"
                                     % (take, batch, m, "int64" if w.dtype == "i32" else "float64", dt)}
    plan.close()
    del x, rot, ws
    torch.cuda.empty_cache()
    return res


def bench_diff_config(args, dev, stream):
    """y = H D x at 256 x 2^14 FP32 with one shared random-sign diagonal D:
    forward and adjoint through the fused signed kernels (the autograd
    function's two calls), cold and warm, beside the same through torch's sign
    multiply and the plain transform; then a whole autograd step."""
    import torch
    import workloads
    from oracle import metrics, signed
    from paper_1609_06641_amd import chw
    w = workloads.CONFIGS["diff_f32"]
    m, batch = w.log2_sizes[0], w.batch
    n, elems = 1 << m, w.batch << w.log2_sizes[0]
    xh = workloads.float_signals(w.seed, batch, m)
    d = workloads.sign_diagonal(5002, n)
    gh = workloads.float_signals(5003, batch, m)
    words = workloads.pack_sign_bits(d.reshape(1, -1)).reshape(-1).view(np.int32)
    signs = torch.from_numpy(words.copy()).to(dev)
    plan = chw.Plan([m] * batch, dtype="f32")
    x = torch.from_numpy(xh.reshape(-1)).to(dev)
    g = torch.from_numpy(gh.reshape(-1)).to(dev)
    rx = Rotation(x, _copies(4 * elems * 4))
    rg = Rotation(g, rx.copies)
    steps = args.steps

    def fused(rot_x, rot_g):
        a, ya = rot_x.next()
        b, yb = rot_g.next()
        plan.forward_signed(a, signs, "shared", 1, out=ya)
        plan.backward_signed(b, signs, "shared", 1, out=yb)
    dflat = torch.from_numpy(np.tile(d.astype(np.float32), batch)).to(dev)

    def unfused(rot_x, rot_g):
        a, ya = rot_x.next()
        b, yb = rot_g.next()
        plan.forward(a * dflat, out=ya)
        torch.mul(plan.backward(b, out=yb), dflat, out=yb)
    cold_ms = time_steps(lambda: fused(rx, rg), steps, args.warmup + rx.copies, stream)
    one_x, one_g = Rotation(x, 1), Rotation(g, 1)
    warm_ms = time_steps(lambda: fused(one_x, one_g), steps, args.warmup, stream)
    unf_ms = time_steps(lambda: unfused(rx, rg), steps, args.warmup + rx.copies, stream)
    plan.set_option("timing", 1)
    acc = None
    for _ in range(steps):
        a, ya = rx.next()
        plan.forward_signed(a, signs, "shared", 1, out=ya)
        t = plan.launch_times()
        b, yb = rg.next()
        plan.backward_signed(b, signs, "shared", 1, out=yb)
        t = t + plan.launch_times()
        acc = np.array(t) if acc is None else acc + np.array(t)
    plan.set_option("timing", 0)
    launches = list(acc / steps)
    ls = [dict(l, name="forward " + l["name"]) for l in plan_launches(plan, 0)] + \
         [dict(l, name="adjoint " + l["name"]) for l in plan_launches(plan, 0, "backward")]
    # elements through the transform: forward and adjoint each take the batch
    res = {"workload": w.note, "dtype": "f32", "elements": elems,
           "copies_rotated": rx.copies, "step": "forward + adjoint (fused signs)"}
    res.update(_step_figures(2 * elems, 8, cold_ms, warm_ms, launches,
                             [dict(l, elements=elems) for l in ls],
                             stored_profile(CONFIG_PROFILES["diff_f32"],
                                            plan.describe()["plan"]["splits"])))
    res["device_ms_per_step"] = round(float(sum(launches)), 5)
    res["unfused_ms_per_step"] = round(unf_ms, 5)
    # forward + adjoint pairs of this run (for per-step counter totals)
    res["forward_calls"] = 2 * (args.warmup + rx.copies + steps) + (args.warmup + steps) + \
        steps + (args.warmup + steps) + 1
    # a whole autograd step (host overhead of autograd included)
    xr = x.clone().requires_grad_(True)

    def ag():
        y = chw.signed_transform(xr, plan, signs, "shared", 1)
        y.backward(g)
    res["autograd_ms_per_step"] = round(time_steps(ag, steps, args.warmup, stream), 5)
    torch.cuda.synchronize()
    y = chw.signed_transform(xr, plan, signs, "shared", 1)
    xr.grad = None
    y.backward(g)
    torch.cuda.synchronize()
    idx = [0, batch - 1]
    yh = y.detach().double().cpu().numpy().reshape(batch, n)
    gx = xr.grad.double().cpu().numpy().reshape(batch, n)
    rel = max(float(metrics.rel_l2(yh[i], signed.signed_forward(xh[i].astype(np.float64), [d])))
              for i in idx)
    relb = max(float(metrics.rel_l2(gx[i], signed.signed_adjoint(gh[i].astype(np.float64), [d])))
               for i in idx)
    res["parity"] = {"sampled_signals": idx, "max_rel_l2_forward": rel,
                     "max_rel_l2_gradient": relb}
    threads = len(os.sched_getaffinity(0))
    sizes = np.full(batch, m, dtype=np.int32)
    dfull = np.tile(d.astype(np.float64), batch)
    t0 = time.perf_counter()
    signed.signed_batch(xh.reshape(-1).astype(np.float64), sizes, [dfull], threads=threads)
    signed.signed_batch(gh.reshape(-1).astype(np.float64), sizes, [dfull], adjoint=True,
                        threads=threads)
    dt = time.perf_counter() - t0
    res["cpu_baseline"] = {"value": round(2 * elems / dt / 1e9, 5), "unit": "Gelem/s",
                           "cores": threads, "kind": "oracle", "cpu": cpu_model(),
                           "sample": "forward and adjoint of all %d signals of 2^%d, float64 "
                                     "plain-C cascade with the sign flips, %.2f s" % (batch, m, dt)}
    plan.close()
    return res


def bench_configs(args, dev, stream):
    out = {}
    for name in CONFIG_WORKLOADS:
        t0 = time.perf_counter()
        out[name] = bench_diff_config(args, dev, stream) if name == "diff_f32" else \
            bench_uniform_config(args, name, dev, stream)
        log("config %s: %.4f ms/step cold, %.4f warm (%.1f s)" % (
            name, out[name]["ms_per_step"], out[name]["warm_ms_per_step"],
            time.perf_counter() - t0))
    return out


# ---------------------------------------------------------------------------
# profile summaries

def _db(path):
    import sqlite3
    dbs = glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit("no rocprofv3 results database under %s" % path)
    return sqlite3.connect(dbs[0])


def _kernel_stats(path):
    con = _db(path)
    rows = con.execute("select name, end - start from kernels order by start").fetchall()
    agg = {}
    for name, d in rows:
        agg.setdefault(name, []).append(d / 1e3)
    return agg


def _counter(path, name):
    con = _db(path)
    rows = con.execute("select kernel_name, value from counters_collection "
                       "where counter_name = ? order by dispatch_id", (name,)).fetchall()
    agg = {}
    for k, v in rows:
        agg.setdefault(k, []).append(float(v))
    return agg


def summarize(args):
    """Write a profiles/ summary from a kernel-trace run and two PMC runs.

    --summarize TRACE FETCH WRITE: rocprofv3 output folders of
      rocprofv3 --kernel-trace --stats -d TRACE -- python3 bench.py ...
      rocprofv3 --pmc FETCH_SIZE     -d FETCH -- python3 bench.py ...
      rocprofv3 --pmc WRITE_SIZE     -d WRITE -- python3 bench.py ...
    The two PMC runs must time --copy-gib G of plain copy besides the
    transform; --calls is the number of transforms each PMC run made.
    """
    trace_dir, fetch_dir, write_dir = args.summarize
    stats = _kernel_stats(trace_dir) if trace_dir != "-" else {}
    # "-" for FETCH and WRITE: a kernel-trace summary without counters
    fetch = _counter(fetch_dir, "FETCH_SIZE") if fetch_dir != "-" else {}
    write = _counter(write_dir, "WRITE_SIZE") if write_dir != "-" else {}
    copy_bytes = int(args.copy_gib * (1 << 30)) // 4 * 4
    copy_name = [k for k in fetch if "copyBuffer" in k]
    ff = fw = None
    if copy_name:
        cf = max(fetch[copy_name[0]])           # KiB per copy dispatch
        cw = max(write[copy_name[0]])
        ff = copy_bytes / 1024.0 / cf
        fw = copy_bytes / 1024.0 / cw
    chw_fetch = sum(sum(v) for k, v in fetch.items() if "chw::" in k)
    chw_write = sum(sum(v) for k, v in write.items() if "chw::" in k)
    traffic = None
    if ff and fw and args.calls:
        traffic = int((chw_fetch * ff + chw_write * fw) * 1024 / args.calls)
    if not stats:
        head = ["Counters from `rocprofv3 --pmc` (per dispatch, averaged over the dispatches)."]
    elif fetch:
        head = ["Kernel durations from `rocprofv3 --kernel-trace --stats` and HBM-side",
                "bytes from two `rocprofv3 --pmc` runs (FETCH_SIZE, then WRITE_SIZE, KiB per",
                "dispatch).  The counters are scaled by what they read for a plain",
                "device-to-device copy of known size in the same run (%.2f GiB read and" % (copy_bytes / 2**30),
                "written): fetch factor %s, write factor %s." % (
                    "%.4f" % ff if ff else "n/a", "%.4f" % fw if fw else "n/a")]
    else:
        head = ["Kernel durations from `rocprofv3 --kernel-trace --stats` (no counters)."]
    lines = ["# %s" % args.title, ""] + head + [
             "", "Commands (on the GPU machine, after `cd /tmp && export TMPDIR=/tmp`; REPO is the",
             "repository root, P an output folder):", ""]
    for c in args.cmd or []:
        lines.append("    " + c)
    bj = {}
    if args.bench_json and os.path.exists(args.bench_json):
        with open(args.bench_json) as f:
            bj = json.loads(f.read().strip().splitlines()[-1])
    trace_calls = bj.get("forward_calls")

    def per_launch(vals, calls):
        """A kernel's dispatches split by launch position within a call (one
        list when the call launches it once or the count does not divide)."""
        n = len(vals)
        q = n // calls if calls and n % calls == 0 and n // calls > 1 else 1
        return [vals[j::q] for j in range(q)]

    def label(k, j, parts):
        return "`%s`" % k[:90] if parts == 1 else "`%s` #%d" % (k[:90], j)
    if stats:
        lines += ["", "| kernel (#j: its j-th launch in a call) | dispatches | avg us | min us | max us |",
                  "|---|---|---|---|---|"]
    for k, v in stats.items():
        if "chw::" in k or "copyBuffer" in k:
            parts = per_launch(v, trace_calls if "chw::" in k else None)
            for j, vj in enumerate(parts):
                lines.append("| %s | %d | %.1f | %.1f | %.1f |" % (label(k, j, len(parts)), len(vj),
                                                                 sum(vj) / len(vj), min(vj), max(vj)))
    if fetch:
        lines += ["", "| kernel | dispatches | FETCH_SIZE KiB avg | WRITE_SIZE KiB avg |", "|---|---|---|---|"]
    for k in fetch:
        if "chw::" in k or "copyBuffer" in k:
            wk = write.get(k, [0])
            fparts = per_launch(fetch[k], args.calls if "chw::" in k and len(wk) == len(fetch[k]) else None)
            wparts = per_launch(wk, args.calls) if len(fparts) > 1 else [wk]
            for j, (fj, wj) in enumerate(zip(fparts, wparts)):
                lines.append("| %s | %d | %.0f | %.0f |" % (label(k, j, len(fparts)), len(fj),
                                                           sum(fj) / len(fj), sum(wj) / max(1, len(wj))))
    counters = {}
    if args.counters:
        con = _db(args.counters)
        rows = con.execute("select kernel_name, counter_name, avg(value), count(*) from "
                           "counters_collection group by kernel_name, counter_name").fetchall()
        for k, c, v, n in rows:
            if "chw::" in k:
                counters.setdefault(k[:90], {})[c] = v
        names = sorted({c for d in counters.values() for c in d})
        lines += ["", "| kernel | " + " | ".join(names) + " |", "|---" * (len(names) + 1) + "|"]
        for k, d in counters.items():
            lines.append("| `%s` | " % k + " | ".join("%.0f" % d.get(c, float("nan")) for c in names) + " |")
        if all(c in names for c in ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE")):
            lines += ["", "Bank-conflict cycles per conflict-free LDS cycle "
                      "(SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)):", ""]
            for k, d in counters.items():
                act, bc = d["SQ_LDS_IDX_ACTIVE"], d["SQ_LDS_BANK_CONFLICT"]
                lines.append("* `%s`: %.3f" % (k, bc / max(1.0, act - bc)))
    splits = bj.get("config", {}).get("splits", bj.get("splits")) if bj else None
    per_kernel = {}
    if ff and fw:
        for k in fetch:
            if "chw::" in k and write.get(k):
                # a kernel launched q > 1 times per call: one entry per launch
                # position within the call ("#j"), from every q-th dispatch
                n = len(fetch[k])
                q = n // args.calls if args.calls and n % args.calls == 0 and \
                    len(write[k]) == n else 1
                for j in range(q):
                    fj, wj = fetch[k][j::q], write[k][j::q]
                    key = k[:90] if q == 1 else "%s#%d" % (k[:90], j)
                    per_kernel[key] = int((sum(fj) / len(fj) * ff + sum(wj) / len(wj) * fw) * 1024)
    summary = {"source_hash": kernel_source_hash(), "calls": args.calls, "splits": splits,
               "fetch_factor": ff, "write_factor": fw,
               "traffic_bytes_per_transform": traffic,
               "kernels_traffic_bytes": per_kernel,
               "kernels_avg_us": {}}
    for k, v in stats.items():
        if "chw::" in k:
            parts = per_launch(v, trace_calls)
            for j, vj in enumerate(parts):
                key = k[:90] if len(parts) == 1 else "%s#%d" % (k[:90], j)
                summary["kernels_avg_us"][key] = round(sum(vj) / len(vj), 2)
    if counters:
        summary["counters"] = counters
    lines += ["", "Machine-readable summary (the benchmark reports `traffic` from it while",
              "`source_hash` matches the kernel sources):", "", "```json",
              json.dumps(summary, indent=1), "```", ""]
    text = "\n".join(lines)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tune", action="store_true",
                    help="autotune the plans instead of timing BENCH_CONFIG")
    ap.add_argument("--plan-config", help="JSON planner options instead of autotuning")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--write-tuning", action="store_true",
                    help="autotune the ragged workload's plans and save them to the tuning file")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other configurations of the workload list")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other orders / Haar / signed forms on the headline batch")
    ap.add_argument("--no-launch-timing", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--workload", default="plain_2p20_f32")
    ap.add_argument("--signed-rounds", type=int, default=0,
                    help="with --workload: time y = H D_k ... H D_1 x (k rounds, fused diagonals)")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="also time a plain device copy of this many GiB (calibration)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE", "FETCH", "WRITE"))
    ap.add_argument("--calls", type=int, default=0)
    ap.add_argument("--counters", help="with --summarize: a rocprofv3 --pmc output folder whose "
                                       "counters are tabulated per kernel")
    ap.add_argument("--title", default="profile")
    ap.add_argument("--cmd", action="append")
    ap.add_argument("--out")
    ap.add_argument("--bench-json", help="with --summarize: the JSON line of the traced run "
                                         "(records the pass splits the profile covers)")
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(signals are independent, so a batch shards across GPUs with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.write_tuning:
        write_tuning(args, dev, stream)
        return
    if os.path.exists(TUNING_FILE) and not args.plan_config and not args.tune:
        from paper_1609_06641_amd import chw
        chw.tuning_load(TUNING_FILE)
    if args.workload in CONFIG_WORKLOADS:
        # one configuration of the workload list, cold and warm (its own line)
        res = bench_diff_config(args, dev, stream) if args.workload == "diff_f32" else \
            bench_uniform_config(args, args.workload, dev, stream)
        if args.copy_gib > 0:
            res["copy_calibration"] = copy_calibration(args.copy_gib, dev, stream, args.steps)
        print(json.dumps(res), flush=True)
        return
    if args.workload != "plain_2p20_f32":
        run_other(args, dev, stream)
        return
    out = {}
    x_host, m = bench_headline(args, dev, stream, out)
    if not args.no_ragged:
        out["bf16_ragged"] = bench_ragged(args, dev, stream, "bf16")
        out["f32_ragged"] = bench_ragged(args, dev, stream, "f32")
    if not args.no_configs:
        out["configs"] = bench_configs(args, dev, stream)
    if args.copy_gib > 0:
        out["copy_calibration"] = copy_calibration(args.copy_gib, dev, stream, args.steps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(x_host, m, min(args.cpu_sample, x_host.shape[0]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
