"""Host-side logic of bench.py (no GPU): the one-GPU guard, the roofline
record and the profile summaries it reads."""

import json
import subprocess
import sys
import os

import pytest

import bench
from paper_1609_06641_amd import chw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr


def _fake_profile(symbols):
    return {"traffic_bytes_per_transform": 3000, "kernels_traffic_bytes": {s: 1000 + i
                                                                          for i, s in enumerate(symbols)}}


def test_roofline_of_the_dominant_launch():
    p = chw.Plan([20] * 4, dtype="f32")
    p.set_option("split_l1", 8)
    ls = bench.plan_launches(p, 0)
    assert [l["elements"] for l in ls] == [4 << 20, 4 << 20]
    assert ls[0]["symbol"].startswith("void chw::chw_stream_kernel<0, 15, 5, 7, 3, false, 1>")
    prof = _fake_profile([l["symbol"] for l in ls])
    r = bench.roofline(8, [2.0, 1.0], ls, prof, 4 << 20)
    assert r["kernel"] == ls[0]["name"] and r["units_per_launch"] == 4 << 20
    assert r["achieved"] == pytest.approx(8 * (4 << 20) / 2e-3 / 1e9, abs=0.06)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["traffic"] == 1000
    t = r["transform"]
    assert t["achieved"] == pytest.approx(8 * (4 << 20) / 3e-3 / 1e9, abs=0.06)
    assert t["traffic"] == 3000
    assert t["measured_hbm_frac"] == pytest.approx(3000 / 3e-3 / 1e9 / 8000.0, abs=1e-4)
    # without per-launch timing the call counts as one unit
    r1 = bench.roofline(8, [3.0], ls, prof, 4 << 20)
    assert r1["traffic"] is None and r1["frac"] == t["frac"]


def test_ragged_launch_elements_cover_the_batch():
    import workloads
    ks = workloads.ragged_log2_sizes(4001)
    p = chw.Plan(ks, dtype="bf16")
    ls = bench.plan_launches(p, 1)
    two_pass = sum(1 << int(k) for k in ks if k > 15)
    one_pass = sum(1 << int(k) for k in ks if k <= 15)
    # every element once in a single-pass launch or once in each pass
    assert sum(l["elements"] for l in ls) == one_pass + 2 * two_pass


def test_every_configuration_names_its_launches():
    # each benchmarked workload's plan (and the larger two- and three-pass
    # sizes) maps every launch to a kernel name and symbol
    import workloads
    cases = [w.log2_sizes * w.batch for w in workloads.CONFIGS.values()
             if len(w.log2_sizes) == 1 and w.dtype != "f64"]
    assert [24] * 16 in cases
    cases += [[m] * 2 for m in range(16, 31)]
    for sizes in cases:
        p = chw.Plan(sizes, dtype="f32")
        for direction in ("forward", "backward"):
            ls = bench.plan_launches(p, 0, direction)
            assert ls and all(l["name"] for l in ls), sizes


def test_profiles_name_their_kernels():
    # the committed summaries carry per-kernel PMC bytes keyed by the symbols
    # plan_launches derives
    for path in (bench.PROFILE_HEADLINE, *bench.PROFILE_RAGGED.values()):
        with open(path) as f:
            text = f.read()
        summary = json.loads(text.split("```json\n")[1].split("\n```")[0])
        assert summary["kernels_traffic_bytes"]
        for sym in summary["kernels_traffic_bytes"]:
            assert sym.startswith("void chw::chw_")
    p = chw.Plan([20] * 4, dtype="f32")
    p.set_option("split_l1", 8)
    with open(bench.PROFILE_HEADLINE) as f:
        assert bench.plan_launches(p, 0)[0]["symbol"] in f.read()


def test_config_profiles_name_the_planned_kernels():
    # every workload line's profile holds PMC bytes for each kernel its plan
    # launches (a profile taken with other kernels cannot lend its traffic)
    import workloads
    for name, path in bench.CONFIG_PROFILES.items():
        w = workloads.CONFIGS[name]
        p = chw.Plan(w.log2_sizes * w.batch, dtype=w.dtype, norm=w.norm)
        with open(path) as f:
            summary = json.loads(f.read().split("```json\n")[1].split("\n```")[0])
        dt = {"f32": 0, "bf16": 1, "f16": 2, "i32": 3}[w.dtype]
        directions = ("forward", "backward") if name == "diff_f32" else ("forward",)
        for direction in directions:
            for launch in bench.plan_launches(p, dt, direction):
                assert launch["key"] in summary["kernels_traffic_bytes"], (name, launch)


def test_launch_keys_number_repeated_kernels():
    ls = [{"symbol": "a"}, {"symbol": "b"}, {"symbol": "a"}, {"symbol": None}]
    assert bench.launch_keys(ls) == ["a#0", "b", "a#1", None]
    # each ragged profile keys every launch of its tuned plan
    import workloads
    ks = workloads.ragged_log2_sizes(4001)
    for dtype, code in (("bf16", 1), ("f32", 0)):
        p = bench.tuned_ragged_plan(ks, workloads.packed_offsets(ks), dtype)
        with open(bench.PROFILE_RAGGED[dtype]) as f:
            summary = json.loads(f.read().split("```json\n")[1].split("\n```")[0])
        for launch in bench.plan_launches(p, code):
            assert launch["key"] in summary["kernels_traffic_bytes"], (dtype, launch)


def test_tuning_file_holds_the_ragged_plans():
    # the committed tuning file has an entry for each ragged plan the
    # benchmark times (four launches and one launch, BF16 and FP32), and
    # loading it leaves the cache empty again
    import workloads
    ks = workloads.ragged_log2_sizes(4001)
    offs = workloads.packed_offsets(ks)
    for dtype in ("bf16", "f32"):
        for persistent in (False, True):
            p = bench.tuned_ragged_plan(ks, offs, dtype, persistent=persistent)
            c = p.describe()["plan"]["config"]
            assert c["exec"] == (2 if persistent else 0)
            p.check()
    assert chw.tuning_count() == 0


def test_source_hash_ignores_comments():
    assert bench._code_only("a // x\n  b /* y\n z */ c\n") == "a b c"
    assert bench._code_only("int x = 1;  // one") == bench._code_only("int x = 1;\n")
