"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments, plans (host logic) and reports the
no-device case."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_06641_amd import chw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "chw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chw_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = chw.load()
    names = _header_functions()
    assert "chw_plan" in names and "chw_forward" in names and "chw_backward" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(chw.SIGNATURES), "binding and header disagree"


def test_version_and_status_strings():
    lib = chw.load()
    assert chw.version().startswith("libchw")
    for code, name in chw.STATUS.items():
        assert lib.chw_status_string(code).decode() == name


def _plan_raw(sizes, offsets=None, dtype=0, norm=0, flags=0, batch=None):
    lib = chw.load()
    h = ctypes.c_void_p()
    s = None if sizes is None else np.ascontiguousarray(sizes, dtype=np.int32)
    o = None if offsets is None else np.ascontiguousarray(offsets, dtype=np.int64)
    n = batch if batch is not None else (0 if s is None else len(s))
    st = lib.chw_plan(ctypes.byref(h), n,
                      None if s is None else s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                      None if o is None else o.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      dtype, norm, flags)
    return st, h


@pytest.mark.parametrize("case,expect", [
    (dict(sizes=[10], batch=-1), 1),
    (dict(sizes=None, batch=3), 1),
    (dict(sizes=[10], dtype=9), 1),
    (dict(sizes=[10], norm=5), 1),
    (dict(sizes=[10], dtype=3, norm=0), 2),            # int32 orthonormal
    (dict(sizes=[10], flags=1 << 9), 1),               # unknown flag
    (dict(sizes=[10], flags=(1 << 2) | (1 << 3)), 1),  # exclusive flags
    (dict(sizes=[-1]), 1),
    (dict(sizes=[31]), 1),
    (dict(sizes=[30]), 0),                             # the largest size (three passes)
    (dict(sizes=[28], flags=1 << 4), 2),               # three passes: dyadic order only
    (dict(sizes=[20], flags=(1 << 6) | (1 << 2)), 1),  # THREE_PASS with PERSISTENT
    (dict(sizes=[21], dtype=4), 2),                    # F64 limit
    (dict(sizes=[4, 4], offsets=[0, 8, 24]), 1),       # overlap
    (dict(sizes=[4, 4], offsets=[0, 16, 20]), 1),      # end below last signal
    (dict(sizes=[4], offsets=[-4, 12]), 1),            # negative
    (dict(sizes=[4, 4], offsets=[0, 17, 40]), 3),      # misaligned
    (dict(sizes=[1, 4], offsets=[1, 4, 40]), 0),       # tiny signal may be unaligned
])
def test_plan_validation(case, expect):
    st, h = _plan_raw(**case)
    assert st == expect, (case, chw.load().chw_last_error())
    if st == 0:
        assert chw.load().chw_plan_destroy(h) == 0
    else:
        assert not h.value
        assert chw.load().chw_last_error().decode()


def test_null_plan_arguments():
    lib = chw.load()
    n = ctypes.c_size_t()
    assert lib.chw_workspace_size(None, ctypes.byref(n)) == 1
    assert lib.chw_forward(None, None, None, None, None) == 1
    assert lib.chw_backward(None, None, None, None, None) == 1
    assert lib.chw_plan_destroy(None) == 0
    assert lib.chw_plan_set_option(None, b"lr12", 5) == 1


def test_empty_batch_is_a_noop():
    st, h = _plan_raw([])
    assert st == 0
    lib = chw.load()
    assert lib.chw_forward(h, None, None, None, None) == 0
    assert lib.chw_plan_destroy(h) == 0


def test_no_device_path():
    # This container has no GPU: compute calls must say so, not crash.
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    p = chw.Plan([10, 10])
    lib = chw.load()
    buf = (ctypes.c_char * 64)()
    st = lib.chw_forward(p.handle, ctypes.addressof(buf), ctypes.addressof(buf), None, None)
    # host buffer is 16-byte aligned by ctypes or not; either misaligned or no device
    assert st in (3, 5)
    aligned = ctypes.create_string_buffer(8192 * 4 + 64)
    a = (ctypes.addressof(aligned) + 15) & ~15
    st = lib.chw_forward(p.handle, ctypes.c_void_p(a), ctypes.c_void_p(a), None, None)
    assert st == 5, lib.chw_last_error()


def test_forward_noalloc_validation():
    # argument checks of the entry point that keeps the intermediate in the
    # library's static scratch; none of these touches the (fake) buffers
    lib = chw.load()
    fake = ctypes.c_void_p(1 << 20)
    assert lib.chw_forward_noalloc(None, fake, fake, None) == 1
    p = chw.Plan([10, 10])
    assert lib.chw_forward_noalloc(p.handle, None, fake, None) == 1
    assert lib.chw_forward_noalloc(p.handle, ctypes.c_void_p((1 << 20) + 4), fake, None) == 3
    # 2^25 two-pass FP32 elements: a 128 MiB intermediate, above the 64 MiB scratch
    big = chw.Plan([20] * 32)
    assert lib.chw_forward_noalloc(big.handle, fake, fake, None) == 2
    assert "64" in lib.chw_last_error().decode() or "67108864" in lib.chw_last_error().decode()
    # 2^24 two-pass elements fit exactly; single-pass plans need no scratch at all
    fits = chw.Plan([20] * 16)
    single = chw.Plan([15] * 4096)
    import torch
    if not torch.cuda.is_available():
        assert lib.chw_forward_noalloc(fits.handle, fake, fake, None) == 5
        assert lib.chw_forward_noalloc(single.handle, fake, fake, None) == 5
    # the empty plan is a no-op
    st, h = _plan_raw([])
    assert lib.chw_forward_noalloc(h, None, None, None) == 0
    assert lib.chw_plan_destroy(h) == 0


def test_describe_and_planner_properties():
    # uniform large signals: two passes, the split covers every level once
    p = chw.Plan([20] * 3, dtype="f32")
    d = p.describe()
    plan = d["plan"]
    assert plan["multi"] == 3 and plan["single"] == 0
    sp = plan["splits"][0]
    assert sp["m"] == 20 and sp["L1"] + (20 - sp["L1"]) == 20
    assert sp["L1"] <= sp["K1"] and 20 - sp["L1"] <= sp["K2"]
    assert p.workspace_size() == 3 * (1 << 20) * 4
    fw = plan["forward"]
    assert len(fw) == 2 and len(plan["backward"]) == 2   # one launch per pass
    assert fw[0]["K"] == sp["K1"] and fw[1]["K"] == sp["K2"]
    assert plan["backward"][0]["K"] == sp["K2"]          # adjoint: last pass first
    # first-pass items: 2^(m - L1) rows in tiles of 2^rows_log2 rows; last-pass
    # items: 2^L1 blocks of 2^(m - L1)
    rows_tiles = (1 << (20 - sp["L1"])) >> sp["rows_log2"]
    last_tiles = (1 << 20) >> sp["K2"]
    # plus one round-boundary tile per 2^15 elements (signed multi-round calls)
    assert plan["items"] == 3 * (rows_tiles + last_tiles + (1 << (20 - 15)))
    p.close()


def test_planner_ragged_and_options():
    # tiny signals last so that packing keeps every larger signal aligned
    sizes = [3, 6, 6, 6, 12, 13, 15, 16, 20, 24, 27, 2, 1, 0]
    p = chw.Plan(sizes, dtype="bf16")
    d = p.describe()["plan"]
    assert d["tiny"] == 3          # 2^m * 2 bytes < 16: m = 0, 1, 2
    assert d["single"] == 7        # 3, 6, 6, 6, 12, 13, 15
    assert d["multi"] == 4
    ms = sorted(s["m"] for s in d["splits"])
    assert ms == [16, 20, 24]                        # two passes
    assert [s["m"] for s in d["splits3"]] == [27]    # three passes above 2^25
    for s in d["splits"]:
        assert s["m"] - s["L1"] <= s["K2"] and s["m"] - s["L1"] >= s["rows_log2"]
    # forced split and register options rebuild the plan
    p2 = chw.Plan([20, 20], dtype="f32")
    p2.set_option("split_l1", 12)
    assert p2.describe()["plan"]["splits"][0]["L1"] == 12
    with pytest.raises(chw.CHWError):
        p2.set_option("split_l1", 11)   # no compiled variant runs 11 levels first
    p2.set_option("lr12", 5)
    assert p2.describe()["plan"]["config"]["lr12"] == 5
    with pytest.raises(chw.CHWError):
        p2.set_option("lr12", 7)
    with pytest.raises(chw.CHWError):
        p2.set_option("nonsense", 1)
    p3 = chw.Plan([14, 14], dtype="f32")
    p3.set_option("single15", 0)
    assert p3.describe()["plan"]["multi"] == 2


def test_planner_chunks():
    # chunking: first pass then last pass for each group of signals
    p = chw.Plan([20] * 8, dtype="f32")
    p.set_option("chunk", 3 << 20)
    d = p.describe()["plan"]
    assert d["config"]["chunk"] == 3 << 20
    fw = d["forward"]
    assert len(fw) == 6                       # chunks of 3, 3, 2 signals
    ends = [r["end"] - r["begin"] for r in fw]
    assert sum(ends) == d["items"]
    sp = d["splits"][0]
    per_first = (1 << (20 - sp["L1"])) >> sp["rows_log2"]
    per_last = (1 << 20) >> sp["K2"]
    assert ends == [3 * per_first, 3 * per_last, 3 * per_first, 3 * per_last,
                    2 * per_first, 2 * per_last]


def test_packed_misaligned_signal_is_rejected():
    # packed back to back, 1 + 2 + 4 elements put the 8-element bf16 signal at
    # element 7: not 16-byte aligned
    with pytest.raises(chw.CHWError) as e:
        chw.Plan([0, 1, 2, 3], dtype="bf16")
    assert e.value.name == "CHW_ERR_MISALIGNED"


def test_planner_packs_small_signals():
    p = chw.Plan([10] * 64, dtype="f32")
    p.set_option("spread", 0)
    d = p.describe()["plan"]
    assert d["items"] == 16 and d["list"] == 0      # 4 consecutive signals per tile
    # gaps force an offset list
    offs = np.arange(65, dtype=np.int64) * 2048
    p = chw.Plan([10] * 64, dtype="f32", offsets=offs)
    p.set_option("spread", 0)
    d = p.describe()["plan"]
    assert d["items"] == 16 and d["list"] == 64
    p.check()


def test_planner_spreads_small_groups():
    # a size group in 2^15-element tiles that would fill fewer than 256 tiles
    # goes one or a few signals per tile (the default); large groups and
    # 2^12-element tiles stay packed
    for ms, items in (([10] * 64, 16), ([14] * 256, 256), ([13] * 600, 200), ([13] * 2000, 500),
                      ([12] * 8192, 8192), ([13] * 8, 8),
                      ([9] * 3 + [20] * 2, 1 + 64 + 512 + 64)):  # + round-boundary tiles
        p = chw.Plan(ms, dtype="f32")
        d = p.describe()["plan"]
        assert d["config"]["spread"] == 1
        assert d["items"] == items, (ms[:2], d["items"])
        p.check()
    p = chw.Plan([13] * 8, dtype="f32")
    p.set_option("spread", 0)
    assert p.describe()["plan"]["items"] == 2
    # the rule looks at the whole launch: groups of 2^13, 2^14 and 2^15 that
    # are each small but together fill 256 tiles stay packed
    ms = [13] * 400 + [14] * 200 + [15] * 60
    assert chw.Plan(ms, dtype="f32").describe()["plan"]["items"] == 100 + 100 + 60


def test_layout_selfcheck():
    ok, rep = chw.layout_selfcheck()
    assert ok, [r for r in rep if not r.get("ok", True)]
    phases = {r["phase"] for r in rep if "phase" in r}
    assert phases == {"rounds", "rounds_from_bit", "contig", "paley", "paley_blocks_2^8..2^(K-1)",
                      "transposed", "transposed_merged"}
    # single-pass 2^12 tiles with 2^5 registers: two rounds after the stages
    # on the loaded vectors, against three from bit 0
    pre = {(r["K"], r["LR"], r["B0"]): r["rounds"] for r in rep if r.get("phase", "").startswith("rounds")}
    assert pre[(12, 5, 0)] == 3 and pre[(12, 5, 2)] == 2 and pre[(12, 5, 3)] == 2
    # 4-byte LDS accesses on gfx950: 32 banks per half-wave.  Every phase of a
    # compiled 4-byte tile (16-byte vectors of 4 words, V = 4, or of 8 BF16 /
    # FP16 elements, V = 8) puts at most one word per bank into a half-wave
    # access; the FP64 tiles (V = 2, 8-byte words) at most two.  The
    # transposed phase is compiled for 2^7 / 2^6 / 2^5 / 2^3 rows in 2^15 tiles
    # and 2^6 / 2^4 / 2^3 rows in 2^12 tiles.
    compiled_rows = {12: (6, 4, 3), 15: (7, 6, 5, 3)}
    for r in rep:
        if "phase" not in r:
            continue
        if r["phase"] == "transposed" and r["rows_log2"] not in compiled_rows[r["K"]]:
            continue
        if r.get("V") == 2 and r["K"] == 15:
            continue  # no FP64 2^15 tiles
        assert r["ways32"] <= (2 if r.get("V") == 2 else 1), r


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("opts", [dict(), dict(exec=2), dict(chunk=1 << 20), dict(single15=0),
                                  dict(split_l1=12), dict(exec=2, lr12=5), dict(stream=1),
                                  dict(stream=0), dict(stream=1, chunk=1 << 22, split_l1=8),
                                  dict(stream=2), dict(split_l1=9), dict(split_l1=9, stream=2),
                                  dict(pipeline=1, chunk=1 << 20), dict(pipeline=1, chunk=1 << 23)])
def test_plan_invariants_random_ragged(seed, opts):
    rng = np.random.default_rng(seed)
    hi = 22 if opts.get("exec") == 2 else 25
    ms = rng.integers(0, hi, size=int(rng.integers(1, 40))).astype(np.int32)
    # offsets with random aligned gaps (tiny signals may sit anywhere)
    offs, o = [], 0
    for k in ms:
        o += int(rng.integers(0, 3)) * 8          # 16-byte aligned for bf16 and f32
        offs.append(o)
        o += max(1 << int(k), 8)
    offs.append(o)
    for dtype in ("f32", "bf16"):
        try:
            p = chw.Plan(ms, dtype=dtype, offsets=np.array(offs, dtype=np.int64))
            for k, v in opts.items():
                p.set_option(k, v)
        except chw.CHWError as e:
            # forced splits may not cover every size
            assert opts.get("split_l1") and e.name == "CHW_ERR_UNSUPPORTED"
            continue
        p.check()
        p.close()


@pytest.mark.parametrize("sizes", [[14] * 8, [12] * 4 + [13, 15], [20, 9, 16], [6] * 5])
def test_workspace_size_does_not_depend_on_options(sizes):
    # Regression: the workspace a caller allocates from chw_workspace_size()
    # must cover every configuration the autotuner or options may switch to
    # (single-pass signals of 2^13..2^15 may be moved to two passes).
    base = chw.Plan(sizes, dtype="f32")
    ws0 = base.workspace_size()
    assert ws0 == 4 * sum(1 << k for k in sizes if k > 12)
    for opts in (dict(single15=0), dict(exec=2), dict(split_l1=9), dict(lr15=6, single15=0)):
        p = chw.Plan(sizes, dtype="f32")
        try:
            for k, v in opts.items():
                p.set_option(k, v)
        except chw.CHWError:
            continue
        assert p.workspace_size() == ws0
        p.check()


def test_dependency_queue_exec_is_disabled():
    p = chw.Plan([20, 20], dtype="f32")
    with pytest.raises(chw.CHWError) as e:
        p.set_option("exec", 1)
    assert e.value.name == "CHW_ERR_UNSUPPORTED"


def test_persistent_plan_shape():
    # default (2^15-element tiles): 2 whole-signal items (20, 20), one tile
    # for the single-pass 2^14 signal and one with the three 2^9 signals
    p = chw.Plan([20, 20, 14, 9, 9, 9], dtype="f32", persistent=True)
    d = p.describe()["plan"]
    assert d["config"]["exec"] == 2 and d["config"]["ptile"] == 0
    assert len(d["forward"]) == 1 and d["forward"][0]["persistent"] == 1
    assert d["forward"][0]["K"] == 15
    assert d["backward"] == d["forward"]
    assert d["items"] == 4 and d["multi"] == 2
    assert all(s["K1"] == 15 and s["K2"] == 15 and s["rows_log2"] == 7 for s in d["splits"])
    p.check()
    # 2^12-element tiles: 3 whole-signal items (20, 20 with 2^4-row first
    # passes, 14 with 2^6 rows) + 1 tile with the three 2^9 signals
    q = chw.Plan([20, 20, 14, 9, 9, 9], dtype="f32", persistent=True)
    q.set_option("ptile", 12)
    d = q.describe()["plan"]
    assert d["forward"][0]["K"] == 12
    assert d["items"] == 4 and d["multi"] == 3
    assert sorted((s["m"], s["rows_log2"]) for s in d["splits"]) == [(14, 6), (20, 4)]
    q.check()
    # signals of 2^22 and 2^23 only in 2^15-element tiles; FP64 only in 2^12
    r = chw.Plan([23, 22, 5], dtype="bf16", persistent=True)
    r.check()
    with pytest.raises(chw.CHWError):
        r.set_option("ptile", 12)
    f = chw.Plan([20, 9], dtype="f64", persistent=True)
    assert f.describe()["plan"]["forward"][0]["K"] == 12
    with pytest.raises(chw.CHWError):
        f.set_option("ptile", 15)


def test_stream_plan_shape():
    # uniform 2^20 batch: the first pass runs 2^15-element tiles (FIRST_A,
    # prefetching), the last pass 2^12-element tiles (one workgroup each)
    p = chw.Plan([20] * 8, dtype="f32")
    d = p.describe()["plan"]
    assert d["config"]["stream"] == 1
    assert [r["K"] for r in d["forward"]] == [15, 12]
    assert [r["stream"] for r in d["forward"]] == [1 + 1, 0]
    assert [r["stream"] for r in d["backward"]] == [0, 1 + 1]
    p.check()
    p.set_option("stream", 0)
    assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [0, 0]
    # 2^22 signals: both passes in 2^15-element tiles
    p = chw.Plan([22] * 2, dtype="f32")
    assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [1 + 1, 1 + 3]
    p.check()
    # single-pass 2^15-element tiles with offset lists stay one workgroup per tile
    offs = np.arange(9, dtype=np.int64) * (1 << 14)
    p = chw.Plan([13] * 8, dtype="f32", offsets=offs)
    assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [0]
    p.check()
    # full single-pass tiles of several signals prefetch only when forced
    # (packed: without spreading, 8 signals of 2^13 fill two tiles)
    p = chw.Plan([13] * 8, dtype="bf16")
    p.set_option("spread", 0)
    assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [0]
    p.set_option("stream", 2)
    assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [1]
    p.check()
    with pytest.raises(chw.CHWError):
        p.set_option("stream", 3)
    # one 2^15 signal per tile: from 1024 tiles on by default
    for b, want in ((1023, 0), (1024, 1)):
        p = chw.Plan([15] * b, dtype="f32")
        assert [r["stream"] for r in p.describe()["plan"]["forward"]] == [want], b
        assert [r["stream"] for r in p.describe()["plan"]["backward"]] == [want], b
        p.check()


def test_plan_invariants_workloads():
    import workloads
    ks = workloads.ragged_log2_sizes(4001)
    offs = workloads.packed_offsets(ks)
    for persistent in (False, True):
        p = chw.Plan(ks, dtype="bf16", offsets=offs, persistent=persistent)
        p.check()
    p = chw.Plan([20] * 1024, dtype="f32")
    p.check()
    p = chw.Plan([24] * 16, dtype="f32")
    p.check()


# ---- signed (random-sign diagonal) entry points: host-side validation --------

def _aligned(buf, align=16):
    return (ctypes.addressof(buf) + align - 1) & ~(align - 1)


def test_sign_words():
    p = chw.Plan([10, 12, 3], dtype="f32")
    assert p.sign_words("shared") == (1 << 12) // 32
    assert p.sign_words("per_element") == (1024 + 4096 + 8 + 31) // 32
    q = chw.Plan([2], dtype="f32")
    assert q.sign_words("shared") == 1 and q.sign_words("per_element") == 1
    n = ctypes.c_size_t()
    assert chw.load().chw_sign_words(p.handle, 7, ctypes.byref(n)) == 1


def test_signed_argument_validation():
    lib = chw.load()
    p = chw.Plan([20, 20], dtype="f32")
    buf = (ctypes.c_char * 256)()
    a = _aligned(buf)
    x = ctypes.c_void_p(a)
    y = ctypes.c_void_p(a + 64)   # distinct, non-overlapping only in address terms
    s = ctypes.c_void_p(a + 128)
    fs, bs = lib.chw_forward_signed, lib.chw_backward_signed
    # NULL plan / NULL signs / misaligned signs / rounds out of range / bad mode
    assert fs(None, x, x, None, s, 1, 1, None) == 1
    assert fs(p.handle, x, x, None, None, 1, 1, None) == 1
    assert fs(p.handle, x, x, None, ctypes.c_void_p(a + 130), 1, 1, None) == 3
    assert fs(p.handle, x, x, None, s, 1, 0, None) == 1
    assert fs(p.handle, x, x, None, s, 1, 65, None) == 1
    assert bs(p.handle, x, x, None, s, 9, 1, None) == 1
    assert "rounds" in lib.chw_last_error().decode() or lib.chw_last_error()
    # several rounds of an out-of-place two-pass call need a workspace (the
    # later rounds run in place on y); checked before any device access
    big = (ctypes.c_char * ((16 << 20) + 64))()
    b = _aligned(big)
    xb, yb = ctypes.c_void_p(b), ctypes.c_void_p(b + (8 << 20))
    st = fs(p.handle, xb, yb, None, s, 1, 3, None)
    assert st == 1 and "workspace" in lib.chw_last_error().decode()


def test_out_of_place_intermediate_through_y_dyadic_only():
    # an out-of-place forward call without a workspace routes the two-pass
    # intermediate through y only in the dyadic order: there every last-pass
    # tile stores into the blocks it loaded, while the sequency order's tile
    # for block g stores into block invgray(g) and the natural order's into
    # runs across the signal, blocks other tiles have yet to load.  Checked
    # before any device access.
    lib = chw.load()
    big = (ctypes.c_char * ((16 << 20) + 64))()
    b = _aligned(big)
    xb, yb = ctypes.c_void_p(b), ctypes.c_void_p(b + (8 << 20))
    for order in ("sequency", "natural"):
        p = chw.Plan([20, 20], dtype="f32", order=order)
        assert lib.chw_forward(p.handle, xb, yb, None, None) == 1, order
        assert "workspace" in lib.chw_last_error().decode()
    p = chw.Plan([20, 20], dtype="f32")
    st = lib.chw_forward(p.handle, xb, yb, None, None)
    assert st != 1 and "workspace" not in lib.chw_last_error().decode()


# ---- coefficient orders: host-side plan shape --------------------------------

def test_order_flags_and_plan_shape():
    lib = chw.load()
    st, h = _plan_raw([10], flags=(1 << 4) | (1 << 5))
    assert st == 1 and "exclusive" in lib.chw_last_error().decode()
    st, h = _plan_raw([10], flags=(1 << 4) | (1 << 2))
    assert st == 2
    for order, code in (("dyadic", 0), ("sequency", 1), ("natural", 2)):
        p = chw.Plan([20] * 4 + [13] * 3 + [1], dtype="f32", order=order)
        d = p.describe()["plan"]
        assert d["config"]["order"] == code
        if code:
            # the forward prefetches like the dyadic one (full 2^15-element
            # tiles of one kind); the adjoint gathers by the order's map, one
            # workgroup per tile
            assert d["config"]["stream"] == 1
            assert any(r["stream"] > 0 for r in d["forward"])
            assert all(r["stream"] == 0 for r in d["backward"])
        if code == 2:
            # the natural order's last pass takes the larger tiles (longer runs
            # of its transposed store)
            assert d["splits"][0]["K2"] == 15
        p.check()
        with pytest.raises(chw.CHWError):
            q = chw.Plan([20] * 4, dtype="f32", order=order)
            if code:
                q.set_option("exec", 2)
            else:
                raise chw.CHWError(1, "dyadic accepts exec 2")


def test_pipelined_chunks_plan_shape():
    p = chw.Plan([20] * 8, dtype="f32")
    p.set_option("chunk", 3 << 20)
    p.set_option("pipeline", 1)
    d = p.describe()["plan"]
    assert d["splits"][0]["K2"] == 15            # both passes in 2^15-element tiles
    per = (1 << (20 - d["splits"][0]["L1"])) >> d["splits"][0]["rows_log2"]
    lens = [r["end"] - r["begin"] for r in d["forward"]]
    assert lens == [3 * per, 3 * 32 + 3 * per, 3 * 32 + 2 * per, 2 * 32]
    assert len(d["backward"]) == 4
    assert d["ws_elems"] == 2 * 3 << 20            # two slots of the largest chunk
    assert p.workspace_size() == 8 << 22           # the reported bound is unchanged
    p.check()


def test_haar_walsh_plan_shape_and_haar_validation():
    lib = chw.load()
    p = chw.Plan.haar_walsh(3, 5, dtype="f32")
    d = p.describe()
    assert d["batch"] == 3 * 6 and d["extent"] == 3 * 32
    p.check()
    h = ctypes.c_void_p()
    assert lib.chw_plan_haar_walsh(ctypes.byref(h), 2, 31, 0, 0, 0) == 1
    assert lib.chw_plan_haar_walsh(ctypes.byref(h), -1, 5, 0, 0, 0) == 1
    assert lib.chw_plan_haar_walsh(None, 2, 5, 0, 0, 0) == 1
    # Haar calls: distinct buffers, and a workspace for signals above 2^12
    q = chw.Plan([14, 3], dtype="f32")
    buf = (ctypes.c_char * ((1 << 17) + 256))()
    a = _aligned(buf)
    x, y = ctypes.c_void_p(a), ctypes.c_void_p(a + 65600)
    assert lib.chw_haar_forward(q.handle, x, x, None, None) == 1
    assert lib.chw_haar_forward(q.handle, x, y, None, None) == 1
    assert "workspace" in lib.chw_last_error().decode()
    assert lib.chw_haar_backward(None, x, y, None, None) == 1


def test_philox_signs_argument_validation():
    # every argument check comes before any device access (status 5 = no device)
    lib = chw.load()
    p = chw.Plan([10, 12], dtype="f32")
    buf = (ctypes.c_char * 64)()
    a = _aligned(buf)
    ph = lib.chw_philox_signs
    assert ph(None, 1, 5, 1, ctypes.c_void_p(a), None) == 1
    assert ph(p.handle, 1, 5, 1, None, None) == 1
    assert ph(p.handle, 1, 5, 1, ctypes.c_void_p(a + 2), None) == 3
    assert ph(p.handle, 1, 5, 0, ctypes.c_void_p(a), None) == 1
    assert ph(p.handle, 1, 5, 65, ctypes.c_void_p(a), None) == 1
    assert ph(p.handle, 9, 5, 1, ctypes.c_void_p(a), None) == 1
    assert ph(p.handle, 1, 5, 1, ctypes.c_void_p(a + 4), None) == 5


def test_nodes_validation():
    # plan restrictions and argument checks come before any device access
    lib = chw.load()
    buf = (ctypes.c_char * 256)()
    a = _aligned(buf)
    x, y, w = ctypes.c_void_p(a), ctypes.c_void_p(a + 64), ctypes.c_void_p(a + 128)
    n = ctypes.c_size_t()
    p = chw.Plan([20] * 4, dtype="f32")
    assert lib.chw_nodes_workspace_size(p.handle, ctypes.byref(n)) == 0
    assert n.value == 4 * (4 * (1 << 20) + 4 * (1 << 8))
    q = chw.Plan([10] * 3, dtype="f32")
    assert q.nodes_workspace_size() == 4 * 3 * 1024
    for bad in (chw.Plan([20] * 2, dtype="bf16"), chw.Plan([10, 11], dtype="f32"),
                chw.Plan([25], dtype="f32"), chw.Plan([8] * 2, dtype="f32", order="sequency"),
                chw.Plan([8] * 2, dtype="i32", norm="none"),
                chw.Plan([8] * 2, dtype="f32", offsets=[0, 512, 1024])):
        assert lib.chw_nodes_workspace_size(bad.handle, ctypes.byref(n)) == 2
        assert lib.chw_nodes_forward(bad.handle, x, y, w, 0, None) == 2
    assert lib.chw_nodes_forward(None, x, y, w, 0, None) == 1
    assert lib.chw_nodes_forward(q.handle, None, y, w, 0, None) == 1
    assert lib.chw_nodes_forward(q.handle, x, y, None, 0, None) == 1
    assert lib.chw_nodes_forward(q.handle, x, y, w, -1, None) == 1
    assert lib.chw_nodes_forward(q.handle, ctypes.c_void_p(a + 2), y, w, 0, None) == 3
    assert lib.chw_nodes_forward(q.handle, x, x, w, 0, None) == 1


def test_turn_plan_shape():
    # round-boundary tiles: one 2^15-element tile per 2^15 elements of every
    # two-pass signal, only where the plan qualifies
    sizes = [16, 20, 21, 24, 25, 12, 3]
    p = chw.Plan(sizes, dtype="f32")
    p.check()
    turn = p.describe()["plan"]["turn"]
    # one launch per first-pass row count: 2^7 rows (m = 16, 20, 21), 2^6 (24),
    # 2^5 (25)
    assert len(turn) == 3 and all(r["K"] == 15 and r["stream"] == 8 for r in turn)
    assert sum(r["end"] - r["begin"] for r in turn) == sum(1 << (k - 15) for k in sizes if k > 15)
    assert [r["end"] - r["begin"] for r in turn] == [2 + 32 + 64, 512, 1024]
    # 2^3 rows: a forced first pass of 12 levels
    b = chw.Plan([20] * 2, dtype="f32")
    b.set_option("split_l1", 12)
    b.check()
    assert [r["end"] - r["begin"] for r in b.describe()["plan"]["turn"]] == [64]
    # three-pass signals take no round-boundary tiles: the plan has none
    assert chw.Plan([26, 20], dtype="f32").describe()["plan"]["turn"] == []
    q = chw.Plan(sizes, dtype="f32")
    q.set_option("stream", 0)
    q.check()
    assert all(r["stream"] == 0 for r in q.describe()["plan"]["turn"])
    assert chw.Plan([20] * 2, dtype="i32", norm="none").describe()["plan"]["turn"]
    for none in (chw.Plan([20] * 2, dtype="bf16"), chw.Plan([20] * 2, dtype="f64"),
                 chw.Plan([20] * 2, dtype="f32", order="natural"),
                 chw.Plan([20] * 2, dtype="f32", persistent=True),
                 chw.Plan([12, 3], dtype="f32")):
        none.check()
        assert none.describe()["plan"]["turn"] == []
    # forced splits whose last-pass blocks are below 2^8 take no round-boundary tiles
    f = chw.Plan([16] * 4, dtype="f32")
    f.set_option("split_l1", 12)
    f.check()
    assert f.describe()["plan"]["splits"][0]["L1"] == 12
    assert f.describe()["plan"]["turn"] == []
    for key, val in (("turn", 0), ("chunk", 1 << 21), ("split_l1", 6)):
        r = chw.Plan([20] * 4, dtype="f32")
        r.set_option(key, val)
        r.check()
        assert r.describe()["plan"]["turn"] == [], key


def test_adjoint_option():
    # chw_backward of a dyadic plan runs the forward launches unless option
    # "adjoint" asks for the synthesis kernels; the option is fixed on use
    # like the planner choices
    p = chw.Plan([20] * 2 + [9] * 3, dtype="f32")
    assert p.describe()["plan"]["config"]["adjoint"] == 0
    p.set_option("adjoint", 1)
    assert p.describe()["plan"]["config"]["adjoint"] == 1
    with pytest.raises(chw.CHWError):
        p.set_option("adjoint", 2)
    p.check()


def test_caller_workspace_is_checked():
    # a caller-supplied workspace too small, strided or on another device is
    # rejected by the binding before any call (the library cannot see its size)
    import torch
    p = chw.Plan([16, 12], dtype="bf16")
    need = p.workspace_size()
    assert need > 0
    x = torch.zeros(p.extent, dtype=torch.bfloat16)
    ok = torch.empty(need, dtype=torch.uint8)
    assert p._check_workspace(ok, x, need) is ok
    assert p._check_workspace(None, x, need) is None
    with pytest.raises(ValueError, match="needs"):
        p._check_workspace(torch.empty(need - 1, dtype=torch.uint8), x, need)
    with pytest.raises(ValueError, match="needs"):
        p._check_workspace(torch.empty(need // 4 - 1, dtype=torch.float32), x, need)
    with pytest.raises(ValueError, match="contiguous"):
        p._check_workspace(torch.empty(2 * need, dtype=torch.uint8)[::2], x, need)
    with pytest.raises(ValueError, match="device"):
        p._check_workspace(torch.empty(need, dtype=torch.uint8, device="meta"), x, need)
    with pytest.raises(TypeError):
        p._check_workspace(np.empty(need, dtype=np.uint8), x, need)


def test_stream_argument_forms():
    assert chw._stream_ptr(0, None) == 0
    assert chw._stream_ptr(12345, None) == 12345

    class S:
        cuda_stream = 777
    assert chw._stream_ptr(S(), None) == 777


def test_tuning_cache_roundtrip(tmp_path):
    # a tuning file written by hand is loaded; plans of its key start from the
    # entry unless made with FLAG_NO_AUTOTUNE; save writes it back
    chw.tuning_clear()
    assert chw.tuning_count() == 0
    ks = [20] * 8 + [12] * 100
    p0 = chw.Plan(ks, dtype="bf16")
    key = p0.describe()["tuning_key"]
    assert p0.describe()["tuned"] == 0
    f = tmp_path / "t.txt"
    f.write_text("# comment\n\n%s lr12=5 lr15=6 single15=1 split_l1=10 exec=0 ptile=0 chunk=0 "
                 "stream=0 pipeline=0 spread=1 occupancy=3\n" % key)
    chw.tuning_load(str(f))
    assert chw.tuning_count() == 1
    p1 = chw.Plan(ks, dtype="bf16")
    d = p1.describe()
    assert d["tuned"] == 1
    c = d["plan"]["config"]
    assert (c["lr12"], c["lr15"], c["split_l1"], c["stream"], c["occupancy"]) == (5, 6, 10, 0, 3)
    assert all(sp["L1"] == 10 for sp in d["plan"]["splits"])
    p2 = chw.Plan(ks, dtype="bf16", flags=chw.FLAG_NO_AUTOTUNE)
    assert p2.describe()["tuned"] == 0
    assert p2.describe()["plan"]["config"]["split_l1"] == -1
    # another dtype, size mix or launch form has another key
    assert chw.Plan(ks, dtype="f32").describe()["tuned"] == 0
    assert chw.Plan(ks + [12] * 200, dtype="bf16").describe()["tuned"] == 0
    assert chw.Plan(ks, dtype="bf16", persistent=True).describe()["tuned"] == 0
    # an option set by the caller replaces the tuned choice
    p1.set_option("lr15", 5)
    assert p1.describe()["tuned"] == 0
    g = tmp_path / "out.txt"
    chw.tuning_save(str(g), comment="made by a test\nsecond line")
    text = g.read_text()
    assert "# made by a test" in text and "# second line" in text
    assert key in text and "occupancy=3" in text
    chw.tuning_clear()
    chw.tuning_load(str(g))
    assert chw.Plan(ks, dtype="bf16").describe()["tuned"] == 1
    chw.tuning_clear()


@pytest.mark.parametrize("line", [
    "k lr12=5",                                                  # options missing
    "k lr12=5 lr15=6 single15=1 split_l1=10 exec=0 ptile=0 chunk=0 stream=0 pipeline=0 spread=1 occupancy=99",
    "k lr12=5 lr15=6 single15=1 split_l1=10 exec=0 ptile=0 chunk=0 stream=0 pipeline=0 spread=1 occupancy=1 bogus=1",
    "k lr12=5 lr12=5 lr15=6 single15=1 split_l1=10 exec=0 ptile=0 chunk=0 stream=0 pipeline=0 spread=1",
    "k lr12=x lr15=6 single15=1 split_l1=10 exec=0 ptile=0 chunk=0 stream=0 pipeline=0 spread=1 occupancy=1",
    "k lr12= lr15=6",
    "k =5",
])
def test_tuning_file_rejects_malformed_lines(tmp_path, line):
    chw.tuning_clear()
    f = tmp_path / "bad.txt"
    f.write_text("# ok\n" + line + "\n")
    with pytest.raises(chw.CHWError) as e:
        chw.tuning_load(str(f))
    assert e.value.name == "CHW_ERR_INVALID_ARGUMENT" and ":2:" in e.value.detail
    assert chw.tuning_count() == 0
    with pytest.raises(chw.CHWError):
        chw.tuning_load(str(tmp_path / "missing.txt"))


def test_occupancy_option():
    p = chw.Plan([20] * 4, dtype="f32", persistent=True)
    p.set_option("occupancy", 2)
    assert p.describe()["plan"]["config"]["occupancy"] == 2
    with pytest.raises(chw.CHWError):
        p.set_option("occupancy", 33)


@pytest.mark.parametrize("sizes,flag", [([26], False), ([29], False), ([30, 20, 12, 3], False),
                                        ([20, 20, 12], True), ([23, 21, 16, 10, 2], True)])
def test_three_pass_plan_shape(sizes, flag):
    # signals above 2^25 (or of 2^20 and more with the THREE_PASS flag) take a
    # first pass into one intermediate, a middle pass between the two
    # intermediates and a last pass into y; the forward runs them in that
    # order and the adjoint in reverse, the workspace holds both intermediates
    p = chw.Plan(sizes, three_pass=flag)
    p.check()
    d = p.describe()["plan"]
    lim = 20 if flag else 26
    three = [m for m in sizes if m >= lim]
    assert d["three"] == len(three)
    assert sorted(q["m"] for q in d["splits3"]) == sorted(set(three))
    for q in d["splits3"]:
        assert q["L1"] + q["L2"] < q["m"] and q["m"] - q["L1"] - q["L2"] <= q["K3"]
    roles = [r["role"] for r in d["forward"]]
    assert roles.count(1) >= 1 and [r["role"] for r in d["backward"]].count(1) == roles.count(1)
    mid = [i for i, r in enumerate(d["forward"]) if r["role"] == 1]
    # elements through the middle pass: the three-pass signals once
    assert sum(d["forward"][i]["elements"] for i in mid) == sum(1 << m for m in three)
    two = sum(1 << m for m in sizes if 12 < m < lim)
    assert p.workspace_size() == 4 * (two + 2 * sum(1 << m for m in three))
    # options do not change the workspace bound
    for k, v in (("lr12", 5), ("lr15", 6), ("stream", 0), ("chunk", 1 << 22)):
        q = chw.Plan(sizes, three_pass=flag)
        q.set_option(k, v)
        q.check()
        assert q.workspace_size() == p.workspace_size()


@pytest.mark.parametrize("seed", range(6))
def test_three_pass_random_plans(seed):
    rng = np.random.default_rng(4400 + seed)
    sizes = sorted((int(v) for v in rng.integers(0, 25, int(rng.integers(1, 12)))), reverse=True)
    p = chw.Plan(sizes, dtype=["f32", "bf16", "i32"][seed % 3],
                 norm="none" if seed % 3 == 2 else "ortho", three_pass=True)
    for k, v in (("lr12", int(rng.choice([5, 6]))), ("lr15", int(rng.choice([5, 6]))),
                 ("stream", int(rng.integers(0, 3))), ("single15", int(rng.integers(0, 2)))):
        p.set_option(k, v)
    p.check()
    assert p.describe()["plan"]["three"] == sum(1 for m in sizes if m >= 20)


def test_other_orders_keep_two_passes_to_2p27():
    for order in ("sequency", "natural"):
        for m in (26, 27):
            p = chw.Plan([m], order=order)
            p.check()
            d = p.describe()["plan"]
            assert d["three"] == 0 and len(d["splits"]) == 1
            assert p.workspace_size() == 4 << m
        with pytest.raises(chw.CHWError):
            chw.Plan([28], order=order)


def test_library_loads_after_torch():
    # torch's HIP runtime carries the same soname as the system one; libchw
    # binds to whichever the process loaded first, so loading it must bring
    # torch in first (else torch would map a second runtime that sees no
    # device).  Checked in a fresh interpreter.
    import subprocess
    import sys
    code = ("import sys; from paper_1609_06641_amd import chw; "
            "assert 'torch' not in sys.modules; chw.load(); "
            "assert 'torch' in sys.modules; print('ok')")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stderr[-2000:]
