"""Parity of the HIP path with the oracle (GPU).  Every comparison is element
by element against the plain CPU oracle on the same seeded inputs."""

import numpy as np
import pytest

import workloads
from oracle import cascade, metrics
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    t = gu.torch()
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    chw.load()


def _sync():
    gu.torch().cuda.synchronize()


# ---------------------------------------------------------------------------
# the small plain workload: 64 x 2^10, float32 orthonormal and int32 exact

def test_plain_small_f32():
    w = workloads.CONFIGS["plain_small_f32"]
    x = workloads.float_signals(w.seed, w.batch, 10)
    p = chw.Plan([10] * w.batch, dtype="f32")
    y = p.forward(gu.dev_tensor(x, "f32"))
    _sync()
    ref = cascade.chw_forward(x.astype(np.float64))
    rel = metrics.rel_l2(gu.host_f64(y).reshape(w.batch, -1), ref)
    print("max rel-L2", rel.max())
    assert rel.max() <= 1e-5


def test_plain_small_i32_bit_exact():
    w = workloads.CONFIGS["plain_small_i32"]
    x = workloads.int_signals(w.seed, w.batch, 10)
    p = chw.Plan([10] * w.batch, dtype="i32", norm="none")
    y = p.forward(gu.dev_tensor(x, "i32"))
    _sync()
    ref = cascade.chw_forward(x.astype(np.int64))
    assert np.abs(ref).max() < 2 ** 31
    assert np.array_equal(gu.host_i64(y).reshape(w.batch, -1), ref)


# ---------------------------------------------------------------------------
# every size 0..22: single pass, two passes, in place and out of place

def _batch_for(m):
    return 3 if m <= 16 else (2 if m <= 20 else 1)


@pytest.mark.parametrize("m", list(range(0, 23)))
def test_sizes_f32_i32(m):
    b = _batch_for(m)
    xf = workloads.float_signals(100 + m, b, m)
    xi = workloads.int_signals(200 + m, b, m)
    sizes = [m] * b
    pf = chw.Plan(sizes, dtype="f32")
    pi = chw.Plan(sizes, dtype="i32", norm="none")
    ref_f = gu.oracle_packed(xf.reshape(-1).astype(np.float64), sizes)
    ref_i = gu.oracle_packed(xi.reshape(-1).astype(np.int64), sizes)
    # out of place (no workspace)
    yf = pf.forward(gu.dev_tensor(xf.reshape(-1), "f32"))
    yi = pi.forward(gu.dev_tensor(xi.reshape(-1), "i32"))
    # in place (workspace when two passes)
    tf = gu.dev_tensor(xf.reshape(-1), "f32")
    pf.forward(tf, out=tf)
    ti = gu.dev_tensor(xi.reshape(-1), "i32")
    pi.forward(ti, out=ti)
    _sync()
    for got in (yf, tf):
        rel = gu.per_signal_rel(gu.host_f64(got), ref_f, sizes)
        assert rel.max() <= 1e-5, (m, rel.max())
    assert np.abs(ref_i).max() < 2 ** 31
    for got in (yi, ti):
        assert np.array_equal(gu.host_i64(got), ref_i), m


@pytest.mark.parametrize("m", [3, 10, 12, 14, 16, 20])
def test_backward_equals_forward_and_oracle(m):
    # H is symmetric: the reversed cascade of transposed factors gives the
    # same numbers; with the same butterfly operands and the scale applied
    # last, bitwise the same.
    b = _batch_for(m)
    x = workloads.float_signals(300 + m, b, m).reshape(-1)
    sizes = [m] * b
    p = chw.Plan(sizes, dtype="f32")
    p.set_option("adjoint", 1)  # the synthesis kernels (forward launches: next test)
    xd = gu.dev_tensor(x, "f32")
    yf = p.forward(xd)
    yb = p.backward(xd)
    _sync()
    assert np.array_equal(gu.host_f64(yf), gu.host_f64(yb))
    ref = gu.oracle_packed(x.astype(np.float64), sizes, adjoint=True)
    assert gu.per_signal_rel(gu.host_f64(yb), ref, sizes).max() <= 1e-5
    xi = workloads.int_signals(400 + m, b, m).reshape(-1)
    pi = chw.Plan(sizes, dtype="i32", norm="none")
    pi.set_option("adjoint", 1)
    ybi = pi.backward(gu.dev_tensor(xi, "i32"))
    _sync()
    assert np.array_equal(gu.host_i64(ybi), gu.oracle_packed(xi.astype(np.int64), sizes,
                                                              adjoint=True))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i32", "f64"])
def test_backward_default_runs_forward_launches(dtype):
    # chw_backward of a dyadic plan runs the forward launches by default; the
    # synthesis kernels (option "adjoint" = 1) give the same bits, and so
    # does the oracle's adjoint cascade up to rounding
    rng = np.random.default_rng(81)
    sizes = [int(k) for k in rng.integers(3, 13, size=40)] + ([16, 20, 14] if dtype != "f64" else [16, 14])
    norm = "none" if dtype == "i32" else "ortho"
    x = np.concatenate([(workloads.int_signals(810 + i, 1, k) if dtype == "i32"
                         else workloads.float_signals(810 + i, 1, k)).reshape(-1)
                        for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, dtype)
    t = gu.torch()
    p = chw.Plan(sizes, dtype=dtype, norm=norm)
    q = chw.Plan(sizes, dtype=dtype, norm=norm)
    q.set_option("adjoint", 1)
    assert p.describe()["plan"]["config"]["adjoint"] == 0
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    yf = p.forward(xd, workspace=ws)
    yb = p.backward(xd, workspace=ws)
    ys = q.backward(xd, workspace=ws)
    _sync()
    assert t.equal(yf, yb) and t.equal(yb, ys)
    if dtype == "i32":
        assert np.array_equal(gu.host_i64(yb), gu.oracle_packed(x.astype(np.int64), sizes,
                                                                 adjoint=True))
    else:
        ref = gu.oracle_packed(gu.host_f64(xd), sizes, adjoint=True)
        assert gu.per_signal_rel(gu.host_f64(yb), ref, sizes).max() <= gu.TOL[dtype]


@pytest.mark.parametrize("m", [23, 24, 25])
def test_large_two_pass_sizes(m):
    # the two-pass sizes above the sweep, each with its own first-pass row count
    # in 2^15-element tiles (m = 23: 2^7 rows, 24: 2^6, 25: 2^5): forward and
    # the synthesis kernels, out of place and in place, against the oracle;
    # int32 bit for bit (inputs in [-8, 7], so |y| < 2^28); and the same bits
    # as the neighbouring first-pass splits
    t = gu.torch()
    xf = workloads.float_signals(900 + m, 1, m).reshape(-1)
    xi = workloads.int_signals(950 + m, 1, m, lo=-8, hi=7).reshape(-1)
    ref_f = gu.oracle_packed(xf.astype(np.float64), [m])
    ref_i = gu.oracle_packed(xi.astype(np.int64), [m])
    outs = {}
    for l1 in (-1, 8, 9, 10):
        if l1 > 0 and not 6 <= m - l1 <= 15:
            continue
        pf = chw.Plan([m], dtype="f32")
        pf.set_option("split_l1", l1)
        pa = chw.Plan([m], dtype="f32")
        pa.set_option("split_l1", l1)
        pa.set_option("adjoint", 1)
        pi = chw.Plan([m], dtype="i32", norm="none")
        pi.set_option("split_l1", l1)
        xd = gu.dev_tensor(xf, "f32")
        yf = pf.forward(xd)
        yb = pa.backward(xd)
        tf = gu.dev_tensor(xf, "f32")
        pf.forward(tf, out=tf)
        yi = pi.forward(gu.dev_tensor(xi, "i32"))
        _sync()
        assert t.equal(yf, tf) and t.equal(yf, yb), (m, l1)
        outs[l1] = yf
        assert gu.per_signal_rel(gu.host_f64(yf), ref_f, [m]).max() <= 1e-5, (m, l1)
        assert np.array_equal(gu.host_i64(yi), ref_i), (m, l1)
    assert all(t.equal(o, outs[-1]) for o in outs.values())
    # the prefetching forms of every launch (the default leaves the 2^6-row
    # first pass to one workgroup per tile)
    p2 = chw.Plan([m], dtype="f32")
    p2.set_option("stream", 2)
    d = p2.describe()["plan"]
    assert all(r["stream"] > 0 for r in d["forward"])
    y2 = p2.forward(gu.dev_tensor(xf, "f32"))
    _sync()
    assert t.equal(y2, outs[-1])
    # the sequency order: the same values, rows listed by sign changes
    ps = chw.Plan([m], dtype="f32", order="sequency")
    ys = ps.forward(gu.dev_tensor(xf, "f32"))
    _sync()
    k = np.arange(1 << m, dtype=np.int64)
    assert np.array_equal(gu.host_f64(ys), gu.host_f64(outs[-1])[k ^ (k >> 1)])


# ---------------------------------------------------------------------------
# precision forms: bf16 / f16 storage, FP32 inside every pass

@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("m,batch", [(12, 8192), (6, 64), (14, 16), (17, 4), (20, 2)])
def test_precision_forms(dtype, m, batch):
    x32 = workloads.outlier_signals(3001 if m == 12 else 3100 + m, batch, m)
    xh = workloads.to_half_precision(x32, dtype)          # RNE-rounded inputs
    x64 = xh.to(gu.torch().float64).numpy().reshape(-1)  # exact
    sizes = [m] * batch
    p = chw.Plan(sizes, dtype=dtype)
    p.set_option("adjoint", 1)  # backward through the synthesis kernels
    y = p.forward(gu.dev_tensor(xh.reshape(-1), dtype))
    yb = p.backward(gu.dev_tensor(xh.reshape(-1), dtype))
    _sync()
    ref = gu.oracle_packed(x64, sizes, threads=16)
    rel = gu.per_signal_rel(gu.host_f64(y), ref, sizes)
    print("%s m=%d max rel-L2 %.3e pooled %.3e" % (dtype, m, rel.max(),
          metrics.pooled_rel_l2(gu.host_f64(y), ref)))
    assert rel.max() <= 4e-3
    assert np.array_equal(gu.host_f64(y), gu.host_f64(yb))


# ---------------------------------------------------------------------------
# ragged batches with gaps: sentinels in the gaps stay untouched

@pytest.mark.parametrize("dtype", ["f32", "i32", "bf16", "f16", "f64"])
def test_ragged_with_gaps(dtype):
    rng = np.random.default_rng(77)
    ms = rng.integers(0, 19 if dtype != "f64" else 17, size=40).astype(np.int32)
    ms[:6] = [0, 1, 2, 3, 12, 16]
    es = {"f32": 4, "i32": 4, "bf16": 2, "f16": 2, "f64": 8}[dtype]
    align = 16 // es
    offs = []
    o = 0
    for k in ms:
        o += int(rng.integers(0, 3)) * align          # gap before the signal
        offs.append(o)
        o += max(1 << int(k), align)
    offs.append(o + align)
    offs = np.array(offs, dtype=np.int64)
    total = int(offs[-1])
    norm = "none" if dtype == "i32" else "ortho"
    if dtype == "i32":
        x = rng.integers(-128, 128, size=total).astype(np.int32)
        sentinel = 123456789
    else:
        x = rng.standard_normal(total).astype(np.float32)
        sentinel = 4242.0
    p = chw.Plan(ms, dtype=dtype, norm=norm, offsets=offs)
    xd = gu.dev_tensor(x, dtype)
    y = gu.dev_tensor(np.full(total, sentinel, dtype=x.dtype), dtype)
    p.forward(xd, out=y)
    _sync()
    mask = np.ones(total, dtype=bool)
    for k, o in zip(ms, offs[:-1]):
        mask[o:o + (1 << int(k))] = False
    if dtype == "i32":
        got = gu.host_i64(y)
        ref = gu.oracle_packed(x.astype(np.int64), ms, offs)
        assert np.array_equal(got[~mask], ref[~mask])
        assert np.all(got[mask] == sentinel)
    else:
        xin = gu.host_f64(xd)
        got = gu.host_f64(y)
        ref = gu.oracle_packed(xin, ms, offs)
        rel = gu.per_signal_rel(got, ref, ms, offs)
        assert rel.max() <= gu.TOL[dtype], rel.max()
        assert np.all(got[mask] == float(gu.torch().tensor(sentinel).to(
            getattr(gu.torch(), gu.TORCH_DT[dtype])).double()))


# ---------------------------------------------------------------------------
# numerics do not depend on tiling or pass split; graph replay

def test_split_invariance_bitwise():
    sizes = [14] * 3 + [20] * 2 + [9] * 5
    x = np.concatenate([workloads.float_signals(500 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, "f32")
    outs = []
    cfgs = [dict(), dict(lr12=5), dict(lr15=6), dict(single15=0),
               dict(split_l1=9), dict(split_l1=6), dict(split_l1=12, lr15=6),
               dict(split_l1=8), dict(chunk=1 << 21), dict(exec=2), dict(exec=2, lr12=5),
               dict(stream=0), dict(stream=0, lr12=5), dict(stream=0, split_l1=12, lr15=6),
               dict(stream=0, split_l1=8, chunk=1 << 21), dict(stream=1, split_l1=6),
               dict(split_l1=10), dict(split_l1=10, stream=0),
               dict(chunk=1 << 20, pipeline=1), dict(chunk=1 << 19, pipeline=1, lr15=6)]
    for cfg in cfgs:
        p = chw.Plan(sizes, dtype="f32")
        for k, v in cfg.items():
            p.set_option(k, v)
        outs.append(gu.host_f64(p.forward(xd)))
    _sync()
    for cfg, o in zip(cfgs[1:], outs[1:]):
        assert np.array_equal(o, outs[0]), cfg
    ref = gu.oracle_packed(x.astype(np.float64), sizes)
    assert gu.per_signal_rel(outs[0], ref, sizes).max() <= 1e-5


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i32"])
def test_stream_bitwise(dtype):
    # launches of full 2^15-element tiles of one kind (single-pass 2^13 and
    # 2^15 signals, the first pass of 2^17 signals, both passes of 2^22
    # signals) in the prefetching form (forced: mode 2), forward and
    # backward, against the one-workgroup-per-tile form and the oracle
    for sizes in ([13] * 8, [15] * 2, [17] * 3, [22] * 2):
        gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
        x = np.concatenate([gen(900 + i, 1, k).reshape(-1) for i, k in enumerate(sizes)])
        xd = gu.dev_tensor(x, dtype)
        for lr in (5, 6):
            res = []
            for stream in (0, 2):
                p = chw.Plan(sizes, dtype=dtype, norm="none" if dtype == "i32" else "ortho")
                p.set_option("adjoint", 1)
                p.set_option("spread", 0)  # full tiles of several 2^13 signals
                p.set_option("lr12", lr)
                p.set_option("lr15", lr)
                p.set_option("stream", stream)
                d = p.describe()["plan"]
                assert any(r["stream"] > 0 for r in d["forward"]) == bool(stream), sizes
                assert all(r["stream"] == 0 or r["K"] == 15 for r in d["forward"] + d["backward"])
                ws = gu.torch().empty(max(p.workspace_size(), 16), dtype=gu.torch().uint8,
                                      device="cuda")
                res.append((gu.host_f64(p.forward(xd)), gu.host_f64(p.backward(xd, workspace=ws))))
            _sync()
            assert np.array_equal(res[0][0], res[1][0]), (sizes, lr)
            assert np.array_equal(res[0][1], res[1][1]), (sizes, lr)
        if dtype == "i32":
            ref = gu.oracle_packed(x.astype(np.int64), sizes)
            assert np.array_equal(res[1][0].astype(np.int64), ref)
        else:
            ref = gu.oracle_packed(gu.host_f64(xd), sizes)
            tol = 4e-3 if dtype == "bf16" else 1e-5
            assert gu.per_signal_rel(res[1][0], ref, sizes).max() <= tol


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "i32"])
def test_vector_stages_bitwise(dtype):
    # single-pass 2^12-element tiles with 2^5 registers run their first stages
    # on the loaded 16-byte vectors (two register rounds); with 2^6 registers
    # they load plainly (two rounds from bit 0).  Same bits, with gaps between
    # the signals (block lists), partial tiles and a signed round.
    rng = np.random.default_rng(77)
    ms = [int(k) for k in rng.integers(3, 13, size=61)] + [12] * 5 + [3] * 9
    align = 8
    offs, o = [], 0
    for k in ms:
        o += int(rng.integers(0, 2)) * align
        offs.append(o)
        o += max(1 << k, align)
    offs.append(o)
    offs = np.array(offs, dtype=np.int64)
    total = int(offs[-1])
    norm = "none" if dtype == "i32" else "ortho"
    x = (rng.integers(-128, 128, size=total).astype(np.int32) if dtype == "i32"
         else rng.standard_normal(total).astype(np.float32))
    xd = gu.dev_tensor(x, dtype)
    t = gu.torch()
    res = []
    for lr in (5, 6):
        p = chw.Plan(ms, dtype=dtype, norm=norm, offsets=offs)
        p.set_option("lr12", lr)
        d = p.describe()["plan"]
        assert {r["LR"] for r in d["forward"] if r["K"] == 12} == {lr}
        s = p.philox_signs(78, 1, "per_element")
        y = t.zeros_like(xd)
        ys = t.zeros_like(xd)
        p.forward(xd, out=y)
        p.forward_signed(xd, s, "per_element", 1, out=ys)
        res.append((y, ys))
    _sync()
    assert t.equal(res[0][0], res[1][0]) and t.equal(res[0][1], res[1][1])
    if dtype == "i32":
        ref = gu.oracle_packed(x.astype(np.int64), ms, offs)
        mask = np.zeros(total, dtype=bool)
        for k, o in zip(ms, offs[:-1]):
            mask[o:o + (1 << k)] = True
        assert np.array_equal(gu.host_i64(res[0][0])[mask], ref[mask])
    else:
        ref = gu.oracle_packed(gu.host_f64(xd), ms, offs)
        assert gu.per_signal_rel(gu.host_f64(res[0][0]), ref, ms, offs).max() <= gu.TOL[dtype]


@pytest.mark.parametrize("m,batch", [(15, 1024), (14, 2048), (13, 4096)])
def test_stream_default_single_pass(m, batch):
    # the default prefetching rule picks the single-pass kernel for launches
    # of 1024 or more 2^15-element tiles, of one signal or several each: same
    # bits as one workgroup per tile, and the oracle's values (first signals)
    sizes = [m] * batch
    x = workloads.float_signals(910 + m, batch, m).reshape(-1)
    xd = gu.dev_tensor(x, "f32")
    res = []
    for stream in (0, 1):
        p = chw.Plan(sizes, dtype="f32")
        p.set_option("stream", stream)
        d = p.describe()["plan"]
        assert [r["stream"] for r in d["forward"] + d["backward"]] == [stream, stream]
        ws = gu.torch().empty(max(p.workspace_size(), 16), dtype=gu.torch().uint8, device="cuda")
        res.append((gu.host_f64(p.forward(xd)), gu.host_f64(p.backward(xd, workspace=ws))))
    _sync()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    n = 64 << m
    ref = gu.oracle_packed(gu.host_f64(xd)[:n], sizes[:64])
    assert gu.per_signal_rel(res[1][0][:n], ref, sizes[:64]).max() <= 1e-5


@pytest.mark.skip(reason="the dependency-counter persistent kernel (exec 1) did not finish "
                         "within 120 s on the GPU twice; cause not established, so it is "
                         "switched off (exec 1 raises CHW_ERR_UNSUPPORTED)")
def test_split_invariance_dependency_queue():
    sizes = [14] * 3 + [20] * 2 + [9] * 5
    p = chw.Plan(sizes, dtype="f32")
    p.set_option("exec", 1)


def test_graph_replay():
    sizes = [16] * 2 + [7] * 9
    x = np.concatenate([workloads.float_signals(600 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    t = gu.torch()
    p = chw.Plan(sizes, dtype="f32", graph=True)
    p.set_option("adjoint", 1)  # the backward graph holds the synthesis kernels
    plain = chw.Plan(sizes, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    ref = gu.host_f64(plain.forward(xd))
    y = t.empty_like(xd)
    for r in range(5):
        y.fill_(float(r))
        p.forward(xd, out=y)
        _sync()
        assert np.array_equal(gu.host_f64(y), ref), r
    # new buffers: the graph is re-captured for them
    x2 = xd * 2
    y2 = t.empty_like(xd)
    p.forward(x2, out=y2)
    _sync()
    assert np.array_equal(gu.host_f64(y2), gu.host_f64(plain.forward(x2)))
    gb = p.backward(xd)
    _sync()
    assert np.array_equal(gu.host_f64(gb), ref)


def test_f64_verify_kernel():
    sizes = [6] * 4 + [12] * 2 + [16, 20]
    x = np.concatenate([np.random.default_rng(700 + i).standard_normal(1 << k)
                        for i, k in enumerate(sizes)])
    p = chw.Plan(sizes, dtype="f64")
    p.set_option("adjoint", 1)
    y = p.forward(gu.dev_tensor(x, "f64"))
    yb = p.backward(gu.dev_tensor(x, "f64"))
    _sync()
    ref = gu.oracle_packed(x, sizes)
    assert gu.per_signal_rel(gu.host_f64(y), ref, sizes).max() <= 1e-13
    assert np.array_equal(gu.host_f64(y), gu.host_f64(yb))


def test_unnormalized_float():
    sizes = [11] * 4
    x = workloads.int_signals(800, 4, 11).reshape(-1)
    p = chw.Plan(sizes, dtype="f32", norm="none")
    y = p.forward(gu.dev_tensor(x.astype(np.float32), "f32"))
    _sync()
    ref = gu.oracle_packed(x.astype(np.int64), sizes)
    assert np.array_equal(gu.host_f64(y), ref.astype(np.float64))  # exact: |y| < 2^24


def test_autotune_with_caller_sized_workspace():
    # Regression: tuning may move 2^14 signals from one pass to two; the
    # workspace sized from workspace_size() before tuning must cover that.
    t = gu.torch()
    sizes = [14] * 8
    x = workloads.float_signals(950, 8, 14).reshape(-1)
    p = chw.Plan(sizes, dtype="f32")
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    xd = gu.dev_tensor(x, "f32")
    y = t.empty_like(xd)
    p.autotune(xd, y, workspace=ws, iters=1)
    p.forward(xd, out=y, workspace=ws)
    _sync()
    ref = gu.oracle_packed(x.astype(np.float64), sizes)
    assert gu.per_signal_rel(gu.host_f64(y), ref, sizes).max() <= 1e-5


@pytest.mark.parametrize("order", ["sequency", "natural"])
def test_autotune_other_orders(order):
    # the tuner skips the candidates the planner refuses for these orders
    # (the persistent launch computes the dyadic order only) and still returns
    # a tuned plan; its output matches the oracle in the plan's order
    from oracle import orders
    t = gu.torch()
    sizes = [16, 16, 12, 9, 14]
    x = np.concatenate([workloads.float_signals(960 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    p = chw.Plan(sizes, dtype="f32", order=order, flags=chw.FLAG_NO_AUTOTUNE)
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    xd = gu.dev_tensor(x, "f32")
    y = t.empty_like(xd)
    p.autotune(xd, y, workspace=ws, iters=1)
    assert p.describe()["plan"]["config"]["exec"] == 0
    p.forward(xd, out=y, workspace=ws)
    _sync()
    dy = gu.oracle_packed(x.astype(np.float64), sizes)
    conv = orders.natural_from_dyadic if order == "natural" else orders.sequency_from_dyadic
    bounds = np.concatenate([[0], np.cumsum([1 << k for k in sizes])])
    ref = np.concatenate([conv(dy[a:b]) for a, b in zip(bounds[:-1], bounds[1:])])
    assert gu.per_signal_rel(gu.host_f64(y), ref, sizes).max() <= 1e-5


def test_autotune_records_the_tuning_cache(tmp_path):
    # a tuned configuration is kept for the process: a new plan of the same
    # key starts from it, and a saved file brings it back after a clear
    t = gu.torch()
    sizes = [17] * 6 + [11] * 40
    x = np.concatenate([workloads.float_signals(970 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    chw.tuning_clear()
    p = chw.Plan(sizes, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    y = t.empty_like(xd)
    p.autotune(xd, y, iters=1)
    cfg = p.describe()["plan"]["config"]
    assert chw.tuning_count() == 1
    q = chw.Plan(sizes, dtype="f32")
    assert q.describe()["tuned"] == 1 and q.describe()["plan"]["config"] == cfg
    f = tmp_path / "tune.txt"
    chw.tuning_save(str(f))
    chw.tuning_clear()
    chw.tuning_load(str(f))
    r = chw.Plan(sizes, dtype="f32")
    assert r.describe()["plan"]["config"] == cfg
    yr = r.forward(xd)
    _sync()
    chw.tuning_clear()
    ref = gu.oracle_packed(x.astype(np.float64), sizes)
    assert gu.per_signal_rel(gu.host_f64(yr), ref, sizes).max() <= 1e-5


def test_streams_concurrent():
    t = gu.torch()
    sizes = [18] * 2
    x = workloads.float_signals(900, 2, 18).reshape(-1)
    ref = gu.oracle_packed(x.astype(np.float64), sizes)
    p = chw.Plan(sizes, dtype="f32")
    s1, s2 = t.cuda.Stream(), t.cuda.Stream()
    xd = gu.dev_tensor(x, "f32")
    t.cuda.synchronize()
    outs = []
    for s in (s1, s2):
        with t.cuda.stream(s):
            ws = t.empty(p.workspace_size(), dtype=t.uint8, device="cuda")
            outs.append(p.forward(xd, workspace=ws, stream=s))
    t.cuda.synchronize()
    for o in outs:
        assert gu.per_signal_rel(gu.host_f64(o), ref, sizes).max() <= 1e-5


# ---------------------------------------------------------------------------
# one persistent launch (ragged batches), with graph replay

@pytest.mark.parametrize("dtype,ptile", [("f32", 12), ("bf16", 12), ("i32", 12), ("f64", 12),
                                         ("f32", 15), ("bf16", 15), ("i32", 15)])
def test_persistent_ragged(dtype, ptile):
    # one workgroup per whole multi-pass signal, in 2^12- or 2^15-element
    # tiles (2^22 and 2^23 signals in the latter only)
    rng = np.random.default_rng(1234)
    ms = rng.integers(3, 21 if dtype != "f64" else 17, size=60).astype(np.int32)
    ms[:4] = [12, 13, 16, 20] if dtype != "f64" else [12, 13, 16, 14]
    if ptile == 15:
        ms[4:6] = [23, 22]
    offs = workloads.packed_offsets(ms)
    total = int(offs[-1])
    norm = "none" if dtype == "i32" else "ortho"
    if dtype == "i32":
        x = rng.integers(-128, 128, size=total).astype(np.int32)
    else:
        x = rng.standard_normal(total).astype(np.float32 if dtype != "f64" else np.float64)
    plain = chw.Plan(ms, dtype=dtype, norm=norm, offsets=offs)
    for graph in (False, True):
        p = chw.Plan(ms, dtype=dtype, norm=norm, offsets=offs, persistent=True, graph=graph)
        p.set_option("ptile", ptile)
        p.set_option("adjoint", 1)
        d = p.describe()["plan"]
        assert len(d["forward"]) == 1 and d["forward"][0]["persistent"] == 1
        assert d["forward"][0]["K"] == ptile
        xd = gu.dev_tensor(x, dtype)
        ws = gu.torch().empty(max(p.workspace_size(), 16), dtype=gu.torch().uint8, device="cuda")
        outs = []
        for rep in range(3):
            y = p.forward(xd, workspace=ws)
            yb = p.backward(xd, workspace=ws)
            _sync()
            outs.append((gu.host_f64(y), gu.host_f64(yb)))
        ref_gpu = gu.host_f64(plain.forward(xd))
        _sync()
        for yf, ybk in outs:
            assert np.array_equal(yf, ref_gpu)      # same numbers as the multi-launch path
            assert np.array_equal(ybk, ref_gpu)     # adjoint = forward
        xin = gu.host_f64(xd)
        if dtype == "i32":
            ref = gu.oracle_packed(x.astype(np.int64), ms, offs)
            assert np.array_equal(outs[0][0].astype(np.int64), ref)
        else:
            ref = gu.oracle_packed(xin, ms, offs)
            assert gu.per_signal_rel(outs[0][0], ref, ms, offs).max() <= gu.TOL[dtype]
