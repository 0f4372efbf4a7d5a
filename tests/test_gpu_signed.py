"""GPU parity of the fused random-sign diagonals (chw_forward_signed /
chw_backward_signed): y = H D_k ... H D_1 x and its adjoint, against the
oracle (oracle.signed) and, bit for bit, against the unfused GPU path (the
sign flips done by torch, then the plain transform per round)."""

import numpy as np
import pytest

import workloads
from oracle import signed
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _signs_dev(words):
    """uint32 numpy words -> int32 device tensor (same bits)."""
    t = gu.torch()
    return t.from_numpy(np.ascontiguousarray(words).reshape(-1).view(np.int32).copy()).to("cuda")


def _sync():
    gu.torch().cuda.synchronize()


def test_diff_workload_fused_sign():
    # y = H D x, 256 x 2^14 FP32 with one shared diagonal; gradient D H^T g
    m, batch = 14, 256
    x = workloads.float_signals(5001, batch, m)
    d = workloads.sign_diagonal(5002, 1 << m)
    g = workloads.float_signals(5003, batch, m)
    t = gu.torch()
    p = chw.Plan([m] * batch, dtype="f32")
    s = _signs_dev(workloads.pack_sign_bits(d))
    xd, gd = gu.dev_tensor(x, "f32"), gu.dev_tensor(g, "f32")
    dd = t.from_numpy(d).to("cuda")
    y = p.forward_signed(xd, s, "shared", 1)
    y_unfused = p.forward(xd * dd)
    gx = p.backward_signed(gd, s, "shared", 1)
    gx_unfused = p.backward(gd) * dd
    _sync()
    assert t.equal(y, y_unfused) and t.equal(gx, gx_unfused)
    d8 = d.astype(np.int8)
    idx = [0, 97, 255]
    ref = signed.signed_forward(x[idx].astype(np.float64), [d8])
    assert np.max([gu.metrics.rel_l2(a, b) for a, b in zip(gu.host_f64(y)[idx], ref)]) <= 1e-5
    ref_g = signed.signed_adjoint(g[idx].astype(np.float64), [d8])
    assert np.max([gu.metrics.rel_l2(a, b) for a, b in zip(gu.host_f64(gx)[idx], ref_g)]) <= 1e-5


def _layout(dtype):
    # tiny, single-pass 2^12 / 2^15 tiles and two-pass signals, with gaps
    sizes = [2, 9, 13, 12, 17, 1, 10] if dtype != "f64" else [0, 9, 13, 12, 17, 10]
    offs, o = [], 0
    for k in sizes:
        o = (o + 7) // 8 * 8 + 8     # aligned gap before every signal
        offs.append(o)
        o += 1 << k
    offs.append(o + 8)
    return sizes, np.array(offs, dtype=np.int64)


def _inputs(dtype, sizes, offs, seed):
    extent = int(offs[-1])
    x = np.zeros(extent, dtype=np.int64 if dtype == "i32" else np.float32)
    for i, k in enumerate(sizes):
        gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
        x[offs[i]:offs[i] + (1 << k)] = gen(seed + i, 1, k)[0]
    return x


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i32", "f64"])
@pytest.mark.parametrize("mode", ["shared", "per_element"])
@pytest.mark.parametrize("rounds", [1, 3])
def test_signed_rounds(dtype, mode, rounds):
    t = gu.torch()
    sizes, offs = _layout(dtype)
    extent = int(offs[-1])
    norm = "none" if dtype == "i32" else "ortho"
    p = chw.Plan(sizes, dtype=dtype, norm=norm, offsets=offs)
    x = _inputs(dtype, sizes, offs, 700)
    xd = gu.dev_tensor(x, dtype)
    xin = gu.host_f64(xd)                         # the values the GPU reads
    nbits = (1 << max(sizes)) if mode == "shared" else extent
    diags = workloads.sign_rounds(710 + rounds, rounds, nbits)
    s = _signs_dev(workloads.pack_sign_bits(diags))
    flat = diags if mode == "per_element" else workloads.expand_shared_signs(diags, sizes, offs)
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    y = p.forward_signed(xd, s, mode, rounds, workspace=ws)
    gy = p.backward_signed(xd, s, mode, rounds, workspace=ws)
    # unfused GPU path: torch flips the signs (exact), the plain transform per round
    dev_d = [gu.dev_tensor(f.astype(np.float64 if dtype == "f64" else np.float32), dtype)
             for f in flat]
    v = xd.clone()
    for r in range(rounds):
        v = p.forward(v * dev_d[r], workspace=ws)
    w = xd.clone()
    for r in reversed(range(rounds)):
        w = p.backward(w, workspace=ws) * dev_d[r]
    _sync()
    mask = np.zeros(extent, dtype=bool)
    same = np.zeros(extent, dtype=bool)   # elements the unfused path must match bit for bit
    for i, k in enumerate(sizes):
        mask[offs[i]:offs[i] + (1 << k)] = True
        # a signal that runs in one tile (or the tiny kernel) keeps the compute
        # type between its rounds; the unfused path stores every round in the
        # plan's dtype, which differs for the narrow types
        if rounds == 1 or dtype != "bf16" or k > 15:
            same[offs[i]:offs[i] + (1 << k)] = True
    yh, vh, gyh, wh = (gu.host_f64(a)[same] for a in (y, v, gy, w))
    assert np.array_equal(yh, vh) and np.array_equal(gyh, wh)
    # oracle (float64 / int64), rounds in order, on the values the GPU read
    if dtype == "i32":
        ref = signed.signed_batch(xin.astype(np.int64), sizes, list(flat), offsets=offs[:-1])
        ref_a = signed.signed_batch(xin.astype(np.int64), sizes, list(flat), offsets=offs[:-1],
                                    adjoint=True)
        wrap = lambda a: (a.astype(np.int64) & 0xffffffff).astype(np.uint32).view(np.int32)  # noqa: E731
        assert np.array_equal(wrap(ref[mask]), gu.host_i64(y)[mask].astype(np.int32))
        assert np.array_equal(wrap(ref_a[mask]), gu.host_i64(gy)[mask].astype(np.int32))
        return
    ref = signed.signed_batch(xin, sizes, list(flat), offsets=offs[:-1])
    ref_a = signed.signed_batch(xin, sizes, list(flat), offsets=offs[:-1], adjoint=True)
    # each round stores its output in the plan's dtype: one rounding per round
    tol = gu.TOL[dtype] * rounds
    y_full, g_full = gu.host_f64(y), gu.host_f64(gy)
    assert gu.per_signal_rel(y_full, ref, sizes, offs).max() <= tol
    assert gu.per_signal_rel(g_full, ref_a, sizes, offs).max() <= tol


def test_signed_all_clear_equals_plain():
    t = gu.torch()
    sizes = [12] * 4 + [16] * 2
    x = np.concatenate([workloads.float_signals(720 + i, 1, k)[0] for i, k in enumerate(sizes)])
    p = chw.Plan(sizes, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    s = t.zeros(p.sign_words("per_element"), dtype=t.int32, device="cuda")
    a = p.forward_signed(xd, s, "per_element", 1)
    b = p.forward(xd)
    _sync()
    assert t.equal(a, b)


def test_signed_graph_replay():
    t = gu.torch()
    sizes = [16] * 2 + [11] * 8
    x = np.concatenate([workloads.float_signals(730 + i, 1, k)[0] for i, k in enumerate(sizes)])
    pg = chw.Plan(sizes, dtype="f32", graph=True)
    pe = chw.Plan(sizes, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    ws = t.empty(max(pg.workspace_size(), 16), dtype=t.uint8, device="cuda")
    sA = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(731, 2, 1 << 16)))
    sB = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(732, 2, 1 << 16)))
    wantA = pe.forward_signed(xd, sA, "shared", 2, workspace=ws)
    wantB = pe.forward_signed(xd, sB, "shared", 2, workspace=ws)
    backA = pe.backward_signed(xd, sA, "shared", 2, workspace=ws)
    _sync()
    # the two-pass signals join their round boundaries (forward and adjoint)
    assert pg.describe()["plan"]["turn"]
    yA, yB, gA = t.empty_like(xd), t.empty_like(xd), t.empty_like(xd)
    for _ in range(3):
        pg.forward_signed(xd, sA, "shared", 2, out=yA, workspace=ws)
        pg.forward_signed(xd, sB, "shared", 2, out=yB, workspace=ws)
        pg.backward_signed(xd, sA, "shared", 2, out=gA, workspace=ws)
        _sync()
        assert t.equal(yA, wantA) and t.equal(yB, wantB) and t.equal(gA, backA)
    assert not t.equal(wantA, wantB)


def test_signed_autograd():
    t = gu.torch()
    m, batch, rounds = 6, 4, 2
    p = chw.Plan([m] * batch, dtype="f64")
    s = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(740, rounds, 1 << m)))
    x = t.from_numpy(workloads.float_signals(741, batch, m).astype(np.float64)).to("cuda")
    x.requires_grad_(True)
    f = lambda v: chw.signed_transform(v, p, s, "shared", rounds)  # noqa: E731
    assert t.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-9)


@pytest.mark.parametrize("mode", ["shared", "per_element"])
def test_signed_prefetching_tiles(mode):
    # full 2^15-element tiles run the prefetching kernel, which fetches the
    # sign bits with the data: same bits with and without it
    t = gu.torch()
    for sizes in ([13] * 8, [15] * 2, [22] * 2):
        x = np.concatenate([workloads.float_signals(750 + i, 1, k)[0] for i, k in enumerate(sizes)])
        xd = gu.dev_tensor(x, "f32")
        res = []
        for stream in (0, 2):
            p = chw.Plan(sizes, dtype="f32")
            p.set_option("spread", 0)  # full tiles of several 2^13 signals
            p.set_option("stream", stream)
            nbits = (1 << max(sizes)) if mode == "shared" else p.extent
            s = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(751, 2, nbits)))
            ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
            res.append((p.forward_signed(xd, s, mode, 2, workspace=ws),
                        p.backward_signed(xd, s, mode, 2, workspace=ws)))
        _sync()
        assert t.equal(res[0][0], res[1][0]) and t.equal(res[0][1], res[1][1]), sizes


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_signed_persistent_and_split_forms(dtype):
    # the persistent launch runs every round of a whole signal in one
    # workgroup; the numbers equal those of one launch per pass and round
    t = gu.torch()
    sizes = [16, 9, 9, 14, 18, 1] if dtype == "f32" else [16, 9, 9, 14, 18, 0]
    x = np.concatenate([workloads.float_signals(760 + i, 1, k)[0] for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, dtype)
    outs = []
    for opts in (dict(), dict(exec=2), dict(single15=0), dict(split_l1=12 if dtype == "f32" else 9)):
        p = chw.Plan(sizes, dtype=dtype)
        for kk, vv in opts.items():
            p.set_option(kk, vv)
        s = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(761, 3, p.extent)))
        ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
        outs.append((gu.host_f64(p.forward_signed(xd, s, "per_element", 3, workspace=ws)),
                     gu.host_f64(p.backward_signed(xd, s, "per_element", 3, workspace=ws))))
    _sync()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


@pytest.mark.parametrize("dtype", ["f32", "i32"])
@pytest.mark.parametrize("mode", ["shared", "per_element"])
@pytest.mark.parametrize("sizes,split", [([16, 21, 12, 24, 3, 25, 20], -1), ([20, 12, 3, 21], 12)],
                         ids=["rows7-5", "rows3"])
def test_round_boundary_tiles_bitwise(dtype, mode, sizes, split):
    # signed multi-round calls join round r's last pass and round r + 1's
    # first pass (KIND_TURN tiles): the same bits as one launch pair per round,
    # with and without prefetching, in place and out of place; every compiled
    # first-pass row count (m = 16, 20, 21: 2^7 rows; 24: 2^6; 25: 2^5; a
    # forced first pass of 12 levels: 2^3).  The adjoint runs the forward
    # launches (diagonals shifted by a round, the last one at the last pass's
    # store) or, with option adjoint, the synthesis boundary tiles; the
    # reference plan's adjoint runs the synthesis kernels one round at a time.
    t = gu.torch()
    norm = "none" if dtype == "i32" else "ortho"
    gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
    x = np.concatenate([gen(760 + i, 1, k)[0] for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, dtype)
    plans = {}
    for turn, stream, adjoint in ((0, 1, 0), (1, 1, 0), (1, 0, 0), (1, 1, 1)):
        p = chw.Plan(sizes, dtype=dtype, norm=norm)
        p.set_option("turn", turn)
        p.set_option("stream", stream)
        p.set_option("adjoint", adjoint)
        if split > 0:
            p.set_option("split_l1", split)
        plans[(turn, stream, adjoint)] = p
    ref_plan = plans[(0, 1, 0)]
    assert ref_plan.describe()["plan"]["turn"] == []
    assert plans[(1, 1, 0)].describe()["plan"]["turn"]
    nbits = (1 << max(sizes)) if mode == "shared" else ref_plan.extent
    ws = t.empty(max(ref_plan.workspace_size(), 16), dtype=t.uint8, device="cuda")
    for rounds in (1, 2, 3, 4):
        s = _signs_dev(workloads.pack_sign_bits(workloads.sign_rounds(770 + rounds, rounds, nbits)))
        want = ref_plan.forward_signed(xd, s, mode, rounds, workspace=ws)
        want_b = ref_plan.backward_signed(xd, s, mode, rounds, workspace=ws)
        for key in ((1, 1, 0), (1, 0, 0), (1, 1, 1)):
            got = plans[key].forward_signed(xd, s, mode, rounds, workspace=ws)
            got_b = plans[key].backward_signed(xd, s, mode, rounds, workspace=ws)
            inplace = xd.clone()
            plans[key].forward_signed(inplace, s, mode, rounds, out=inplace, workspace=ws)
            inplace_b = xd.clone()
            plans[key].backward_signed(inplace_b, s, mode, rounds, out=inplace_b, workspace=ws)
            _sync()
            assert t.equal(got, want), (rounds, key)
            assert t.equal(inplace, want), (rounds, key, "in place")
            assert t.equal(got_b, want_b), (rounds, key, "adjoint")
            assert t.equal(inplace_b, want_b), (rounds, key, "adjoint in place")


def test_round_boundary_tiles_against_oracle():
    t = gu.torch()
    sizes = [16, 20, 12]
    rounds = 3
    x = np.concatenate([workloads.float_signals(780 + i, 1, k)[0] for i, k in enumerate(sizes)])
    p = chw.Plan(sizes, dtype="f32")
    assert p.describe()["plan"]["turn"]
    xd = gu.dev_tensor(x, "f32")
    s = p.philox_signs(781, rounds, "per_element")
    ws = t.empty(p.workspace_size(), dtype=t.uint8, device="cuda")
    y = p.forward_signed(xd, s, "per_element", rounds, workspace=ws)
    g = p.backward_signed(xd, s, "per_element", rounds, workspace=ws)
    _sync()
    from oracle import philox
    diags = philox.diagonals(philox.sign_words(781, rounds, p.sign_words("per_element")), p.extent)
    ref = signed.signed_batch(x.astype(np.float64), sizes, list(diags))
    assert gu.per_signal_rel(gu.host_f64(y), ref, sizes).max() <= gu.TOL["f32"] * rounds
    ref_g = signed.signed_batch(x.astype(np.float64), sizes, list(diags), adjoint=True)
    assert gu.per_signal_rel(gu.host_f64(g), ref_g, sizes).max() <= gu.TOL["f32"] * rounds
