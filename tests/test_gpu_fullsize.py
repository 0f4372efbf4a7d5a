"""Parity at the full workload sizes, in the launch configuration the bench
times: sampled signals against the oracle one by one, plus properties that
hold for every signal (Parseval, the DC term, involution)."""

import numpy as np
import pytest

import bench
import workloads
from oracle import metrics
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gu.torch().cuda.is_available():
        pytest.skip("no GPU")


def _invariants(x, y, m, tol):
    """x, y: (batch, 2^m) device tensors of the orthonormal transform."""
    torch = gu.torch()
    xd, yd = x.double(), y.double()
    nx = torch.linalg.vector_norm(xd, dim=1)
    ny = torch.linalg.vector_norm(yd, dim=1)
    parseval = float(torch.max(torch.abs(ny - nx) / nx))
    dc = yd[:, 0] - xd.sum(dim=1) * 2.0 ** (-m / 2)
    dc_err = float(torch.max(torch.abs(dc) / nx))
    assert parseval <= tol, parseval
    assert dc_err <= tol, dc_err
    return parseval


def test_plain_2p20_f32_bench_config():
    torch = gu.torch()
    w = workloads.CONFIGS["plain_2p20_f32"]
    m, b = 20, w.batch
    xh = workloads.float_signals(w.seed, b, m)
    x = torch.from_numpy(xh).cuda()
    plan = chw.Plan([m] * b, dtype="f32")       # the configuration the bench times
    for k, v in bench.BENCH_CONFIG["plan"].items():
        plan.set_option(k, v)
    y = plan.forward(x)
    torch.cuda.synchronize()
    idx = [0, 1, 517, b - 2, b - 1] + list(np.random.default_rng(7).integers(0, b, 3))
    ref = gu.oracle_packed(xh[idx].astype(np.float64).reshape(-1), [m] * len(idx), threads=16)
    got = y[idx].double().cpu().numpy().reshape(-1)
    rel = gu.per_signal_rel(got, ref, [m] * len(idx))
    assert rel.max() <= 1e-5
    _invariants(x, y, m, 1e-5)
    # involution: H(Hx) = x on all signals
    z = plan.forward(y)
    torch.cuda.synchronize()
    err = torch.linalg.vector_norm((z - x).double(), dim=1) / torch.linalg.vector_norm(x.double(), dim=1)
    assert float(err.max()) <= 2e-5


def test_plain_2p24_f32():
    torch = gu.torch()
    w = workloads.CONFIGS["plain_2p24_f32"]
    m, b = 24, w.batch
    xh = workloads.float_signals(w.seed, b, m)
    x = torch.from_numpy(xh).cuda()
    plan = chw.Plan([m] * b, dtype="f32")
    y = plan.forward(x)
    torch.cuda.synchronize()
    idx = [0, b - 1]
    ref = gu.oracle_packed(xh[idx].astype(np.float64).reshape(-1), [m] * 2, threads=2)
    rel = gu.per_signal_rel(y[idx].double().cpu().numpy().reshape(-1), ref, [m] * 2)
    assert rel.max() <= 1e-5
    _invariants(x, y, m, 1e-5)


@pytest.mark.skip(reason="the dependency-counter persistent kernel ran for minutes on "
                         "the GPU (killed for silence); its cause is not established, so "
                         "that kernel is switched off (exec 1 raises CHW_ERR_UNSUPPORTED)")
def test_ragged_full_dependency_queue():
    from paper_1609_06641_amd import chw as c
    ks = workloads.ragged_log2_sizes(4001)
    p = c.Plan(ks, dtype="f32", offsets=workloads.packed_offsets(ks))
    p.set_option("exec", 1)


def _ragged_inputs(dtype):
    torch = gu.torch()
    ks = workloads.ragged_log2_sizes(4001)
    offs = workloads.packed_offsets(ks)
    xr = workloads.ragged_values(4002, ks, offs)
    if dtype == "bf16":
        xt = workloads.to_half_precision(xr, "bf16").cuda()
    else:
        xt = torch.from_numpy(xr).cuda()
    return ks, offs, xt


def _ragged_check(ks, offs, xt, y, dtype, label):
    # every signal with m <= 12 against the oracle, plus 40 large ones
    rng = np.random.default_rng(5)
    small = np.nonzero(ks <= 12)[0]
    large = rng.choice(np.nonzero(ks > 12)[0], 40, replace=False)
    sel = np.concatenate([small, large])
    xin = xt.double().cpu().numpy()
    yout = y.double().cpu().numpy()
    xs = np.concatenate([xin[offs[i]:offs[i] + (1 << ks[i])] for i in sel])
    ys = np.concatenate([yout[offs[i]:offs[i] + (1 << ks[i])] for i in sel])
    ref = gu.oracle_packed(xs, ks[sel], threads=16)
    rel = gu.per_signal_rel(ys, ref, ks[sel])
    tol = 1e-5 if dtype == "f32" else 4e-3
    print("%s: max rel-L2 %.3e over %d signals" % (label, rel.max(), len(sel)))
    assert rel.max() <= tol
    # Parseval on every signal (segment sums)
    seg = np.repeat(np.arange(len(ks)), np.left_shift(1, ks.astype(np.int64)))
    nx = np.sqrt(np.bincount(seg, weights=xin ** 2))
    ny = np.sqrt(np.bincount(seg, weights=yout ** 2))
    assert np.max(np.abs(ny - nx) / nx) <= (1e-5 if dtype == "f32" else 8e-3)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("persistent", [False, True])
def test_ragged_full(dtype, persistent):
    # the planner's own choices: one launch per pass (persistent=False), or
    # the one persistent launch (exec 2) the flag selects; graph-replayed
    torch = gu.torch()
    ks, offs, xt = _ragged_inputs(dtype)
    plan = chw.Plan(ks, dtype=dtype, offsets=offs, graph=True, persistent=persistent)
    d = plan.describe()["plan"]
    assert d["config"]["exec"] == (2 if persistent else 0)
    if persistent:
        assert all(r["persistent"] for r in d["forward"])
    ws = torch.empty(max(plan.workspace_size(), 16), dtype=torch.uint8, device="cuda")
    y = plan.forward(xt, workspace=ws)
    torch.cuda.synchronize()
    _ragged_check(ks, offs, xt, y, dtype, "%s persistent=%s" % (dtype, persistent))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ragged_full_bench_config(dtype):
    # the launch configuration the benchmark times for the ragged form
    torch = gu.torch()
    ks, offs, xt = _ragged_inputs(dtype)
    plan = bench.tuned_ragged_plan(ks, offs, dtype)
    ws = torch.empty(max(plan.workspace_size(), 16), dtype=torch.uint8, device="cuda")
    y = plan.forward(xt, workspace=ws)
    torch.cuda.synchronize()
    _ragged_check(ks, offs, xt, y, dtype, "%s bench config" % dtype)


@pytest.mark.parametrize("m", [23, 25, 26, 27])
def test_largest_sizes_f32(m):
    # large single signals (2^26 and 2^27 take three passes), one signal,
    # out of place and in place, whole signal against the oracle
    torch = gu.torch()
    xh = workloads.float_signals(900 + m, 1, m)
    ref = gu.oracle_packed(xh.astype(np.float64).reshape(-1), [m], threads=1)
    p = chw.Plan([m], dtype="f32")
    x = torch.from_numpy(xh.reshape(-1)).cuda()
    y = p.forward(x)
    t = x.clone()
    p.forward(t, out=t)
    back = p.backward(y)
    torch.cuda.synchronize()
    for got in (y, t):
        assert metrics.rel_l2(got.double().cpu().numpy(), ref) <= 1e-5
    assert metrics.rel_l2(back.double().cpu().numpy(), xh.reshape(-1).astype(np.float64)) <= 2e-5


def test_largest_size_i32_wraps_exactly():
    # 2^27 int32 inputs in [1, 127]: the DC coefficient (about 2^33) wraps,
    # the others stay in range; every element equals the int64 oracle modulo
    # 2^32
    torch = gu.torch()
    m = 27
    xh = workloads.int_signals(927, 1, m, lo=1, hi=127).reshape(-1)
    ref = gu.oracle_packed(xh.astype(np.int64), [m], threads=1)
    p = chw.Plan([m], dtype="i32", norm="none")
    y = p.forward(gu.dev_tensor(xh, "i32"))
    torch.cuda.synchronize()
    wrapped = (ref & 0xFFFFFFFF).astype(np.uint32).view(np.int32)
    assert np.abs(ref).max() >= 2 ** 31
    assert np.array_equal(y.cpu().numpy(), wrapped)
