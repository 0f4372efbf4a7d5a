"""GPU parity of the sequency and natural coefficient orders: bit for bit the
dyadic result permuted (forward) / the dyadic adjoint of the un-permuted input
(backward), and the oracle's ordered transform."""

import numpy as np
import pytest

import workloads
from oracle import orders
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _sync():
    gu.torch().cuda.synchronize()


def _perm(order, m):
    """Dyadic index of every output position of a signal of 2^m."""
    n = 1 << m
    k = np.arange(n, dtype=np.int64)
    if order == "natural":
        r = np.zeros(n, dtype=np.int64)
        for b in range(m):
            r |= ((k >> b) & 1) << (m - 1 - b)
        return r
    return k ^ (k >> 1)


def _layout(dtype):
    sizes = [1, 7, 12, 13, 15, 17, 20, 22] if dtype != "f64" else [0, 7, 12, 13, 17, 20]
    if dtype == "bf16":
        sizes[0] = 2
    offs, o = [], 0
    for k in sizes:
        o = (o + 7) // 8 * 8 + 8
        offs.append(o)
        o += 1 << k
    offs.append(o)
    return sizes, np.array(offs, dtype=np.int64)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i32", "f64"])
@pytest.mark.parametrize("order", ["sequency", "natural"])
def test_order_is_a_permutation_of_dyadic(dtype, order):
    t = gu.torch()
    sizes, offs = _layout(dtype)
    norm = "none" if dtype == "i32" else "ortho"
    extent = int(offs[-1])
    gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
    x = np.zeros(extent, dtype=np.int64 if dtype == "i32" else np.float32)
    for i, k in enumerate(sizes):
        x[offs[i]:offs[i] + (1 << k)] = gen(800 + i, 1, k)[0]
    xd = gu.dev_tensor(x, dtype)
    pd = chw.Plan(sizes, dtype=dtype, norm=norm, offsets=offs)
    po = chw.Plan(sizes, dtype=dtype, norm=norm, offsets=offs, order=order)
    ws = t.empty(max(po.workspace_size(), pd.workspace_size(), 16), dtype=t.uint8, device="cuda")
    yd = gu.host_f64(pd.forward(xd, workspace=ws))
    yo = gu.host_f64(po.forward(xd, workspace=ws))
    go = gu.host_f64(po.backward(xd, workspace=ws))
    # the adjoint: the dyadic adjoint of the input un-permuted to dyadic order
    g_dy = np.zeros(extent)
    xh = gu.host_f64(xd)
    for i, k in enumerate(sizes):
        n, o = 1 << k, offs[i]
        g_dy[o + _perm(order, k)] = xh[o:o + n]
    gd = gu.host_f64(pd.backward(gu.dev_tensor(g_dy, dtype), workspace=ws))
    _sync()
    for i, k in enumerate(sizes):
        n, o = 1 << k, offs[i]
        assert np.array_equal(yo[o:o + n], yd[o:o + n][_perm(order, k)]), (order, k)
        assert np.array_equal(go[o:o + n], gd[o:o + n]), (order, k, "adjoint")
    # oracle: the dyadic cascade reordered by the definitions' closed forms
    for i, k in enumerate(sizes[:6]):
        n, o = 1 << k, offs[i]
        ref = gu.oracle_packed(xh[o:o + n].astype(np.int64 if dtype == "i32" else np.float64), [k])
        ref = orders.natural_from_dyadic(ref) if order == "natural" else orders.sequency_from_dyadic(ref)
        if dtype == "i32":
            assert np.array_equal(yo[o:o + n].astype(np.int64), ref)
        else:
            assert gu.metrics.rel_l2(yo[o:o + n], ref) <= gu.TOL[dtype]


@pytest.mark.parametrize("order", ["sequency", "natural"])
def test_order_signed_rounds(order):
    # two signed rounds: the second diagonal applies to the first round's
    # output in the plan's order; equal to the unfused path
    t = gu.torch()
    sizes = [9, 12, 14, 18]
    x = np.concatenate([workloads.float_signals(820 + i, 1, k)[0] for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, "f32")
    p = chw.Plan(sizes, dtype="f32", order=order)
    diags = workloads.sign_rounds(821, 2, p.extent)
    s = t.from_numpy(workloads.pack_sign_bits(diags).reshape(-1).view(np.int32).copy()).cuda()
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    y = p.forward_signed(xd, s, "per_element", 2, workspace=ws)
    g = p.backward_signed(xd, s, "per_element", 2, workspace=ws)
    d = [t.from_numpy(diags[r].astype(np.float32)).cuda() for r in range(2)]
    v = p.forward(p.forward(xd * d[0], workspace=ws) * d[1], workspace=ws)
    w = p.backward(p.backward(xd, workspace=ws) * d[1], workspace=ws) * d[0]
    _sync()
    assert t.equal(y, v) and t.equal(g, w)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "i32"])
@pytest.mark.parametrize("order", ["sequency", "natural"])
def test_order_prefetching_bitwise(dtype, order):
    # the forward prefetching kernels of the other orders (full 2^15-element
    # tiles: single-pass 2^13 and 2^15 signals, first and last passes of
    # 2^17, 2^22 and 2^24 signals) against one workgroup per tile, bit for bit
    t = gu.torch()
    norm = "none" if dtype == "i32" else "ortho"
    gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
    for sizes in ([13] * 8, [15] * 2, [17] * 3, [22] * 2, [24]):
        x = np.concatenate([gen(830 + i, 1, k).reshape(-1) for i, k in enumerate(sizes)])
        xd = gu.dev_tensor(x, dtype)
        outs = []
        for stream in (0, 2):
            p = chw.Plan(sizes, dtype=dtype, norm=norm, order=order)
            p.set_option("spread", 0)
            p.set_option("stream", stream)
            d = p.describe()["plan"]
            assert any(r["stream"] > 0 for r in d["forward"]) == bool(stream), sizes
            assert all(r["stream"] == 0 for r in d["backward"])
            ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
            outs.append(p.forward(xd, workspace=ws))
        _sync()
        assert t.equal(outs[0], outs[1]), (order, sizes)


@pytest.mark.parametrize("order", ["sequency", "natural"])
def test_order_out_of_place_without_workspace(order):
    # an out-of-place forward call of these orders always takes a workspace
    # (their last-pass tiles store into blocks that other tiles have yet to
    # load, so y cannot hold the intermediate); the binding supplies one.
    # Large two-pass signals, one workgroup per tile and prefetching: the
    # dyadic result permuted, bit for bit.
    t = gu.torch()
    sizes = [24, 25]
    x = np.concatenate([workloads.float_signals(840 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    xd = gu.dev_tensor(x, "f32")
    yd = gu.host_f64(chw.Plan(sizes, dtype="f32").forward(xd))
    for stream in (0, 1):
        p = chw.Plan(sizes, dtype="f32", order=order)
        p.set_option("stream", stream)
        yo = gu.host_f64(p.forward(xd))
        _sync()
        o = 0
        for k in sizes:
            n = 1 << k
            assert np.array_equal(yo[o:o + n], yd[o:o + n][_perm(order, k)]), (order, k, stream)
            o += n
