"""GPU parity of the Haar transform alone (chw_haar_forward / _backward,
eq. 2) and of the Haar-Walsh plan (eq. 4) against the oracle."""

import numpy as np
import pytest

import workloads
from oracle import cascade, dense
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _sync():
    gu.torch().cuda.synchronize()


def _oracle_haar(x, adjoint=False):
    exact = np.issubdtype(np.asarray(x).dtype, np.integer)
    v = np.array(x, dtype=np.int64 if exact else np.float64)
    c = 1 if exact else float(np.sqrt(0.5))
    (cascade.haar_adjoint if adjoint else cascade.haar_forward)(v, 0, v.shape[-1], c)
    return v


def _layout(sizes):
    offs, o = [], 0
    for k in sizes:
        o = (o + 7) // 8 * 8 + 8
        offs.append(o)
        o += 1 << k
    offs.append(o)
    return np.array(offs, dtype=np.int64)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f16", "i32", "f64"])
def test_haar_forward_backward(dtype):
    t = gu.torch()
    sizes = [0, 1, 3, 5, 12, 13, 17, 25] if dtype in ("f32", "i32") else [0, 2, 6, 12, 14, 19]
    offs = _layout(sizes)
    extent = int(offs[-1])
    norm = "none" if dtype == "i32" else "ortho"
    gen = workloads.int_signals if dtype == "i32" else workloads.float_signals
    x = np.zeros(extent, dtype=np.int64 if dtype == "i32" else np.float32)
    for i, k in enumerate(sizes):
        x[offs[i]:offs[i] + (1 << k)] = gen(900 + i, 1, k)[0]
    xd = gu.dev_tensor(x, dtype)
    xh = gu.host_f64(xd)
    p = chw.Plan(sizes, dtype=dtype, norm=norm, offsets=offs)
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    y = gu.host_f64(p.haar_forward(xd, workspace=ws))
    g = gu.host_f64(p.haar_backward(xd, workspace=ws))
    _sync()
    for i, k in enumerate(sizes):
        n, o = 1 << k, offs[i]
        seg = xh[o:o + n].astype(np.int64) if dtype == "i32" else xh[o:o + n]
        ref, ref_a = _oracle_haar(seg), _oracle_haar(seg, adjoint=True)
        if dtype == "i32":
            wrap = lambda a: (a & 0xffffffff).astype(np.uint32).view(np.int32)  # noqa: E731
            assert np.array_equal(y[o:o + n].astype(np.int32), wrap(ref)), k
            assert np.array_equal(g[o:o + n].astype(np.int32), wrap(ref_a)), k
        else:
            assert gu.metrics.rel_l2(y[o:o + n], ref) <= gu.TOL[dtype], k
            assert gu.metrics.rel_l2(g[o:o + n], ref_a) <= gu.TOL[dtype], k


def test_haar_round_trip_and_small_dense():
    t = gu.torch()
    m = 6
    psi = dense.haar_matrix(m)
    x = workloads.float_signals(910, 16, m).astype(np.float64)
    p = chw.Plan([m] * 16, dtype="f64")
    y = gu.host_f64(p.haar_forward(gu.dev_tensor(x, "f64")))
    assert np.max(np.abs(y.reshape(16, -1) - x @ psi.T)) < 1e-13
    sizes = [20, 9, 14]
    x = np.concatenate([workloads.float_signals(911 + i, 1, k)[0] for i, k in enumerate(sizes)])
    q = chw.Plan(sizes, dtype="f32")
    ws = t.empty(max(q.workspace_size(), 16), dtype=t.uint8, device="cuda")
    xd = gu.dev_tensor(x, "f32")
    back = q.haar_backward(q.haar_forward(xd, workspace=ws), workspace=ws)
    _sync()
    assert gu.metrics.rel_l2(gu.host_f64(back), x.astype(np.float64)) <= 1e-6


@pytest.mark.parametrize("m", [0, 1, 5, 10])
def test_haar_walsh_plan_matches_eq4(m):
    batch = 3
    w = workloads.float_signals(920 + m, batch, m).astype(np.float64)
    p = chw.Plan.haar_walsh(batch, m, dtype="f64")
    y = gu.host_f64(p.forward(gu.dev_tensor(w.reshape(-1), "f64"))).reshape(batch, -1)
    yt = gu.host_f64(p.backward(gu.dev_tensor(w.reshape(-1), "f64"))).reshape(batch, -1)
    hw = dense.haar_walsh(m)
    assert np.max(np.abs(y - w @ hw.T)) < 1e-12
    assert np.max(np.abs(yt - w @ hw)) < 1e-12


def test_haar_walsh_after_haar_is_the_transform():
    # eq. (4) with Theorem 1: H_m x = diag(1, H_0, ..., H_{m-1}) Psi_m x
    t = gu.torch()
    m, batch = 20, 4
    x = workloads.float_signals(930, batch, m)
    xd = gu.dev_tensor(x.reshape(-1), "f32")
    p = chw.Plan([m] * batch, dtype="f32")
    hw = chw.Plan.haar_walsh(batch, m, dtype="f32")
    ws = t.empty(max(p.workspace_size(), hw.workspace_size(), 16), dtype=t.uint8, device="cuda")
    via = hw.forward(p.haar_forward(xd, workspace=ws), workspace=ws)
    direct = p.forward(xd, workspace=ws)
    _sync()
    a, b = gu.host_f64(via).reshape(batch, -1), gu.host_f64(direct).reshape(batch, -1)
    assert max(gu.metrics.rel_l2(a[i], b[i]) for i in range(batch)) <= 1e-5
