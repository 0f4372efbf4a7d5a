"""Three HBM passes (signals above 2^27, or of 2^20 and more with the
THREE_PASS flag): the same stages in the same order as the two-pass split, so
bit for bit the two-pass result at the sizes both take, and the oracle's:
element by element where the oracle runs in seconds, through sampled outputs
of eq. (1) and invariants at the largest sizes."""

import numpy as np
import pytest

import workloads
from oracle import cascade
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _sync():
    gu.torch().cuda.synchronize()


def _bits(t):
    tt = gu.torch()
    return t.view(tt.int16 if t.element_size() == 2 else tt.int32 if t.element_size() == 4
                  else tt.int64)


def _inputs(sizes, dtype, seed):
    parts = []
    for i, k in enumerate(sizes):
        if dtype == "i32":
            parts.append(workloads.int_signals(seed + i, 1, k).reshape(-1))
        else:
            parts.append(workloads.float_signals(seed + i, 1, k).reshape(-1))
    return np.concatenate(parts)


CASES = [("f32", [20, 12, 21, 3]), ("bf16", [21, 20, 9]), ("f16", [20, 16]),
         ("i32", [22, 20, 11])]


@pytest.mark.parametrize("dtype,sizes", CASES, ids=[c[0] for c in CASES])
def test_three_pass_equals_two_pass_and_oracle(dtype, sizes):
    t = gu.torch()
    norm = "none" if dtype == "i32" else "ortho"
    x = _inputs(sizes, dtype, 8100)
    xd = gu.dev_tensor(x, dtype)
    p3 = chw.Plan(sizes, dtype=dtype, norm=norm, three_pass=True)
    p2 = chw.Plan(sizes, dtype=dtype, norm=norm)
    assert p3.describe()["plan"]["three"] == sum(1 for m in sizes if m >= 20)
    print("three-pass", dtype, sizes, flush=True)
    y3 = p3.forward(xd)
    y2 = p2.forward(xd)
    _sync()
    assert t.equal(_bits(y3), _bits(y2)), "three passes differ from two"
    # the synthesis kernels of the adjoint (option set before a plan's first
    # use), both splits, and the default backward (the forward launches)
    a3 = chw.Plan(sizes, dtype=dtype, norm=norm, three_pass=True)
    a2 = chw.Plan(sizes, dtype=dtype, norm=norm)
    for q in (a3, a2):
        q.set_option("adjoint", 1)
    g3 = a3.backward(xd)
    g2 = a2.backward(xd)
    d3 = p3.backward(xd)
    _sync()
    assert t.equal(_bits(g3), _bits(g2)) and t.equal(_bits(d3), _bits(y2))
    # against the oracle on the values the GPU read
    xin = gu.host_f64(xd) if dtype != "i32" else gu.host_i64(xd)
    ref = gu.oracle_packed(xin, sizes)
    if dtype == "i32":
        assert np.array_equal(gu.host_i64(y3).astype(np.int32), ref.astype(np.int32))
    else:
        assert gu.per_signal_rel(gu.host_f64(y3), ref, sizes).max() <= gu.TOL[dtype]


def test_three_pass_in_place_signed_and_noalloc():
    t = gu.torch()
    sizes = [21, 20, 14]
    x = _inputs(sizes, "f32", 8200)
    xd = gu.dev_tensor(x, "f32")
    p3 = chw.Plan(sizes, dtype="f32", three_pass=True)
    p2 = chw.Plan(sizes, dtype="f32")
    ref = p2.forward(xd)
    y = xd.clone()
    p3.forward(y, out=y)                    # in place
    z = t.empty_like(xd)
    p3.forward_noalloc(xd, z)               # intermediates in the static scratch
    # two signed rounds with per-element diagonals drawn on the device
    s = p2.philox_signs(77, 2, "per_element")
    ys3 = p3.forward_signed(xd, s, "per_element", 2)
    ys2 = p2.forward_signed(xd, s, "per_element", 2)
    gs3 = p3.backward_signed(xd, s, "per_element", 2)
    gs2 = p2.backward_signed(xd, s, "per_element", 2)
    _sync()
    assert t.equal(y, ref) and t.equal(z, ref)
    assert t.equal(ys3, ys2) and t.equal(gs3, gs2)


def _check_large(m, dtype, samples, involution):
    """One signal of 2^m: sampled outputs of eq. (1) (O(n) each), Parseval and
    the DC term; optionally H(Hx) = x."""
    x = workloads.float_signals(8300 + m, 1, m).reshape(-1)
    xd = gu.dev_tensor(x, dtype)
    xin = gu.host_f64(xd)  # the values the GPU read (rounded for bf16)
    p = chw.Plan([m], dtype=dtype)
    d = p.describe()["plan"]
    assert d["three"] == 1, d
    print("three-pass", dtype, "m", m, flush=True)
    y = p.forward(xd)
    _sync()
    yh = gu.host_f64(y)
    tol = gu.TOL[dtype]
    nx = float(np.sqrt(np.sum(xin * xin)))
    # Parseval (H is orthonormal) and the DC term y_0 = 2^{-m/2} sum x
    assert abs(float(np.sqrt(np.sum(yh * yh))) - nx) <= 4 * tol * nx
    rng = np.random.default_rng(m)
    idx = [0, 1, (1 << m) - 1] + [int(v) for v in rng.integers(0, 1 << m, samples)]
    rms = nx * 2.0 ** (-m / 2.0)  # root mean square of the outputs (Parseval)
    for i in idx:
        c = cascade.coefficient(xin, i)
        # the relative-L2 tolerance spread over the outputs, with room for
        # an output above the mean; narrow storage adds its own rounding
        bound = 8 * tol * rms + (2.0 ** -8 * abs(c) if dtype != "f32" else 0.0)
        assert abs(yh[i] - c) <= bound, (i, yh[i], c)
    if involution:
        z = p.forward(y)
        _sync()
        zh = gu.host_f64(z)
        assert float(np.sqrt(np.sum((zh - xin) ** 2))) <= 2 * tol * nx
    del x, xd, y


def test_three_pass_2p28_f32():
    _check_large(28, "f32", 4, involution=True)


def test_three_pass_2p28_bf16():
    _check_large(28, "bf16", 2, involution=False)


def test_three_pass_2p30_f32():
    # the largest supported size: 4 GiB per buffer, 8 GiB of workspace
    _check_large(30, "f32", 1, involution=False)
