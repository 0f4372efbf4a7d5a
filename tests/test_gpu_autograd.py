"""Differentiation through CHWFunction: y = H (d * x) with a random +-1 diagonal
d; the backward runs the hand-written adjoint (chw_backward)."""

import numpy as np
import pytest

import workloads
from oracle import cascade, dense
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gu.torch().cuda.is_available():
        pytest.skip("no GPU")


def test_gradcheck_f64():
    torch = gu.torch()
    w = workloads.CONFIGS["gradcheck_f64"]
    m, b = 6, w.batch
    plan = chw.Plan([m] * b, dtype="f64")
    d = torch.from_numpy(workloads.sign_diagonal(5002, 1 << m).astype(np.float64)).cuda()
    x = torch.from_numpy(np.random.default_rng(w.seed).standard_normal((b, 1 << m))).cuda()
    x.requires_grad_(True)

    def f(inp):
        return chw.transform((inp * d).reshape(-1).contiguous(), plan).reshape(b, -1)

    assert torch.autograd.gradcheck(f, (x,), eps=1e-6, atol=1e-9, rtol=1e-7)


def test_diff_workload_f32():
    # 256 x 2^14 float32: gradient vs the oracle adjoint and vs the dense
    # reference gradient (H D)^T g on a subset
    torch = gu.torch()
    w = workloads.CONFIGS["diff_f32"]
    m, b = 14, w.batch
    n = 1 << m
    plan = chw.Plan([m] * b, dtype="f32")
    d_np = workloads.sign_diagonal(5002, n)
    x_np = workloads.float_signals(5001, b, m)
    g_np = workloads.float_signals(5003, b, m)
    d = torch.from_numpy(d_np).cuda()
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    g = torch.from_numpy(g_np).cuda()
    y = chw.transform((x * d).reshape(-1).contiguous(), plan).reshape(b, n)
    (y * g).sum().backward()
    torch.cuda.synchronize()
    yh = y.detach().double().cpu().numpy()
    gx = x.grad.double().cpu().numpy()
    # forward vs oracle
    ref_y = gu.oracle_packed((x_np.astype(np.float64) * d_np).reshape(-1), [m] * b).reshape(b, n)
    assert np.max(np.linalg.norm(yh - ref_y, axis=1) / np.linalg.norm(ref_y, axis=1)) <= 1e-5
    # gradient: d * H^T g (oracle adjoint)
    ref_g = d_np * gu.oracle_packed(g_np.astype(np.float64).reshape(-1), [m] * b,
                                    adjoint=True).reshape(b, n)
    rel = np.linalg.norm(gx - ref_g, axis=1) / np.linalg.norm(ref_g, axis=1)
    assert rel.max() <= 1e-5, rel.max()


@pytest.mark.parametrize("m", [4, 9, 12])
def test_dense_reference_gradient(m):
    torch = gu.torch()
    n = 1 << m
    b = 3
    plan = chw.Plan([m] * b, dtype="f32")
    d_np = workloads.sign_diagonal(77 + m, n)
    x = torch.from_numpy(workloads.float_signals(88 + m, b, m)).cuda().requires_grad_(True)
    g_np = workloads.float_signals(99 + m, b, m)
    y = chw.transform((x * torch.from_numpy(d_np).cuda()).reshape(-1).contiguous(), plan)
    (y.reshape(b, n) * torch.from_numpy(g_np).cuda()).sum().backward()
    torch.cuda.synchronize()
    hd = dense.hadamard_paley(m) * d_np[None, :]        # H D (dense, float64)
    ref = g_np.astype(np.float64) @ hd                   # rows of (H D)^T g
    got = x.grad.double().cpu().numpy()
    rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert rel.max() <= 1e-5


def test_finite_difference_f64():
    torch = gu.torch()
    m, b = 10, 2
    n = 1 << m
    plan = chw.Plan([m] * b, dtype="f64")
    rng = np.random.default_rng(31)
    d = torch.from_numpy(workloads.sign_diagonal(41, n).astype(np.float64)).cuda()
    x = torch.from_numpy(rng.standard_normal((b, n))).cuda().requires_grad_(True)
    g = torch.from_numpy(rng.standard_normal((b, n))).cuda()
    v = torch.from_numpy(rng.standard_normal((b, n))).cuda()

    def loss(inp):
        return (chw.transform((inp * d).reshape(-1).contiguous(), plan).reshape(b, n) * g).sum()

    loss(x).backward()
    eps = 1e-5
    with torch.no_grad():
        fd = (loss(x + eps * v) - loss(x - eps * v)) / (2 * eps)
    an = (x.grad * v).sum()
    torch.cuda.synchronize()
    assert abs(float(fd) - float(an)) <= 1e-8 * max(1.0, abs(float(an)))
