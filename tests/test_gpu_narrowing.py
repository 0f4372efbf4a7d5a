"""The BF16 / FP16 forms narrow by round to nearest even, pinned bit for bit.

The narrow-storage forms widen the stored input exactly, run every pass in
FP32 (the intermediate between HBM passes is FP32 too) and round only at the
final store.  The FP32 plan runs the same butterflies on the same operands in
the same order (eqs. (1)-(3): the stages do not depend on the dtype), so on
the widened input it produces exactly the values the narrow form rounds.
Hence: narrow result == RNE(FP32 result on the widened input), element by
element.  A relative-L2 bound cannot tell RNE from truncation (one ulp either
way), this comparison can; the host test tests/test_narrowing_host.py plants
truncation and shows that this check rejects it.
"""

import numpy as np
import pytest

import bench
import workloads
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gu.torch().cuda.is_available():
        pytest.skip("no GPU")
    chw.load()


def _pair(sizes, dtype, offsets=None, options=None):
    p_h = chw.Plan(sizes, dtype=dtype, offsets=offsets)
    p_f = chw.Plan(sizes, dtype="f32", offsets=offsets)
    for k, v in (options or {}).items():
        p_h.set_option(k, v)
        p_f.set_option(k, v)
    return p_h, p_f


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_precision_workload_full_size_rne(dtype):
    # 8192 x 2^12, N(0,1) with 1% outliers x100, rounded to the dtype (the
    # precision workload at its full size, single-pass tiles)
    torch = gu.torch()
    b, m = 8192, 12
    xh = workloads.to_half_precision(workloads.outlier_signals(3001, b, m), dtype)
    xd = xh.reshape(-1).cuda()
    p_h, p_f = _pair([m] * b, dtype)
    yh = p_h.forward(xd)
    yf = p_f.forward(xd.float())
    # the adjoint through the synthesis kernels narrows the same way
    p_h2, p_f2 = _pair([m] * b, dtype, options={"adjoint": 1})
    gh = p_h2.backward(xd)
    gf = p_f2.backward(xd.float())
    torch.cuda.synchronize()
    assert gu.narrowing_mismatches(yh, yf, dtype) == 0
    assert gu.narrowing_mismatches(gh, gf, dtype) == 0


def _two_pass_set():
    rng = np.random.default_rng(9101)
    sizes = [20, 17, 16, 13, 14, 15, 12, 9, 6, 3, 18, 16]
    sizes += [int(k) for k in rng.integers(4, 17, size=20)]
    x = np.concatenate([workloads.outlier_signals(9100 + i, 1, k).reshape(-1)
                        for i, k in enumerate(sizes)])
    return sizes, x


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
@pytest.mark.parametrize("options", [{}, {"lr12": 6, "lr15": 6, "single15": 0},
                                     {"exec": 2}, {"adjoint": 1}])
def test_ragged_two_pass_rne(dtype, options):
    torch = gu.torch()
    sizes, x32 = _two_pass_set()
    xd = workloads.to_half_precision(x32, dtype).cuda()
    p_h, p_f = _pair(sizes, dtype, options=options)
    ws = torch.empty(max(p_h.workspace_size(), p_f.workspace_size(), 16),
                     dtype=torch.uint8, device="cuda")
    yh = p_h.forward(xd, workspace=ws)
    torch.cuda.synchronize()
    yf = p_f.forward(xd.float(), workspace=ws)
    if options.get("adjoint"):
        gh = p_h.backward(xd, workspace=ws)
        torch.cuda.synchronize()
        gf = p_f.backward(xd.float(), workspace=ws)
    torch.cuda.synchronize()
    assert gu.narrowing_mismatches(yh, yf, dtype) == 0
    if options.get("adjoint"):
        assert gu.narrowing_mismatches(gh, gf, dtype) == 0


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_large_two_pass_rne(dtype):
    # each first-pass row count of the 2^15-element tiles at its largest size
    # (2^23: 2^7 rows, 2^24: 2^6, 2^25: 2^5), in the dyadic and sequency
    # orders and with and without prefetching
    torch = gu.torch()
    sizes = [24, 23, 25]
    x32 = np.concatenate([workloads.outlier_signals(9200 + i, 1, k).reshape(-1)
                          for i, k in enumerate(sizes)])
    xd = workloads.to_half_precision(x32, dtype).cuda()
    for order in ("dyadic", "sequency"):
        for stream in (1, 0):
            p_h = chw.Plan(sizes, dtype=dtype, order=order)
            p_f = chw.Plan(sizes, dtype="f32", order=order)
            for p in (p_h, p_f):
                p.set_option("stream", stream)
            yh = p_h.forward(xd)
            torch.cuda.synchronize()
            yf = p_f.forward(xd.float())
            torch.cuda.synchronize()
            assert gu.narrowing_mismatches(yh, yf, dtype) == 0, (order, stream)
            del yh, yf


def test_ragged_bf16_bench_form_rne():
    # the ragged workload at its full size (20000 signals, 2^30 elements) in
    # the launch configuration the benchmark times, against the FP32 plan of
    # the same configuration; the whole output on the device with torch's
    # conversion, a sample on the host
    torch = gu.torch()
    ks = workloads.ragged_log2_sizes(4001)
    offs = workloads.packed_offsets(ks)
    xb = workloads.to_half_precision(workloads.ragged_values(4002, ks, offs), "bf16").cuda()
    p_h = bench.tuned_ragged_plan(ks, offs, "bf16")
    p_f = bench.tuned_ragged_plan(ks, offs, "f32")
    ws = torch.empty(max(p_h.workspace_size(), 16), dtype=torch.uint8, device="cuda")
    yh = p_h.forward(xb, workspace=ws)
    torch.cuda.synchronize()
    del ws
    xf = xb.float()
    yf = p_f.forward(xf)
    torch.cuda.synchronize()
    del xf
    bad = int((yh.view(torch.int16) != yf.to(torch.bfloat16).view(torch.int16)).sum())
    assert bad == 0
    sel = torch.from_numpy(np.random.default_rng(3).integers(0, yh.numel(), 1 << 20)).cuda()
    assert gu.narrowing_mismatches(yh[sel], yf[sel], "bf16") == 0
