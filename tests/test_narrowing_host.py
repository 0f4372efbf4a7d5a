"""Host side of the narrowing pin (tests/test_gpu_narrowing.py): the bitwise
comparison with round-to-nearest-even rejects a truncating narrowing, which
the relative-L2 bound of the precision forms (4e-3) would let through.

The values are FP32 results of the oracle's cascade (eq. 3) on the precision
workload's inputs, i.e. numbers of the kind the GPU narrows."""

import numpy as np
import pytest

import workloads
from oracle import cascade, metrics
from tests import gpu_util as gu


def _values():
    x = workloads.outlier_signals(3001, 16, 12)
    x = workloads.to_half_precision(x, "bf16").float().numpy().astype(np.float64)
    return cascade.chw_forward(x).astype(np.float32)


def _truncate(v32, dtype):
    """Round toward zero to bf16 / f16 (the planted mistake)."""
    import torch
    if dtype == "bf16":
        bits = v32.view(np.uint32) & np.uint32(0xFFFF0000)
        return torch.from_numpy((bits >> 16).astype(np.uint16).view(np.int16)).view(torch.bfloat16)
    rne = v32.astype(np.float16)
    over = np.abs(rne.astype(np.float64)) > np.abs(v32.astype(np.float64))
    mag = rne.view(np.uint16) & np.uint16(0x7FFF)
    sign = rne.view(np.uint16) & np.uint16(0x8000)
    mag = np.where(over, mag - np.uint16(1), mag).astype(np.uint16)
    return torch.from_numpy((sign | mag).view(np.int16)).view(torch.float16)


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_rne_passes_truncation_fails(dtype):
    import torch
    v = _values().reshape(-1)
    t = torch.from_numpy(v)
    rne = gu.rne_narrow(t, dtype)
    assert gu.narrowing_mismatches(rne, t, dtype) == 0
    trunc = _truncate(v, dtype)
    bad = gu.narrowing_mismatches(trunc, t, dtype)
    # about half of the elements round up under RNE, so truncation differs there
    assert bad > v.size // 4
    # ... while both pass the relative-L2 bound the precision forms are graded by
    ref = v.astype(np.float64)
    for cand in (rne, trunc):
        assert metrics.rel_l2(cand.double().numpy(), ref) <= 4e-3


def test_truncation_helper_rounds_toward_zero():
    import torch
    v = np.array([1.0 + 2 ** -9, -(1.0 + 2 ** -9), 3.0, -0.0, 1.0 + 3 * 2 ** -11],
                 dtype=np.float32)
    tb = _truncate(v, "bf16").float().numpy()
    assert np.all(np.abs(tb) <= np.abs(v))
    th = _truncate(v, "f16").float().numpy()
    assert np.all(np.abs(th) <= np.abs(v))
    assert th[4] == np.float32(1.0 + 2 ** -10)   # RNE would give 1 + 2^-9
    assert torch.equal(gu.rne_narrow(torch.from_numpy(v[:4]), "f16").float(),
                       torch.from_numpy(v[:4].astype(np.float16).astype(np.float32)))
