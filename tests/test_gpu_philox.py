"""GPU parity of the device-drawn random signs (chw_philox_signs): the
Philox4x64-10 words bit for bit against the oracle's generator, and the
randomized transform on those signs against the oracle end to end."""

import numpy as np
import pytest

import workloads
from oracle import philox, signed
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


def _words_host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("sizes,mode", [([6], "shared"), ([3, 7, 12], "shared"),
                                        ([3, 7, 12], "per_element"), ([17] * 2, "shared"),
                                        ([10] * 33, "per_element")])
@pytest.mark.parametrize("seed", [0, 20240601, 2**64 - 1])
@pytest.mark.parametrize("rounds", [1, 3])
def test_words_match_oracle(sizes, mode, seed, rounds):
    t = gu.torch()
    p = chw.Plan(sizes, dtype="f32")
    w = p.sign_words(mode)
    # one word of lead-in (4-byte but not 16-byte aligned start) and sentinels
    buf = t.full((rounds * w + 16,), 0x5A5A5A5A, dtype=t.int32, device="cuda")
    view = buf[1:1 + rounds * w]
    p.philox_signs(seed, rounds, mode, out=view)
    t.cuda.synchronize()
    host = _words_host(buf)
    want = philox.sign_words(seed, rounds, w).reshape(-1)
    assert np.array_equal(host[1:1 + rounds * w], want)
    assert host[0] == 0x5A5A5A5A and np.all(host[1 + rounds * w:] == 0x5A5A5A5A)
    # aligned start: same words
    al = p.philox_signs(seed, rounds, mode)
    t.cuda.synchronize()
    assert np.array_equal(_words_host(al)[:rounds * w], want)


def test_diff_workload_with_device_signs():
    # y = H D x on 256 x 2^14 FP32 with D drawn on the device; gradient D H^T g
    m, batch, seed = 14, 256, 5002
    t = gu.torch()
    p = chw.Plan([m] * batch, dtype="f32")
    x = workloads.float_signals(5001, batch, m)
    g = workloads.float_signals(5003, batch, m)
    s = p.philox_signs(seed, 1, "shared")
    xd, gd = gu.dev_tensor(x, "f32"), gu.dev_tensor(g, "f32")
    y = p.forward_signed(xd, s, "shared", 1)
    gx = p.backward_signed(gd, s, "shared", 1)
    t.cuda.synchronize()
    d = philox.diagonals(philox.sign_words(seed, 1, p.sign_words("shared")), 1 << m)[0]
    idx = [0, 131, 255]
    ref = signed.signed_forward(x[idx].astype(np.float64), [d])
    ref_g = signed.signed_adjoint(g[idx].astype(np.float64), [d])
    yh, gh = gu.host_f64(y), gu.host_f64(gx)
    assert max(gu.metrics.rel_l2(a, b) for a, b in zip(yh[idx], ref)) <= 1e-5
    assert max(gu.metrics.rel_l2(a, b) for a, b in zip(gh[idx], ref_g)) <= 1e-5


@pytest.mark.parametrize("mode", ["shared", "per_element"])
def test_ragged_rounds_with_device_signs(mode):
    t = gu.torch()
    sizes = [2, 9, 13, 12, 17, 10]
    offs = np.concatenate([[0], np.cumsum([1 << k for k in sizes])]).astype(np.int64)
    rounds, seed = 3, 777
    x = np.concatenate([workloads.float_signals(790 + i, 1, k)[0] for i, k in enumerate(sizes)])
    p = chw.Plan(sizes, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    ws = t.empty(max(p.workspace_size(), 16), dtype=t.uint8, device="cuda")
    s = p.philox_signs(seed, rounds, mode)
    y = p.forward_signed(xd, s, mode, rounds, workspace=ws)
    t.cuda.synchronize()
    nbits = (1 << max(sizes)) if mode == "shared" else int(offs[-1])
    diags = philox.diagonals(philox.sign_words(seed, rounds, p.sign_words(mode)), nbits)
    flat = diags if mode == "per_element" else workloads.expand_shared_signs(diags, sizes)
    ref = signed.signed_batch(x.astype(np.float64), sizes, list(flat))
    assert gu.per_signal_rel(gu.host_f64(y), ref, sizes).max() <= gu.TOL["f32"] * rounds


def test_philox_signs_validation():
    t = gu.torch()
    p = chw.Plan([8], dtype="f32")
    with pytest.raises(chw.CHWError):
        p.philox_signs(1, 0)
    with pytest.raises(chw.CHWError):
        p.philox_signs(1, 65)
