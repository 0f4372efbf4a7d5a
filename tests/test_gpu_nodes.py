"""GPU parity of the factor-by-factor node evaluation (chw_nodes_forward, the
decomposition of Sec. 4): every size class of its two kernels (sub-vectors
inside a tile, chunks with a sums pass) and the chunked schedule, against
the oracle."""

import numpy as np
import pytest

import workloads
from paper_1609_06641_amd import chw
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("batch,m,chunk", [
    (3, 1, 0), (5, 3, 0), (64, 10, 0), (2, 11, 0), (3, 12, 0), (2, 13, 0), (4, 14, 3),
    (2, 16, 0), (2, 20, 0), (3, 20, 1), (1, 24, 0),
])
def test_nodes_match_oracle(batch, m, chunk):
    t = gu.torch()
    x = workloads.float_signals(1300 + m, batch, m).reshape(-1)
    p = chw.Plan([m] * batch, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    ws = t.full((p.nodes_workspace_size() // 4,), float("nan"), dtype=t.float32, device="cuda")
    y = t.full_like(xd, float("nan"))
    p.nodes_forward(xd, out=y, workspace=ws, chunk=chunk)
    t.cuda.synchronize()
    ref = gu.oracle_packed(x.astype(np.float64), [m] * batch)
    assert gu.per_signal_rel(gu.host_f64(y), ref, [m] * batch).max() <= gu.TOL["f32"]
    # the input is left alone
    assert np.array_equal(gu.host_f64(xd), x.astype(np.float64))


def test_nodes_repeat_with_dirty_workspace():
    # a second call on a workspace holding the first call's data gives the same bits
    t = gu.torch()
    m, batch = 18, 4
    x = workloads.float_signals(1350, batch, m).reshape(-1)
    p = chw.Plan([m] * batch, dtype="f32")
    xd = gu.dev_tensor(x, "f32")
    ws = t.empty(p.nodes_workspace_size(), dtype=t.uint8, device="cuda")
    a = p.nodes_forward(xd, workspace=ws)
    b = p.nodes_forward(xd, workspace=ws, chunk=2)
    t.cuda.synchronize()
    assert t.equal(a, b)
