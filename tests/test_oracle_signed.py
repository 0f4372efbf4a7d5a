"""Pins of the randomized (signed) oracle, oracle.signed, against the dense
definition y = H D_k ... H D_1 x with H from eq. (1)."""

import numpy as np
import pytest

import workloads
from oracle import c_oracle, cascade, dense, signed


def _dense_signed(m, diags, exact=False):
    h = dense.hadamard_paley(m, exact=exact)
    mat = np.eye(1 << m, dtype=h.dtype)
    for d in diags:
        mat = h @ np.diag(d.astype(h.dtype)) @ mat
    return mat


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_signed_matches_dense_product(m, k):
    n = 1 << m
    diags = workloads.sign_rounds(11 + m, k, n)
    x = workloads.float_signals(21, 3, m).astype(np.float64)
    want = x @ _dense_signed(m, diags).T
    got = signed.signed_forward(x, list(diags))
    assert np.max(np.abs(got - want)) < 1e-12 * np.sqrt(n)
    # the adjoint is the transposed product
    g = workloads.float_signals(22, 3, m).astype(np.float64)
    want_a = g @ _dense_signed(m, diags)
    got_a = signed.signed_adjoint(g, list(diags))
    assert np.max(np.abs(got_a - want_a)) < 1e-12 * np.sqrt(n)


@pytest.mark.parametrize("m", [1, 4, 7])
def test_signed_integer_exact(m):
    n = 1 << m
    diags = workloads.sign_rounds(5, 2, n)
    x = workloads.int_signals(23, 2, m).astype(np.int64)
    want = x @ _dense_signed(m, diags, exact=True).T
    got = signed.signed_forward(x, list(diags))
    assert got.dtype == np.int64 and np.array_equal(got, want)


def test_signed_special_diagonals():
    m, n = 6, 64
    x = workloads.float_signals(24, 2, m).astype(np.float64)
    plus, minus = np.ones(n, np.int8), -np.ones(n, np.int8)
    assert np.array_equal(signed.signed_forward(x, [plus]), cascade.chw_forward(x))
    assert np.array_equal(signed.signed_forward(x, [minus]), -cascade.chw_forward(x))
    # two rounds with D = I: H H = I (the transform is an involution)
    assert np.allclose(signed.signed_forward(x, [plus, plus]), x, atol=1e-13)


def test_signed_round_order_matters():
    m, n = 5, 32
    diags = workloads.sign_rounds(3, 2, n)
    x = workloads.float_signals(25, 1, m).astype(np.float64)
    a = signed.signed_forward(x, [diags[0], diags[1]])
    b = signed.signed_forward(x, [diags[1], diags[0]])
    assert not np.allclose(a, b)


def test_signed_dot_identity():
    m, n = 9, 512
    diags = list(workloads.sign_rounds(9, 3, n))
    x = workloads.float_signals(26, 1, m).astype(np.float64)[0]
    g = workloads.float_signals(27, 1, m).astype(np.float64)[0]
    lhs = np.dot(signed.signed_forward(x, diags), g)
    rhs = np.dot(x, signed.signed_adjoint(g, diags))
    assert abs(lhs - rhs) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(g)


@pytest.mark.parametrize("adjoint", [False, True])
def test_signed_batch_matches_per_signal(adjoint):
    sizes = [3, 10, 6, 12]
    offs = np.array([0, 16, 16 + 1024 + 32, 16 + 1024 + 32 + 64, 16 + 1024 + 32 + 64 + 4096],
                    dtype=np.int64)
    extent = int(offs[-1])
    x = np.zeros(extent)
    for i, k in enumerate(sizes):
        x[offs[i]:offs[i] + (1 << k)] = workloads.float_signals(30 + i, 1, k)[0]
    shared = workloads.sign_rounds(31, 2, 1 << max(sizes))
    flat = workloads.expand_shared_signs(shared, sizes, offs)
    got = signed.signed_batch(x, sizes, list(flat), offsets=offs[:-1], adjoint=adjoint)
    for i, k in enumerate(sizes):
        n = 1 << k
        fn = signed.signed_adjoint if adjoint else signed.signed_forward
        want = fn(x[offs[i]:offs[i] + n], [d[:n] for d in shared])
        assert np.allclose(got[offs[i]:offs[i] + n], want, rtol=0, atol=1e-12)
    assert c_oracle.chw_batch is not None


def test_pack_sign_bits_layout():
    d = workloads.sign_rounds(8, 2, 100)
    words = workloads.pack_sign_bits(d)
    assert words.shape == (2, 4) and words.dtype == np.uint32
    for r in range(2):
        for b in range(100):
            assert ((int(words[r, b // 32]) >> (b % 32)) & 1) == int(d[r, b] < 0)
        assert int(words[r, 3]) >> 4 == 0   # bits past n stay clear


# ---- planted mistakes in the signed oracle (on the CPU) -----------------------

def _signed_pins_hold(fwd, adj):
    ok = True
    for m, k in ((3, 1), (4, 2), (5, 3)):
        n = 1 << m
        diags = workloads.sign_rounds(40 + m, k, n)
        x = np.arange(1, n + 1, dtype=np.int64) * 5 - 11
        mat = _dense_signed(m, diags, exact=True)
        ok &= np.array_equal(fwd(x, list(diags)), mat @ x)
        ok &= np.array_equal(adj(x, list(diags)), mat.T @ x)
    return bool(ok)


def test_signed_pins_hold_unmutated():
    assert _signed_pins_hold(signed.signed_forward, signed.signed_adjoint)


def _sign_after_transform(x, diags, exact=None):
    v = x
    for d in diags:
        v = cascade.chw_forward(v, exact) * d.astype(np.int64)
    return v


def _rounds_reversed(x, diags, exact=None):
    return signed.signed_forward(x, list(reversed(list(diags))), exact)


def _adjoint_sign_before(g, diags, exact=None):
    v = g
    for d in reversed(list(diags)):
        v = cascade.chw_adjoint(v * d.astype(np.int64), exact)
    return v


def _adjoint_rounds_forward_order(g, diags, exact=None):
    v = g
    for d in diags:
        v = cascade.chw_adjoint(v, exact) * d.astype(np.int64)
    return v


@pytest.mark.parametrize("fwd,adj", [
    (_sign_after_transform, signed.signed_adjoint),
    (_rounds_reversed, signed.signed_adjoint),
    (signed.signed_forward, _adjoint_sign_before),
    (signed.signed_forward, _adjoint_rounds_forward_order),
])
def test_signed_planted_mistakes_are_caught(fwd, adj):
    assert not _signed_pins_hold(fwd, adj)
