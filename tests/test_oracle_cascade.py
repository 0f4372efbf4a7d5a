"""Pins for the oracle cascade (Sec. 2), its adjoint, the op counter (Lemma 1,
Theorem 2) and the plain-C twin."""

import numpy as np
import pytest

from oracle import c_oracle, cascade, dense, metrics


# ---------------------------------------------------------------------------
# hand-worked examples

def test_worked_example_m2(golden_hand):
    x = golden_hand["x_m2"][0]
    v = x.astype(np.int64).copy()
    cascade.haar_forward(v, 0, 4, 1)
    assert np.array_equal(v, golden_hand["after_Psi2"][0])
    assert np.array_equal(cascade.chw_forward(x), golden_hand["after_F1_m2"][0])


def test_worked_example_m3(golden_hand):
    x = golden_hand["x_m3"][0]
    v = x.astype(np.int64).copy()
    sched = cascade.cascade_schedule(3)
    stages = {0: "after_Psi3", 1: "after_F1_m3", 2: "after_F2_m3"}
    for f in range(3):
        for factor, lo, size in sched:
            if factor == f:
                cascade.haar_forward(v, lo, size, 1)
        assert np.array_equal(v, golden_hand[stages[f]][0]), f
    assert np.array_equal(cascade.chw_forward(x), golden_hand["after_F2_m3"][0])


# ---------------------------------------------------------------------------
# cascade = dense H_m

def _inputs(m, rng):
    n = 1 << m
    xs = [rng.standard_normal(n), np.eye(n)[0], np.eye(n)[n - 1]]
    psi = dense.haar_matrix(m)
    xs += [psi.T[:, k] for k in range(min(n, 4))]  # Haar basis vectors (eq. 4)
    return np.stack(xs)


@pytest.mark.parametrize("m", range(0, 11))
def test_cascade_equals_dense(m):
    rng = np.random.default_rng(100 + m)
    h = dense.hadamard_paley(m)
    x = _inputs(m, rng)
    y = cascade.chw_forward(x)
    assert np.max(np.abs(y - x @ h.T)) <= 1e-12 * max(1, np.max(np.abs(x)) * (1 << m))
    xi = rng.integers(-128, 128, size=(3, 1 << m))
    assert np.array_equal(cascade.chw_forward(xi),
                          xi @ dense.hadamard_paley(m, exact=True).T)


@pytest.mark.parametrize("m", range(0, 7))
def test_brute_force_every_basis_vector(m):
    # All columns: H_m e_j must be column j of the closed form.
    n = 1 << m
    eye = np.eye(n, dtype=np.int64)
    cols = cascade.chw_forward(eye)          # row j = H' e_j
    assert np.array_equal(cols.T, cascade.closed_form(m, exact=True))


@pytest.mark.parametrize("m", range(1, 15))
def test_cascade_bitwise_equals_radix2(m):
    # The cascade performs the butterflies of the textbook radix-2 WHT over
    # index bits 0..m-1 (same operands, same order), read in dyadic order:
    # bitwise equal in float64.
    rng = np.random.default_rng(7 + m)
    x = rng.standard_normal((2, 1 << m))
    a = cascade.chw_forward(x)
    b = cascade.radix2_paley(x)
    assert np.array_equal(a, b)
    xi = rng.integers(-128, 128, size=(2, 1 << m))
    assert np.array_equal(cascade.chw_forward(xi), cascade.radix2_paley(xi))


@pytest.mark.parametrize("m,split", [(8, 3), (9, 4), (10, 5), (10, 1), (7, 6)])
def test_level_split(m, split):
    # After the first `split` stages, the rest of the cascade is CHW_{m-split}
    # on each of 2^split contiguous blocks (the induction step of the proof in
    # Sec. 5, applied `split` times).  Stage t = all Haar levels at depth t.
    rng = np.random.default_rng(m * 10 + split)
    x = rng.integers(-128, 128, size=1 << m)
    n = 1 << m
    # first `split` stages in the cascade's own layout
    v = x.astype(np.int64).copy()
    for t in range(split):
        blk = n >> t
        w = v.reshape(1 << t, blk)
        a = w[:, 0::2].copy()
        b = w[:, 1::2].copy()
        w[:, :blk // 2] = a + b
        w[:, blk // 2:] = a - b
        v = w.reshape(n)
    rest = cascade.chw_forward(v.reshape(1 << split, n >> split)).reshape(n)
    assert np.array_equal(rest, cascade.chw_forward(x))


def test_schedule_matches_theorem2_structure():
    # Proof of Theorem 2: one Haar of size 2^m and 2^{m-1-r} of size 2^r for
    # r = 1..m-1; the blocks are the second halves of F_r's blocks.
    for m in range(1, 12):
        sched = cascade.cascade_schedule(m)
        sizes = [s for _f, _o, s in sched]
        assert sizes.count(1 << m) == 1
        for r in range(1, m):
            assert sizes.count(1 << r) == 1 << (m - 1 - r)
        for f, o, s in sched[1:]:
            big = 2 * s
            assert o % big == s           # second half of a block of 2s
            assert s == 1 << (m - f)


# ---------------------------------------------------------------------------
# operation counts (Lemma 1, Theorem 2)

@pytest.mark.parametrize("k", range(0, 16))
def test_lemma1_haar_count(k):
    ctr = cascade.OpCounter()
    cascade.haar_forward(np.zeros(1 << k, dtype=np.int64), 0, 1 << k, 1, ctr)
    assert ctr.adds == 2 * ((1 << k) - 1)


@pytest.mark.parametrize("m", range(1, 21))
def test_theorem2_count(m):
    total = cascade.count_ops(m)
    assert total == m * (1 << m)
    # the three lines of the proof of Theorem 2
    line1 = 2 * ((1 << m) - 1) + sum((1 << (m - 1 - r)) * 2 * ((1 << r) - 1)
                                     for r in range(1, m))
    line2 = (1 << (m + 1)) - 2 + sum(1 << m for r in range(1, m)) \
        - sum(1 << (m - r) for r in range(1, m))
    line3 = (1 << (m + 1)) - 2 + (1 << m) * (m - 1) - 2 * ((1 << (m - 1)) - 1)
    assert total == line1 == line2 == line3


@pytest.mark.parametrize("m", range(2, 12))
def test_per_factor_count(m):
    # factor r performs 2^{r-1} Haars of 2^{m-r}: 2^{r-1} * 2(2^{m-r}-1)
    # = 2^m - 2^r additions
    for r in range(1, m):
        ctr = cascade.OpCounter()
        v = np.zeros(1 << m, dtype=np.int64)
        for f, o, s in cascade.cascade_schedule(m):
            if f == r:
                cascade.haar_forward(v, o, s, 1, ctr)
        assert ctr.adds == (1 << m) - (1 << r)


# ---------------------------------------------------------------------------
# invariants

@pytest.mark.parametrize("m", [0, 1, 2, 5, 9, 12])
def test_invariants(m):
    rng = np.random.default_rng(31 + m)
    n = 1 << m
    x = rng.standard_normal((3, n))
    y = cascade.chw_forward(x)
    # Parseval (orthonormal H_m)
    assert np.allclose(np.linalg.norm(y, axis=1), np.linalg.norm(x, axis=1), rtol=1e-12)
    # DC term: first row of H_m is 2^{-m/2} (1 ... 1)
    assert np.allclose(y[:, 0], x.sum(axis=1) * 2.0 ** (-m / 2), rtol=1e-12, atol=1e-12)
    # involution H(Hx) = x
    assert np.allclose(cascade.chw_forward(y), x, atol=1e-11)
    # integer form: H'(H'x) = n x
    xi = rng.integers(-128, 128, size=(2, n))
    assert np.array_equal(cascade.chw_forward(cascade.chw_forward(xi)), n * xi)
    # impulse e_j -> column j of H_m
    j = n // 3 if n > 2 else 0
    e = np.zeros(n)
    e[j] = 1
    assert np.allclose(cascade.chw_forward(e), dense.hadamard_paley(m)[:, j], atol=1e-14)


@pytest.mark.parametrize("m", range(0, 13))
def test_adjoint(m):
    rng = np.random.default_rng(55 + m)
    n = 1 << m
    g = rng.standard_normal((2, n))
    x = rng.standard_normal((2, n))
    ht = cascade.chw_adjoint(g)
    # dense transpose (small m)
    if m <= 9:
        assert np.allclose(ht, g @ dense.hadamard_paley(m), atol=1e-12)
    # dot test <Hx, g> = <x, H^T g>
    lhs = np.sum(cascade.chw_forward(x) * g, axis=1)
    rhs = np.sum(x * ht, axis=1)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    # H symmetric: the adjoint equals the forward (exact in integers)
    gi = rng.integers(-128, 128, size=(2, n))
    assert np.array_equal(cascade.chw_adjoint(gi), cascade.chw_forward(gi))
    assert np.allclose(ht, cascade.chw_forward(g), atol=1e-12)


def test_integer_range_extremes():
    # After t stages every value is a +-1 combination of 2^t inputs, so with
    # |x| <= 128 and n <= 2^22 nothing leaves int32.  Extremes at m = 22 via
    # the C twin (shown equal to the Python cascade below).
    m = 22
    n = 1 << m
    for val in (127, -128):
        y = c_oracle.chw_batch(np.full(n, val, dtype=np.int64), [m])
        assert y[0] == val * n and np.all(y[1:] == 0)
    # x = 127 * (row i of H'_m) gives y_i = 127 * 2^22
    i = 12345
    ri = cascade.bitrev(i, m)
    j = np.arange(n, dtype=np.int64)
    pop = np.zeros(n, dtype=np.int64)
    t = ri & j
    while np.any(t):
        pop += t & 1
        t >>= 1
    row = np.where(pop & 1, -1, 1).astype(np.int64)
    y = c_oracle.chw_batch(127 * row, [m])
    assert y[i] == 127 * n
    assert np.max(np.abs(y)) < 2 ** 31


# ---------------------------------------------------------------------------
# the plain-C twin equals the Python cascade

def test_c_oracle_matches_python():
    rng = np.random.default_rng(2024)
    sizes = np.array([0, 1, 2, 3, 6, 10, 12, 4, 9], dtype=np.int32)
    # ragged layout with gaps between signals
    offs = []
    o = 5
    for k in sizes:
        offs.append(o)
        o += (1 << int(k)) + int(rng.integers(0, 7))
    offs = np.array(offs, dtype=np.int64)
    total = o + 3
    xf = rng.standard_normal(total)
    xi = rng.integers(-128, 128, size=total)
    for adj in (False, True):
        yf = c_oracle.chw_batch(xf, sizes, offs, adjoint=adj, threads=3)
        yi = c_oracle.chw_batch(xi, sizes, offs, adjoint=adj, threads=2)
        mask = np.ones(total, dtype=bool)
        for k, off in zip(sizes, offs):
            n = 1 << int(k)
            fn = cascade.chw_adjoint if adj else cascade.chw_forward
            assert np.array_equal(yf[off:off + n], fn(xf[off:off + n]))
            assert np.array_equal(yi[off:off + n], fn(xi[off:off + n]))
            mask[off:off + n] = False
        assert np.array_equal(yf[mask], xf[mask])   # gaps untouched
        assert np.array_equal(yi[mask], xi[mask])


def test_c_oracle_rows_threads_agree():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((12, 1 << 11))
    a = c_oracle.chw_rows(x, threads=1)
    b = c_oracle.chw_rows(x, threads=5)
    assert np.array_equal(a, b)
    assert np.array_equal(a, cascade.chw_forward(x))


def test_metrics():
    y = np.array([[3.0, 4.0], [0.0, 0.0]])
    yh = np.array([[3.0, 4.5], [0.0, 0.1]])
    r = metrics.rel_l2(yh, y)
    assert np.isclose(r[0], 0.1) and np.isclose(r[1], 0.1)
    assert metrics.exact_equal(np.array([1, -2]), np.array([1, -2], dtype=np.int32))


@pytest.mark.parametrize("m", [1, 3, 6, 9])
def test_coefficient_rows_of_eq1(m):
    # each output of the O(n) single-coefficient form equals the row of the
    # dense H_m of eq. (1) applied to the vector (integer: exactly; float:
    # to rounding), and, for float input, the cascade's output
    from oracle import dense
    rng = np.random.default_rng(900 + m)
    n = 1 << m
    xi = rng.integers(-128, 128, n)
    xf = rng.standard_normal(n)
    Hi = dense.hadamard_paley(m, exact=True)
    Hf = dense.hadamard_paley(m)
    yc = cascade.chw_forward(xf)
    for i in range(n):
        assert cascade.coefficient(xi, i, chunk=5) == int(Hi[i] @ xi)
        got = cascade.coefficient(xf, i, chunk=7)
        assert abs(got - Hf[i] @ xf) <= 1e-12 * (1 + abs(got))
        assert abs(got - yc[i]) <= 1e-12 * (1 + abs(got))


def test_coefficient_catches_a_wrong_row():
    # a planted mistake (the row index not bit-reversed) changes the result
    m = 5
    x = np.random.default_rng(1).standard_normal(1 << m)
    i = 1  # bitrev_5(1) = 16 != 1
    good = cascade.coefficient(x, i)
    r = np.int64(i)
    j = np.arange(1 << m, dtype=np.int64)
    wrong = float(np.sum(np.where(np.bitwise_count(j & r) & 1, -x, x))) * 2.0 ** (-m / 2)
    assert abs(good - wrong) > 1e-6
