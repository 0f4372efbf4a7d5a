"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one.  This shows the pins constrain every part of the oracle: a
dropped term, a wrong sign or index, a transposed operand, a wrong order."""

import numpy as np
import pytest

from oracle import cascade, dense
from tests.conftest import load_golden

GOLD = load_golden("hand_worked_m2_m3.txt")


def _pins_hold():
    """Run a compact version of the pins; True iff all of them hold."""
    ok = True
    # hand-worked cascade examples (Sec. 2)
    ok &= np.array_equal(cascade.chw_forward(GOLD["x_m3"][0]), GOLD["after_F2_m3"][0])
    ok &= np.array_equal(cascade.chw_forward(GOLD["x_m2"][0]), GOLD["after_F1_m2"][0])
    # hand-worked matrices (eqs. 1-2)
    ok &= np.array_equal(dense.hadamard_paley(3, exact=True), GOLD["H3"])
    ok &= np.array_equal(dense.haar_matrix(3, exact=True), GOLD["Psi3"])
    for m in (3, 4, 5):
        # Theorem 1 exact, closed form, cascade = dense
        h = dense.hadamard_paley(m, exact=True)
        ok &= np.array_equal(dense.theorem1_rhs(m, exact=True), h)
        ok &= np.array_equal(cascade.closed_form(m, exact=True), h)
        x = np.arange(1, (1 << m) + 1, dtype=np.int64) * 3 - 7
        ok &= np.array_equal(cascade.chw_forward(x), h @ x)
        ok &= np.array_equal(cascade.chw_adjoint(x), h.T @ x)
        # op count (Theorem 2)
        ok &= cascade.count_ops(m) == m * (1 << m)
        # orthonormal forms: Parseval and eq. (4)
        xf = np.linspace(-1, 2, 1 << m)
        ok &= bool(np.isclose(np.linalg.norm(cascade.chw_forward(xf)), np.linalg.norm(xf)))
        ok &= bool(np.allclose(dense.hadamard_paley(m) @ dense.haar_matrix(m).T,
                               dense.haar_walsh(m), atol=1e-12))
    return bool(ok)


def test_unmutated_pins_hold():
    assert _pins_hold()


def _level_swapped(v, lo, length, c, counter=None):
    half = length // 2
    a = v[..., lo:lo + length:2].copy()
    b = v[..., lo + 1:lo + length:2].copy()
    v[..., lo:lo + half] = (a - b) * c      # details in the lower half
    v[..., lo + half:lo + length] = (a + b) * c


def _level_sign(v, lo, length, c, counter=None):
    half = length // 2
    a = v[..., lo:lo + length:2].copy()
    b = v[..., lo + 1:lo + length:2].copy()
    v[..., lo:lo + half] = (a + b) * c
    v[..., lo + half:lo + length] = (b - a) * c   # second minus first


def _level_no_count(v, lo, length, c, counter=None):
    half = length // 2
    a = v[..., lo:lo + length:2].copy()
    b = v[..., lo + 1:lo + length:2].copy()
    v[..., lo:lo + half] = (a + b) * c
    v[..., lo + half:lo + length] = (a - b) * c     # forgets to count


def _haar_one_level_short(v, lo, length, c, counter=None):
    while length >= 4:
        cascade.haar_level(v, lo, length, c, counter)
        length //= 2


def _sched_lower_half(m):
    n = 1 << m
    out = [(0, 0, n)] if m >= 1 else []
    for r in range(1, m):
        big = 1 << (m - r + 1)
        for b in range(1 << (r - 1)):
            out.append((r, b * big, big // 2))
    return out


_orig_sched = cascade.cascade_schedule


def _sched_reversed_factors(m):
    s = _orig_sched(m)
    return s[:1] + sorted(s[1:], key=lambda t: -t[0])


def _sched_missing_last(m):
    return [t for t in _orig_sched(m) if t[0] != m - 1 or m < 2]


def _adj_fine_to_coarse(v, lo, length, c, counter=None):
    h = length // 2
    while h >= 1:
        a = v[..., lo:lo + h].copy()
        d = v[..., lo + h:lo + 2 * h].copy()
        v[..., lo:lo + 2 * h:2] = (a + d) * c
        v[..., lo + 1:lo + 2 * h:2] = (a - d) * c
        h //= 2


def _hadamard_natural(m, exact=False):
    dt, c = (np.int64, 1) if exact else (np.float64, 1 / np.sqrt(2))
    a = np.ones((1, 1), dtype=dt)
    for _ in range(m):
        a = np.vstack([np.kron(np.array([[1, 1]], dtype=dt), a),
                       np.kron(np.array([[1, -1]], dtype=dt), a)])  # operands swapped
        if not exact:
            a = a * c
    return a


def _haar_bad_detail(m, exact=False):
    dt, c = (np.int64, 1) if exact else (np.float64, 1 / np.sqrt(2))
    a = np.ones((1, 1), dtype=dt)
    for k in range(m):
        a = np.vstack([np.kron(a, np.array([[1, 1]], dtype=dt)),
                       np.kron(np.eye(1 << k, dtype=dt), np.array([[-1, 1]], dtype=dt))])
        if not exact:
            a = a * c
    return a


def _factor_transposed_blocks(m, r, exact=False):
    inner = dense.block_diag(dense.haar_matrix(m - r, exact), dense.identity(m - r, exact))
    return np.kron(dense.identity(r - 1, exact), inner)


MUTATIONS = [
    ("detail/sum halves swapped", cascade, "haar_level", _level_swapped),
    ("difference sign flipped", cascade, "haar_level", _level_sign),
    ("op counter drops terms", cascade, "haar_level", _level_no_count),
    ("Haar pyramid one level short", cascade, "haar_forward", _haar_one_level_short),
    ("factor acts on lower half", cascade, "cascade_schedule", _sched_lower_half),
    ("factors in reverse order", cascade, "cascade_schedule", _sched_reversed_factors),
    ("last factor dropped", cascade, "cascade_schedule", _sched_missing_last),
    ("synthesis fine-to-coarse", cascade, "haar_adjoint", _adj_fine_to_coarse),
    ("eq.1 Kronecker operands swapped", dense, "hadamard_paley", _hadamard_natural),
    ("eq.2 detail sign flipped", dense, "haar_matrix", _haar_bad_detail),
    ("Theorem 1 blocks swapped", dense, "theorem1_factor", _factor_transposed_blocks),
]


@pytest.mark.parametrize("name,mod,attr,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(monkeypatch, name, mod, attr, bad):
    monkeypatch.setattr(mod, attr, bad)
    assert not _pins_hold(), "planted mistake not caught: " + name
