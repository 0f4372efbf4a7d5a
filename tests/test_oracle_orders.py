"""Pins of oracle.orders: the natural and sequency orders from their
definitions (Kronecker power; rows sorted by sign changes) against the
dyadic matrix of eq. (1) and the closed-form reorderings."""

import numpy as np
import pytest
from scipy.linalg import hadamard

from oracle import cascade, dense, orders


@pytest.mark.parametrize("m", range(0, 8))
def test_sylvester_is_the_library_hadamard(m):
    assert np.array_equal(orders.sylvester_matrix(m, exact=True), hadamard(1 << m))


@pytest.mark.parametrize("m", range(1, 9))
def test_sequency_rows_have_s_sign_changes(m):
    w = orders.sequency_matrix(m, exact=True)
    assert np.array_equal(orders.sign_changes(w), np.arange(1 << m))


@pytest.mark.parametrize("m", range(1, 9))
def test_reorderings_match_the_matrices(m):
    h = dense.hadamard_paley(m, exact=True)
    # rows: natural row k = dyadic row bitrev(k); sequency row s = dyadic row gray(s)
    assert np.array_equal(orders.natural_from_dyadic(h.T).T, orders.sylvester_matrix(m, exact=True))
    assert np.array_equal(orders.sequency_from_dyadic(h.T).T, orders.sequency_matrix(m, exact=True))


@pytest.mark.parametrize("m", [3, 6, 10])
def test_ordered_transforms_of_a_vector(m):
    x = np.arange(1, (1 << m) + 1, dtype=np.int64) * 7 % 23 - 11
    y = cascade.chw_forward(x)
    n = 1 << m
    if n <= 256:
        assert np.array_equal(orders.natural_from_dyadic(y), orders.sylvester_matrix(m, True) @ x)
        assert np.array_equal(orders.sequency_from_dyadic(y), orders.sequency_matrix(m, True) @ x)
    # both are permutations of the dyadic coefficients
    assert np.array_equal(np.sort(orders.natural_from_dyadic(y)), np.sort(y))
    assert np.array_equal(np.sort(orders.sequency_from_dyadic(y)), np.sort(y))


def test_planted_order_mistakes_are_caught():
    m = 5
    h = dense.hadamard_paley(m, exact=True)
    wrong_nat = h  # dyadic taken for natural
    wrong_seq = h[[orders.gray(s) ^ 1 if s else 0 for s in range(1 << m)]]
    assert not np.array_equal(wrong_nat, orders.sylvester_matrix(m, True))
    assert not np.array_equal(orders.sign_changes(wrong_seq), np.arange(1 << m))
