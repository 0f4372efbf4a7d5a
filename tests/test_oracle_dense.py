"""Pins for the dense oracle matrices (eqs. 1-4), checked against facts the
paper and mathematics fix rather than against the oracle itself."""

import numpy as np
import pytest
import scipy.linalg

from oracle import cascade, dense


def test_hand_worked_matrices(golden_hand):
    # Hand derivations of eqs. (1)-(2) and Theorem 1's factor for m = 2, 3.
    assert np.array_equal(dense.hadamard_paley(2, exact=True), golden_hand["H2"])
    assert np.array_equal(dense.haar_matrix(2, exact=True), golden_hand["Psi2"])
    assert np.array_equal(dense.hadamard_paley(3, exact=True), golden_hand["H3"])
    assert np.array_equal(dense.haar_matrix(3, exact=True), golden_hand["Psi3"])
    assert np.array_equal(dense.theorem1_factor(3, 2, exact=True), golden_hand["F3_2"])


@pytest.mark.parametrize("m", range(0, 11))
def test_entries_and_shapes(m):
    h = dense.hadamard_paley(m, exact=True)
    p = dense.haar_matrix(m, exact=True)
    assert h.shape == p.shape == (1 << m, 1 << m)
    assert set(np.unique(h)) <= {-1, 1}
    assert set(np.unique(p)) <= {-1, 0, 1}
    # orthonormal form = unnormalized form scaled by 2^{-m/2} (eqs. 1-2)
    s = 2.0 ** (-m / 2.0)
    assert np.allclose(dense.hadamard_paley(m), s * h, atol=1e-13)
    # Haar rows of eq. (2) have support 2^m (scaling row) and 2^{m-j} at scale j
    if m >= 1:
        support = (p != 0).sum(axis=1)
        assert support[0] == 1 << m
        for j in range(m):
            assert np.all(support[1 << j:2 << j] == 1 << (m - j))


@pytest.mark.parametrize("m", range(1, 11))
def test_theorem1_exact_integer(m):
    # Theorem 1 (eq. 3) as an exact identity in the unnormalized integers.
    assert np.array_equal(dense.theorem1_rhs(m, exact=True),
                          dense.hadamard_paley(m, exact=True))


@pytest.mark.parametrize("m", range(1, 10))
def test_theorem1_float(m):
    err = np.max(np.abs(dense.theorem1_rhs(m) - dense.hadamard_paley(m)))
    assert err <= 1e-12


@pytest.mark.parametrize("m", range(2, 8))
def test_factor_block_pattern(m):
    # The expansion after Theorem 1: F_r is block diagonal with 2^{r-1} blocks
    # of 2^{m-r+1}; each block is identity on its first half and Psi_{m-r} on
    # its second half.
    n = 1 << m
    for r in range(1, m):
        f = dense.theorem1_factor(m, r, exact=True)
        big = 1 << (m - r + 1)
        half = big // 2
        psi = dense.haar_matrix(m - r, exact=True)
        expect = np.zeros((n, n), dtype=np.int64)
        for b in range(1 << (r - 1)):
            o = b * big
            expect[o:o + half, o:o + half] = np.eye(half, dtype=np.int64)
            expect[o + half:o + big, o + half:o + big] = psi
        assert np.array_equal(f, expect), (m, r)


@pytest.mark.parametrize("m", range(0, 10))
def test_orthogonality_symmetry_involution(m):
    h = dense.hadamard_paley(m)
    p = dense.haar_matrix(m)
    eye = np.eye(1 << m)
    assert np.allclose(h @ h.T, eye, atol=1e-12)
    assert np.allclose(p @ p.T, eye, atol=1e-12)
    assert np.allclose(h, h.T, atol=0)          # symmetric
    assert np.allclose(h @ h, eye, atol=1e-12)  # involution


@pytest.mark.parametrize("m", range(1, 10))
def test_haar_walsh_eq4(m):
    # eq. (4): H_m Psi_m^T = diag(1, H_0, H_1, ..., H_{m-1})
    lhs = dense.hadamard_paley(m) @ dense.haar_matrix(m).T
    assert np.allclose(lhs, dense.haar_walsh(m), atol=1e-12)


@pytest.mark.parametrize("m", range(0, 9))
def test_closed_form(m):
    assert np.array_equal(cascade.closed_form(m, exact=True),
                          dense.hadamard_paley(m, exact=True))


@pytest.mark.parametrize("m", range(0, 11))
def test_library_sylvester_bitreversed(m):
    # scipy's Sylvester (natural-order) Hadamard with its rows bit-reversed is
    # the dyadic-order matrix of eq. (1).
    syl = scipy.linalg.hadamard(1 << m).astype(np.int64)
    perm = [cascade.bitrev(i, m) for i in range(1 << m)]
    assert np.array_equal(syl[perm], dense.hadamard_paley(m, exact=True))
