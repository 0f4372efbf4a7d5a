"""Pins of the oracle's Philox4x64-10 sign generator against numpy's own
Philox bit generator (numpy.random.Philox is Philox4x64-10: its raw output
after counter c is the block of counter c + 1)."""

import numpy as np
import pytest

import workloads
from oracle import philox

M64 = (1 << 64) - 1


def _dec(counter):
    """counter - 1 over the four 64-bit words (borrow upwards)."""
    c = [int(v) for v in counter]
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = M64
    return c


def _numpy_blocks(counter, key, nblocks):
    bg = np.random.Philox(counter=np.array(_dec(counter), dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4 * nblocks)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 0, 0), (123, 0)),
    ((M64, 3, 9, 1), (2**63 + 5, 77)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
    ((M64, M64, M64, M64), (M64, M64)),
])
def test_block_matches_numpy_philox(counter, key):
    got = philox.philox4x64_10(counter, key)
    want = tuple(int(v) for v in _numpy_blocks(counter, key, 1))
    assert got == want


def test_random_counters_match_numpy():
    rng = np.random.default_rng(77)
    for _ in range(50):
        c = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        k = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert philox.philox4x64_10(c, k) == tuple(int(v) for v in _numpy_blocks(c, k, 1))


@pytest.mark.parametrize("seed,rounds,words", [(0, 1, 8), (1, 3, 61), (2**64 - 1, 2, 5),
                                               (987654321, 2, 1000)])
def test_sign_words_match_numpy_stream(seed, rounds, words):
    """A round's words are numpy's raw stream from block (0, r, 0, 0) on,
    each 64-bit output split low half first."""
    got = philox.sign_words(seed, rounds, words)
    nblocks = (words + 7) // 8
    for r in range(rounds):
        raw = _numpy_blocks((0, r, 0, 0), (seed, 0), nblocks).astype("<u8")
        want = raw.view("<u4")[:words]
        np.testing.assert_array_equal(got[r], want)


def test_diagonals_invert_the_packing():
    d = workloads.sign_rounds(4242, 3, 1000)
    np.testing.assert_array_equal(philox.diagonals(workloads.pack_sign_bits(d), 1000), d)


def test_signs_are_balanced():
    n = 1 << 16
    d = philox.diagonals(philox.sign_words(31337, 2, n // 32), n)
    frac = (d < 0).mean(axis=1)
    # 6 standard deviations of a fair coin over n draws
    assert np.all(np.abs(frac - 0.5) < 6 * 0.5 / np.sqrt(n))
    # the rounds differ
    assert (d[0] != d[1]).mean() > 0.45


def _pins_hold(fn):
    for c, k in [((5, 7, 0, 0), (123, 0)), ((M64, 3, 9, 1), (2**63 + 5, 77))]:
        if fn(c, k) != tuple(int(v) for v in _numpy_blocks(c, k, 1)):
            return False
    return True


def _swapped_multipliers(counter, key):
    saved = philox.M0, philox.M1
    philox.M0, philox.M1 = saved[1], saved[0]
    try:
        return philox.philox4x64_10(counter, key)
    finally:
        philox.M0, philox.M1 = saved


def _no_key_bump(counter, key):
    saved = philox.W0, philox.W1
    philox.W0, philox.W1 = 0, 0
    try:
        return philox.philox4x64_10(counter, key)
    finally:
        philox.W0, philox.W1 = saved


def _outputs_permuted(counter, key):
    o = philox.philox4x64_10(counter, key)
    return (o[2], o[1], o[0], o[3])


def test_philox_pins_hold_unmutated():
    assert _pins_hold(philox.philox4x64_10)


@pytest.mark.parametrize("fn", [_swapped_multipliers, _no_key_bump, _outputs_permuted])
def test_philox_planted_mistakes_are_caught(fn):
    assert not _pins_hold(fn)
