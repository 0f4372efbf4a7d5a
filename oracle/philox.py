"""Philox4x64-10 random signs, on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not a passage of the paper: the random-sign diagonals of the randomized form
(oracle.signed) are drawn from the counter-based generator Philox4x64-10 of
J. Salmon, M. Moraes, R. Dror and D. Shaw ("Parallel random numbers: as easy
as 1, 2, 3", SC 2011), written here from that definition with plain Python
integers:

    a round maps the counter block (c0, c1, c2, c3) under key (k0, k1) to
        (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0)),
    where hi / lo are the upper / lower 64 bits of the 128-bit product; the key
    is bumped by the Weyl increments (W0, W1) after every round; ten rounds.

Sign words: word w of round r is 32-bit word (w mod 8) of the block with
counter (w // 8, r, 0, 0) and key (seed, 0), the block's outputs o_0..o_3
giving words 2i (low half of o_i) and 2i + 1 (high half).  Bit b of a round
(bit b % 32 of word b // 32) set means the sign -1.
"""

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
_MASK = (1 << 64) - 1


def philox4x64_10(counter, key):
    """One Philox4x64-10 block: four 64-bit counter words, two key words ->
    four 64-bit outputs."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> 64) ^ c3 ^ k1, p0 & _MASK)
        k0 = (k0 + W0) & _MASK
        k1 = (k1 + W1) & _MASK
    return c0, c1, c2, c3


def sign_words(seed, rounds, words):
    """uint32 array (rounds, words) of packed sign bits."""
    out = np.zeros((rounds, words), dtype=np.uint32)
    for r in range(rounds):
        for g in range((words + 7) // 8):
            o = philox4x64_10((g, r, 0, 0), (seed, 0))
            for i in range(8):
                w = 8 * g + i
                if w < words:
                    out[r, w] = (o[i // 2] >> (32 * (i % 2))) & 0xFFFFFFFF
    return out


def diagonals(words, n):
    """The +1 / -1 diagonals (int8, shape (rounds, n)) that packed sign words
    describe: entry b is -1 where bit b % 32 of word b // 32 is set."""
    words = np.atleast_2d(np.asarray(words, dtype=np.uint32))
    b = np.arange(n)
    bits = (words[:, b // 32] >> (b % 32).astype(np.uint32)) & 1
    return np.where(bits == 1, -1, 1).astype(np.int8)
