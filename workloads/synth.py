"""Seeded synthetic signal generators (no transform arithmetic here)."""

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
import os

import numpy as np


def _rng(seed, i):
    return np.random.default_rng([int(seed), int(i)])


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def float_signals(seed, batch, m, first=0, out=None):
    """(batch, 2^m) float32, row b drawn N(0,1) from stream [seed, first + b]."""
    n = 1 << m
    if out is None:
        out = np.empty((batch, n), dtype=np.float32)

    def fill(b):
        out[b] = _rng(seed, first + b).standard_normal(n, dtype=np.float32)

    if batch * n >= (1 << 22):
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(batch)))
    else:
        for b in range(batch):
            fill(b)
    return out


def int_signals(seed, batch, m, first=0, lo=-128, hi=127):
    """(batch, 2^m) int32, uniform integers in [lo, hi] (both inclusive)."""
    n = 1 << m
    out = np.empty((batch, n), dtype=np.int32)
    for b in range(batch):
        out[b] = _rng(seed, first + b).integers(lo, hi + 1, size=n, dtype=np.int32)
    return out


def outlier_signals(seed, batch, m, first=0, p=0.01, scale=100.0):
    """(batch, 2^m) float32: N(0,1), then an independent Bernoulli(p) mask per
    element (drawn after the values, same stream) whose elements are x scale."""
    n = 1 << m
    out = np.empty((batch, n), dtype=np.float32)
    for b in range(batch):
        g = _rng(seed, first + b)
        v = g.standard_normal(n, dtype=np.float32)
        mask = g.random(n) < p
        v[mask] *= np.float32(scale)
        out[b] = v
    return out


def to_half_precision(x, dtype):
    """Round float32 values to 'bf16' or 'f16' with round-to-nearest-even.

    Returns a torch CPU tensor of that dtype (torch's CPU conversion rounds to
    nearest even)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    return t.to(torch.bfloat16 if dtype == "bf16" else torch.float16)


def ragged_log2_sizes(seed=4001, count=20000, budget=1 << 30, lo=6, hi=20):
    """Sequential budgeted draw of log2 sizes uniform in [lo, hi].

    Each size is drawn U{lo..hi}; if it would leave too little room for the
    remaining signals at the smallest size, it is redrawn uniformly from the
    sizes that still fit.  The list is then shuffled.  Every size in [lo, hi]
    can occur, all `count` signals are kept and the total stays <= budget.
    """
    g = np.random.default_rng(int(seed))
    total = 0
    ks = []
    for i in range(count):
        k = int(g.integers(lo, hi + 1))
        reserve = (1 << lo) * (count - i - 1)
        if total + (1 << k) + reserve > budget:
            room = budget - total - reserve
            top = min(hi, room.bit_length() - 1)
            if top < lo:
                raise ValueError("budget too small for the remaining signals")
            k = int(g.integers(lo, top + 1))
        total += 1 << k
        ks.append(k)
    perm = g.permutation(count)
    return np.asarray(ks, dtype=np.int32)[perm]


def packed_offsets(log2_sizes):
    """int64 offsets[batch + 1]: exclusive prefix sum of 2^m_i (back to back)."""
    sizes = np.left_shift(np.int64(1), np.asarray(log2_sizes, dtype=np.int64))
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    return off


def ragged_values(seed, log2_sizes, offsets=None, fill=0.0):
    """Flat float32 buffer with signal i drawn N(0,1) from stream [seed, i].

    Elements outside every signal (gaps) are set to `fill`."""
    log2_sizes = np.asarray(log2_sizes)
    if offsets is None:
        offsets = packed_offsets(log2_sizes)
    total = int(offsets[-1]) if len(offsets) > len(log2_sizes) else \
        int(offsets[-1] + (1 << int(log2_sizes[-1])))
    out = np.full(total, fill, dtype=np.float32)

    def fillsig(i):
        n = 1 << int(log2_sizes[i])
        o = int(offsets[i])
        out[o:o + n] = _rng(seed, i).standard_normal(n, dtype=np.float32)

    if total >= (1 << 22):
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fillsig, range(len(log2_sizes))))
    else:
        for i in range(len(log2_sizes)):
            fillsig(i)
    return out


def sign_diagonal(seed, n):
    """Random +-1 diagonal of length n (p = 1/2 each), float32."""
    g = np.random.default_rng(int(seed))
    return np.where(g.random(n) < 0.5, -1.0, 1.0).astype(np.float32)


def sign_rounds(seed, rounds, n):
    """`rounds` random +-1 diagonals of length n (p = 1/2 each), int8; round r
    draws from the stream [seed, r] (round 0 with rounds = 1 equals nothing
    else in this module)."""
    out = np.empty((rounds, n), dtype=np.int8)
    for r in range(rounds):
        out[r] = np.where(_rng(seed, r).random(n) < 0.5, -1, 1)
    return out


def pack_sign_bits(d):
    """Pack +-1 entries (last axis) into uint32 words, the layout the GPU
    library reads: bit b is bit b % 32 of word b // 32, set where the entry
    is -1.  Rows (rounds) stay separate: shape (..., ceil(n / 32))."""
    d = np.asarray(d)
    n = d.shape[-1]
    words = (n + 31) // 32
    bits = np.zeros(d.shape[:-1] + (words * 32,), dtype=np.uint8)
    bits[..., :n] = (d < 0)
    packed = np.packbits(bits.reshape(d.shape[:-1] + (words, 4, 8)), axis=-1,
                         bitorder="little")
    return packed.reshape(d.shape[:-1] + (words, 4)).view(np.uint32).reshape(d.shape[:-1] + (words,))


def expand_shared_signs(d_shared, log2_sizes, offsets=None, extent=None):
    """Per-element +-1 array over a buffer from one diagonal shared by every
    signal (signal i takes entries 0 .. 2^{m_i} - 1); gaps get +1."""
    sizes = np.asarray(log2_sizes, dtype=np.int64)
    if offsets is None:
        offsets = packed_offsets(sizes)
    offsets = np.asarray(offsets, dtype=np.int64)
    extent = int(offsets[-1]) if extent is None else extent
    d_shared = np.asarray(d_shared)
    out = np.ones(d_shared.shape[:-1] + (extent,), dtype=d_shared.dtype)
    for i, k in enumerate(sizes):
        n = 1 << int(k)
        out[..., offsets[i]:offsets[i] + n] = d_shared[..., :n]
    return out


@dataclass
class Workload:
    """A named synthetic workload (shapes of the paper's setting)."""
    name: str
    dtype: str            # 'f32', 'bf16', 'f16', 'i32', 'f64'
    norm: str             # 'ortho' or 'none'
    log2_sizes: list = field(default_factory=list)  # per signal (uniform: one value)
    batch: int = 0
    seed: int = 0
    note: str = ""


# The workloads the library is measured and tested on.
CONFIGS = {
    "plain_small_f32": Workload("plain_small_f32", "f32", "ortho", [10], 64, 1001,
                                "64 x 2^10 float32 N(0,1), orthonormal"),
    "plain_small_i32": Workload("plain_small_i32", "i32", "none", [10], 64, 1002,
                                "64 x 2^10 int32 uniform [-128,127], unnormalized"),
    "plain_2p20_f32": Workload("plain_2p20_f32", "f32", "ortho", [20], 1024, 2001,
                               "1024 x 2^20 float32 N(0,1), orthonormal"),
    "plain_2p24_f32": Workload("plain_2p24_f32", "f32", "ortho", [24], 16, 2002,
                               "16 x 2^24 float32 N(0,1), orthonormal"),
    "precision_bf16": Workload("precision_bf16", "bf16", "ortho", [12], 8192, 3001,
                               "8192 x 2^12, N(0,1) + 1% x100 outliers, RNE to bf16"),
    "precision_f16": Workload("precision_f16", "f16", "ortho", [12], 8192, 3001,
                              "8192 x 2^12, N(0,1) + 1% x100 outliers, RNE to f16"),
    "ragged_f32": Workload("ragged_f32", "f32", "ortho", [], 20000, 4002,
                           "20000 signals, log2 sizes U[6,20] budgeted to 2^30"),
    "ragged_bf16": Workload("ragged_bf16", "bf16", "ortho", [], 20000, 4002,
                            "ragged sizes as ragged_f32, values RNE to bf16"),
    "diff_f32": Workload("diff_f32", "f32", "ortho", [14], 256, 5001,
                         "y = H D x, 256 x 2^14 float32, D seeded +-1"),
    "gradcheck_f64": Workload("gradcheck_f64", "f64", "ortho", [6], 4, 5004,
                              "gradcheck in float64, 4 x 2^6"),
}
