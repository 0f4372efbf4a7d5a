"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no part of the transform's arithmetic: it only draws
random numbers and lays signals out in memory.  Both the CPU oracle and the
GPU path receive the same arrays from here.

Recipe (all inputs are synthetic; the paper has no datasets):
  * per-signal streams ``numpy.random.default_rng([seed, i])`` so any single
    signal i can be regenerated alone;
  * float32 values ``standard_normal(n, dtype=float32)``;
  * integer values uniform in [-128, 127], both ends inclusive;
  * the precision workload: N(0,1) float32, then an independent
    Bernoulli(0.01) mask per element (same stream) whose elements are scaled
    by 100, then rounded to bfloat16 / float16 with round-to-nearest-even
    (torch's CPU conversion);
  * the ragged workload: 20000 log2 sizes drawn uniform in [6, 20] under a
    total budget of 2^30 elements (sequential budgeted draw, see
    ``ragged_log2_sizes``), packed back to back by int64 offsets;
  * the differentiation workload: a shared random +-1 diagonal;
  * the randomized (signed) form: k diagonals of +-1 entries (p = 1/2), round
    r from the stream [seed, r], packed into uint32 sign bits for the GPU
    (bit b of a round is bit b % 32 of word b // 32, set for -1).
"""

from .synth import (  # noqa: F401
    CONFIGS,
    Workload,
    float_signals,
    int_signals,
    outlier_signals,
    packed_offsets,
    ragged_log2_sizes,
    ragged_values,
    expand_shared_signs,
    pack_sign_bits,
    sign_diagonal,
    sign_rounds,
    to_half_precision,
)
