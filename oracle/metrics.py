"""Comparison metrics used to grade a transform result against the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

rel_l2: per signal ||y_hat - y||_2 / ||y||_2 in float64 (the absolute norm
||y_hat||_2 when ||y||_2 == 0).  The graded value is the maximum over the
signals of a batch; the pooled value (all signals concatenated) is also
reported.
"""

import numpy as np


def rel_l2(y_hat, y):
    """Per-signal relative L2 error along the last axis (float64)."""
    a = np.asarray(y_hat, dtype=np.float64)
    b = np.asarray(y, dtype=np.float64)
    diff = np.sqrt(np.sum((a - b) ** 2, axis=-1))
    ref = np.sqrt(np.sum(b ** 2, axis=-1))
    out = np.where(ref > 0, diff / np.where(ref > 0, ref, 1.0), diff)
    return out


def max_rel_l2(y_hat, y):
    return float(np.max(rel_l2(y_hat, y))) if np.size(y) else 0.0


def pooled_rel_l2(y_hat, y):
    a = np.asarray(y_hat, dtype=np.float64).ravel()
    b = np.asarray(y, dtype=np.float64).ravel()
    ref = np.sqrt(np.sum(b ** 2))
    diff = np.sqrt(np.sum((a - b) ** 2))
    return float(diff / ref) if ref > 0 else float(diff)


def exact_equal(y_hat, y):
    """Bit-exact integer comparison after widening both sides to int64."""
    return bool(np.array_equal(np.asarray(y_hat, dtype=np.int64),
                               np.asarray(y, dtype=np.int64)))
