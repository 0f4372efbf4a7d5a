"""Randomized Hadamard transform with random-sign diagonals, on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Not a passage of the paper: this is the form in which the transform is used
for sketching and random rotations,

    y = H D_k ... H D_2 H D_1 x,        D_r = diag(d_r),  d_r in {+1, -1}^n,

each H being the CHW transform of Sec. 2 / eq. (3) (oracle.cascade), applied
to the elementwise product of the round's diagonal with the previous round's
output (x for the first round).  The adjoint is the transpose of that product:

    D_1 H^T D_2 H^T ... D_k H^T g.

Float input runs in float64 (orthonormal H), integer input in int64 (H'),
exactly as oracle.cascade does; the sign flips are exact in both.

Functions
---------
signed_forward   y for one batch of equal-size signals (shape (..., 2^m)).
signed_adjoint   the adjoint of signed_forward.
signed_batch     the same on a flat buffer of ragged signals (offsets), with
                 the plain-C cascade of oracle.c_oracle doing each round.
"""

import numpy as np

from . import c_oracle
from .cascade import chw_adjoint, chw_forward


def _check_signs(d, n):
    d = np.asarray(d)
    if d.shape[-1] != n or not np.all(np.abs(d) == 1):
        raise ValueError("a diagonal must hold n entries of +1 / -1")
    return d


def signed_forward(x, diagonals, exact=None):
    """H D_k ... H D_1 x; diagonals = [d_1, ..., d_k] (each broadcast over the
    batch dimensions of x)."""
    v = x
    for d in diagonals:
        d = _check_signs(d, np.shape(x)[-1])
        v = chw_forward(np.asarray(v) * d.astype(np.asarray(v).dtype), exact)
    return v


def signed_adjoint(g, diagonals, exact=None):
    """D_1 H^T D_2 H^T ... D_k H^T g (the rounds in reverse order)."""
    v = g
    for d in reversed(list(diagonals)):
        d = _check_signs(d, np.shape(g)[-1])
        w = chw_adjoint(v, exact)
        v = w * d.astype(w.dtype)
    return v


def signed_batch(x_flat, log2_sizes, diagonals_flat, offsets=None, adjoint=False,
                 threads=8):
    """Rounds of the signed transform on a flat buffer of ragged signals.

    x_flat          float64 or int64 buffer holding signal i at
                    [offsets[i], offsets[i] + 2^{m_i}) (offsets: the batch's
                    start offsets; packed back to back if None).
    diagonals_flat  list of k arrays of +1 / -1 over the same buffer: entry e
                    is the sign of buffer element e in that round.
    Elements outside every signal carry no meaning in the result.
    """
    v = np.asarray(x_flat)
    diags = [np.asarray(d).astype(v.dtype) for d in diagonals_flat]
    order = list(reversed(diags)) if adjoint else diags
    for d in order:
        if adjoint:
            v = c_oracle.chw_batch(v, log2_sizes, offsets, adjoint=True, threads=threads) * d
        else:
            v = c_oracle.chw_batch(v * d, log2_sizes, offsets, adjoint=False, threads=threads)
    return v
