"""Coefficient orders of the Walsh-Hadamard transform, on the CPU.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper computes the dyadic (Paley) order of eq. (1).  The same
coefficients are often wanted in two other orders:

  natural (Sylvester)  the Kronecker power of [[1, 1], [1, -1]]: entry (k, j)
                       is (-1)^popcount(k & j) (times 2^{-m/2});
  sequency (Walsh)     the rows sorted by their number of sign changes, so row
                       s changes sign s times.

Functions
---------
sylvester_matrix   natural-order matrix built as a Kronecker power.
sequency_matrix    the dyadic matrix of eq. (1) with its rows sorted by the
                   sign changes counted in each row (brute force, small m).
sign_changes       number of sign changes of every row of a matrix.
natural_from_dyadic, sequency_from_dyadic
                   reorder a dyadic-ordered result y (last axis): natural
                   coefficient k is dyadic bitrev_m(k); sequency coefficient s
                   is dyadic gray(s) = s ^ (s >> 1) (row p of eq. (1) has
                   invgray(p) sign changes).  These closed forms are what the
                   matrices above are checked against.
"""

import numpy as np

from .cascade import bitrev
from .dense import hadamard_paley


def sylvester_matrix(m, exact=False):
    h1 = np.array([[1, 1], [1, -1]], dtype=np.int64 if exact else np.float64)
    out = np.ones((1, 1), dtype=h1.dtype)
    for _ in range(m):
        out = np.kron(out, h1)
    return out if exact else out * 2.0 ** (-m / 2)


def sign_changes(mat):
    s = np.sign(mat)
    return np.sum(s[:, 1:] != s[:, :-1], axis=1)


def sequency_matrix(m, exact=False):
    h = hadamard_paley(m, exact)
    order = np.argsort(sign_changes(h), kind="stable")
    return h[order]


def gray(s):
    return s ^ (s >> 1)


def natural_from_dyadic(y):
    y = np.asarray(y)
    m = int(np.log2(y.shape[-1]))
    idx = np.array([bitrev(k, m) for k in range(1 << m)], dtype=np.int64)
    return y[..., idx]


def sequency_from_dyadic(y):
    y = np.asarray(y)
    n = y.shape[-1]
    idx = gray(np.arange(n, dtype=np.int64))
    return y[..., idx]
