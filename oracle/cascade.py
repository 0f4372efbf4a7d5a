"""The CHW cascade on the CPU, in the order the paper gives it.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Arrays are batches: shape (..., n) with n = 2^m; every signal of the batch is
transformed independently.  Float input is promoted exactly to float64 and
the orthonormal transform is computed with a 1/sqrt(2) per Haar level, as the
recursions of eqs. (1)-(2) carry it.  Integer input is promoted to int64 and
the unnormalized transform (every 1/sqrt(2) dropped) is computed exactly.

Functions
---------
chw_forward       literal cascade: Psi_m, then F_1, ..., F_{m-1} (Sec. 2,
                  eq. 3), identity blocks not performed.
chw_adjoint       H_m^T: transposed factors in reverse order, then Psi_m^T.
haar_forward      Psi_k on a slice (the building block; Lemma 1).
haar_adjoint      Psi_k^T on a slice (Haar synthesis).
count_ops         add/sub counter of the literal cascade (Lemma 1, Thm. 2).
cascade_schedule  the list of Haar transforms the cascade applies.
closed_form       entries of H_m from the popcount formula (independent).
radix2_paley      textbook in-place radix-2 WHT (natural order) followed by
                  the bit-reversal permutation to dyadic order (independent).
coefficient       one output y_i of H_m x from the popcount formula, O(n), for
                  signals too large for the cascade to be run in a test.
"""

import numpy as np

_C = float(np.sqrt(0.5))  # correctly rounded 1/sqrt(2)


# --------------------------------------------------------------------------
# helpers

def log2_exact(n):
    """m with n == 2^m, or ValueError."""
    n = int(n)
    if n < 1 or (n & (n - 1)) != 0:
        raise ValueError("signal length must be a power of two, got %d" % n)
    return n.bit_length() - 1


def _promote(x, exact):
    x = np.asarray(x)
    if exact:
        if not np.issubdtype(x.dtype, np.integer):
            raise TypeError("the unnormalized integer form needs integer input")
        return x.astype(np.int64, copy=True)
    return x.astype(np.float64, copy=True)


def _is_exact(x, exact):
    if exact is None:
        return np.issubdtype(np.asarray(x).dtype, np.integer)
    return bool(exact)


class OpCounter:
    """Counts additions and subtractions (the paper's 'operations').

    The 1/sqrt(2) scalings are not counted: Lemma 1's 2(2^m - 1) is exactly
    the number of sums and differences of the Haar pyramid.
    """

    def __init__(self):
        self.adds = 0

    def add(self, k):
        self.adds += int(k)


# --------------------------------------------------------------------------
# the Haar building block, eq. (2) read as an algorithm

def haar_level(v, lo, length, c, counter=None):
    """One level of the Haar transform on v[..., lo:lo+length].

    Pairs (x_{2p}, x_{2p+1}) become the scaled sum and difference; sums go to
    the lower half, differences to the upper half.  This is one step of the
    recursion of eq. (2): the first block row Psi_k (x) (1 1) takes pairwise
    sums, the second block row I_k (x) (1 -1) takes pairwise differences
    (first minus second).
    """
    half = length // 2
    a = v[..., lo:lo + length:2].copy()
    b = v[..., lo + 1:lo + length:2].copy()
    s = a + b
    d = a - b
    if c != 1:
        s = s * c
        d = d * c
    v[..., lo:lo + half] = s
    v[..., lo + half:lo + length] = d
    if counter is not None:
        counter.add(2 * half * _nsig(v))


def haar_forward(v, lo, length, c, counter=None):
    """Psi_k on v[..., lo:lo+length] (length = 2^k), in place.

    Unrolling eq. (2): Psi_{k} = diag(Psi_{k-1}, I_{k-1}) . (level on all 2^k)
    so the levels run on a shrinking block of sums: 2^k, 2^{k-1}, ..., 2.
    Output order: scaling coefficient, coarsest detail, ..., finest details.
    """
    while length >= 2:
        haar_level(v, lo, length, c, counter)
        length //= 2


def haar_adjoint(v, lo, length, c, counter=None):
    """Psi_k^T on v[..., lo:lo+length] (Haar synthesis), in place.

    Transpose of eq. (2): Psi_{k+1}^T [s; d] = c (Psi_k^T s (x) (1,1)^T
    + d (x) (1,-1)^T), i.e. out[2p] = c((Psi_k^T s)[p] + d[p]) and
    out[2p+1] = c((Psi_k^T s)[p] - d[p]).  Synthesis therefore runs from the
    coarsest scale (h = 1) to the finest (h = length/2).
    """
    h = 1
    while h < length:
        a = v[..., lo:lo + h].copy()
        d = v[..., lo + h:lo + 2 * h].copy()
        s = a + d
        t = a - d
        if c != 1:
            s = s * c
            t = t * c
        v[..., lo:lo + 2 * h:2] = s
        v[..., lo + 1:lo + 2 * h:2] = t
        if counter is not None:
            counter.add(2 * h * _nsig(v))
        h *= 2


def _nsig(v):
    return int(np.prod(v.shape[:-1])) if v.ndim > 1 else 1


# --------------------------------------------------------------------------
# the cascade, Theorem 1 / eq. (3)

def cascade_schedule(m):
    """Haar transforms applied by the CHW cascade, in execution order.

    Returns a list of (factor, offset, size): factor 0 is Psi_m on the whole
    vector; factor r (1 <= r <= m-1) is F_r = I_{r-1} (x) diag(I_{m-r},
    Psi_{m-r}): for each of its 2^{r-1} blocks of B = 2^{m-r+1} elements,
    Psi_{m-r} acts on the second half [bB + B/2, bB + B).  The identity
    halves are not performed (Sec. 2).
    """
    n = 1 << m
    sched = [(0, 0, n)] if m >= 1 else []
    for r in range(1, m):
        big = 1 << (m - r + 1)
        for b in range(1 << (r - 1)):
            sched.append((r, b * big + big // 2, big // 2))
    return sched


def chw_forward(x, exact=None, counter=None):
    """y = H_m x by the Cascading Haar Wavelet algorithm (Sec. 2, eq. 3).

    exact=None picks the integer form for integer input.  Float: y = H_m x
    (orthonormal, eq. 1).  Integer: y = H'_m x in int64 (every 1/sqrt(2)
    dropped; Theorem 1 still holds exactly).  m = 0 is the identity
    (H_0 = 1).
    """
    ex = _is_exact(x, exact)
    v = _promote(x, ex)
    m = log2_exact(v.shape[-1])
    c = 1 if ex else _C
    for _factor, lo, size in cascade_schedule(m):
        haar_forward(v, lo, size, c, counter)
    return v


def chw_adjoint(g, exact=None, counter=None):
    """H_m^T g: the transposed factors of eq. (3) in reverse order.

    H_m^T = Psi_m^T F_1^T ... F_{m-1}^T, so F_{m-1}^T acts first and Psi_m^T
    last; each F_r^T applies Psi_{m-r}^T (synthesis) on the same blocks that
    F_r used.
    """
    ex = _is_exact(g, exact)
    v = _promote(g, ex)
    m = log2_exact(v.shape[-1])
    c = 1 if ex else _C
    for _factor, lo, size in reversed(cascade_schedule(m)):
        haar_adjoint(v, lo, size, c, counter)
    return v


def count_ops(m):
    """Number of add/sub operations of the literal cascade for one signal."""
    ctr = OpCounter()
    chw_forward(np.zeros(1 << m, dtype=np.int64), exact=True, counter=ctr)
    return ctr.adds


# --------------------------------------------------------------------------
# independent cross-checks (not the paper's algorithm)

def bitrev(i, m):
    """Reverse the low m bits of the integer i."""
    r = 0
    for _ in range(m):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def closed_form(m, exact=False):
    """H_m[i, j] = 2^{-m/2} (-1)^{popcount(bitrev_m(i) & j)}.

    A closed form of eq. (1): each recursion step of eq. (1) pairs the new
    most significant row bit with the new least significant column bit, so the
    row index enters bit-reversed.  Built entry by entry, O(4^m).
    """
    n = 1 << m
    out = np.empty((n, n), dtype=np.int64)
    for i in range(n):
        ri = bitrev(i, m)
        for j in range(n):
            out[i, j] = -1 if bin(ri & j).count("1") & 1 else 1
    if exact:
        return out
    return out.astype(np.float64) * (2.0 ** (-m / 2.0))


def coefficient(x, i, exact=None, chunk=1 << 22):
    """y_i = sum_j H_m[i, j] x_j with the entries of closed_form:
    2^{-m/2} (-1)^{popcount(bitrev_m(i) & j)} (float, in float64), or the
    +-1 entries summed exactly in int64 (integer input).  One row of eq. (1)
    in O(n) time and O(chunk) memory, for single outputs of large signals."""
    x = np.asarray(x).reshape(-1)
    n = x.shape[0]
    m = log2_exact(n)
    ex = _is_exact(x, exact)
    r = np.int64(bitrev(int(i), m))
    acc = 0 if ex else 0.0
    for lo in range(0, n, chunk):
        j = np.arange(lo, min(n, lo + chunk), dtype=np.int64)
        neg = (np.bitwise_count(j & r) & 1).astype(bool)
        v = x[lo:lo + j.shape[0]]
        v = v.astype(np.int64) if ex else v.astype(np.float64)
        acc += v[~neg].sum() - v[neg].sum()
    if ex:
        return int(acc)
    return float(acc) * 2.0 ** (-m / 2.0)


def radix2_paley(x, exact=None):
    """Textbook in-place radix-2 WHT, then reorder natural -> dyadic.

    The butterflies run over index bits t = 0, 1, ..., m-1 (stride 1, 2, 4,
    ...), the element with bit t clear receiving the sum; the result is in
    natural (Sylvester) order and is read at bit-reversed positions to give
    the dyadic order: y[i] = nat[bitrev_m(i)].
    """
    ex = _is_exact(x, exact)
    v = _promote(x, ex)
    n = v.shape[-1]
    m = log2_exact(n)
    c = 1 if ex else _C
    h = 1
    while h < n:
        w = v.reshape(v.shape[:-1] + (n // (2 * h), 2, h))
        a = w[..., 0, :].copy()
        b = w[..., 1, :].copy()
        s = a + b
        d = a - b
        if c != 1:
            s = s * c
            d = d * c
        w[..., 0, :] = s
        w[..., 1, :] = d
        v = w.reshape(v.shape)
        h *= 2
    perm = np.array([bitrev(i, m) for i in range(n)], dtype=np.int64)
    return v[..., perm]
