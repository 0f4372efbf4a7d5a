"""Dense matrices of the CHW paper, built straight from its recursions.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Two numeric kinds are supported everywhere:
  exact=False -> float64, with the 1/sqrt(2) factor of each recursion step
                 (the orthonormal matrices of the paper);
  exact=True  -> int64, with every 1/sqrt(2) dropped.  The recursions then
                 give H'_m = 2^{m/2} H_m with entries +-1 and
                 Psi'_m = 2^{m/2} Psi_m with entries in {0, +-1}.  Because
                 the proof of Theorem 1 (Sec. 5) only ever uses the 1/sqrt(2)
                 as a common factor, Theorem 1 holds exactly for the primed
                 matrices (H'_m = {prod F'_r} Psi'_m), which gives the oracle an
                 exact integer identity to be pinned by.

Matrix sizes: everything here is O(4^m) memory; the tests stay at m <= 10.
"""

import numpy as np

_C = float(np.sqrt(0.5))  # correctly rounded 1/sqrt(2)


def _kind(exact):
    return (np.int64, 1) if exact else (np.float64, _C)


def identity(k, exact=False):
    """I_k: the 2^k x 2^k identity (notation of Sec. 2, after eq. 2)."""
    dt, _ = _kind(exact)
    return np.eye(1 << k, dtype=dt)


def hadamard_paley(m, exact=False):
    """H_m, the Hadamard matrix with columns in dyadic (Paley) order, eq. (1).

    H_0 = 1;  H_{k+1} = c [ H_k (x) (1  1) ; H_k (x) (1 -1) ],  c = 1/sqrt(2)
    (c = 1 in the exact form).
    """
    dt, c = _kind(exact)
    a = np.ones((1, 1), dtype=dt)
    plus = np.array([[1, 1]], dtype=dt)
    minus = np.array([[1, -1]], dtype=dt)
    for _ in range(m):
        top = np.kron(a, plus)
        bot = np.kron(a, minus)
        a = np.vstack([top, bot])
        if not exact:
            a = a * c
    return a


def haar_matrix(m, exact=False):
    """Psi_m, the Haar matrix, eq. (2).

    Psi_0 = 1;  Psi_{k+1} = c [ Psi_k (x) (1  1) ; I_k (x) (1 -1) ].
    Row order is coarse to fine (scaling row first, then the coarsest detail,
    ..., the 2^{m-1} finest details last).
    """
    dt, c = _kind(exact)
    a = np.ones((1, 1), dtype=dt)
    plus = np.array([[1, 1]], dtype=dt)
    minus = np.array([[1, -1]], dtype=dt)
    for k in range(m):
        top = np.kron(a, plus)
        bot = np.kron(identity(k, exact), minus)
        a = np.vstack([top, bot])
        if not exact:
            a = a * c
    return a


def block_diag(*blocks):
    """Block-diagonal matrix of square blocks (plain construction)."""
    n = sum(b.shape[0] for b in blocks)
    dt = np.result_type(*[b.dtype for b in blocks])
    out = np.zeros((n, n), dtype=dt)
    o = 0
    for b in blocks:
        k = b.shape[0]
        out[o:o + k, o:o + k] = b
        o += k
    return out


def theorem1_factor(m, r, exact=False):
    """F_r = I_{r-1} (x) diag(I_{m-r}, Psi_{m-r}), the r-th factor of eq. (3).

    Valid for 1 <= r <= m-1.  It splits a length-2^m vector into 2^{r-1}
    blocks of 2^{m-r+1}; inside each block the first half is left alone and
    Psi_{m-r} acts on the second half (the block pattern written out after
    Theorem 1 in Sec. 2).
    """
    if not 1 <= r <= m - 1:
        raise ValueError("factor index r must satisfy 1 <= r <= m-1")
    inner = block_diag(identity(m - r, exact), haar_matrix(m - r, exact))
    return np.kron(identity(r - 1, exact), inner)


def theorem1_rhs(m, exact=False):
    """Right-hand side of eq. (3): {F_{m-1} ... F_2 F_1} Psi_m.

    The product convention of Sec. 2 puts the r=1 factor rightmost, so Psi_m
    acts first, then F_1, then F_2, ...  For m = 1 the product is empty and
    the result is Psi_1 (the base case of the induction in Sec. 5).
    """
    if m < 1:
        raise ValueError("Theorem 1 is stated for m >= 1")
    acc = haar_matrix(m, exact)
    for r in range(1, m):
        acc = theorem1_factor(m, r, exact) @ acc
    return acc


def haar_walsh(m, exact=False):
    """diag(1, H_0, H_1, ..., H_{m-1}), the right-hand side of eq. (4).

    Eq. (4) states H_m Psi_m^T equals this matrix (orthonormal form only).
    """
    blocks = [np.ones((1, 1), dtype=_kind(exact)[0])]
    blocks += [hadamard_paley(k, exact) for k in range(m)]
    return block_diag(*blocks)
