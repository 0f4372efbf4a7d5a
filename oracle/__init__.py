"""CPU oracle for the Cascading Haar Wavelet (CHW) Walsh-Hadamard transform.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
CPU statement of what the CHW method computes, written from the paper
(A. Thompson, "The Cascading Haar Wavelet algorithm for computing the
Walsh-Hadamard Transform").  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import, call or link anything here.
The GPU library never depends on it, and it shares no code, header, table or
helper with the GPU library.

Arithmetic is FP64 for the orthonormal (float) forms and int64 for the
unnormalized integer form.

Modules
-------
dense    -- dense matrices: H_m (eq. 1), Psi_m (eq. 2), the factors of
            Theorem 1 (eq. 3) and the Haar-Walsh matrix (eq. 4).
cascade  -- the CHW cascade itself (Sec. 2), its adjoint (transpose of
            eq. 3), the operation counter (Lemma 1, Theorem 2) and the
            independent cross-checks (closed form, textbook radix-2 WHT).
metrics  -- relative-L2 and exactness comparisons.
c_oracle -- ctypes loader for the plain-C cascade in chw_oracle.c (same
            algorithm, used where Python is too slow: large parity samples
            and the CPU baseline timing).
orders   -- the natural (Sylvester) and sequency (Walsh) coefficient orders
            from their definitions, and the reorderings of the dyadic result.
signed   -- the randomized form y = H D_k ... H D_1 x with random-sign
            diagonals and its adjoint (not in the paper; each round is the
            cascade above applied to a sign-flipped vector).
philox   -- Philox4x64-10 random-sign words (a published counter-based
            generator, not the paper's), as the device generates them.

Every function names the passage of the paper it follows.  Nothing here is
"parity unpinned": each function is pinned by tests marked ``not gpu`` against
facts the paper or mathematics fixes (hand-worked examples under
tests/golden, Theorem 1 as an exact integer identity, eq. 4, the closed
form of the Paley-ordered Hadamard matrix, the library Sylvester matrix,
Lemma 1 / Theorem 2 counts, orthogonality, Parseval and involution).
"""

from . import dense, cascade, metrics, orders, philox, signed  # noqa: F401
