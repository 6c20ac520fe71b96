"""Oracle: the block Wiedemann projection sequence.

Section 2.2 ("Coppersmith Block Wiedemann") defines the sequence of s x s
matrices X A^i Y for blocks X, Y of s vectors; Section 2.5 (step 2 of the
"Block Wiedemann Rank Algorithm") computes it on a preconditioned matrix for
i = 0 .. 2n/s + O(1); Section 2.3 notes the preconditioners of the form A^T A.
The matrix iterated here is

    B = D_c A^T D_r A D_c        (n x n, symmetric)

with D_r (m x m) and D_c (n x n) diagonal; D_c = identity gives the plain
A^T D A form.  The sequence is

    S_k = U^T B^k V   (mod p),   k = 0 .. L-1,

with U, V in GF(p)^{n x s}.  S_0 = U^T V counts as the first term, so L terms
take L-1 applications of B.

Everything here is exact integer arithmetic followed by a reduction mod p: a
product of sparse matrix and block (scipy's CSR product on int64) is exact as
long as the bound checked in ``_exact_bound_ok`` holds, and every other
product is reduced mod p before it is summed.  Larger values take the Python
big-integer path.

Parity pinned by: S_0 = U^T V; A = I gives S_k = U^T (D_c D_r D_c)^k V; A = 0
gives S_k = 0 for k >= 1; a one-row A = a gives
S_k = d^k (a D_c^2 a^T)^(k-1) (U^T D_c a^T)(a D_c V) for k >= 1; U = V gives
symmetric S_k; linearity in V; and a dense big-integer power of B.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr_mod(m, n, row_ptr, col_idx, val, p, signed=True):
    """CSR matrix with values as small signed integers (signed=True) or reduced to [0, p)."""
    v = np.asarray(val, dtype=np.int64)
    if not signed:
        v = v % p
    M = sp.csr_matrix((v, np.asarray(col_idx, dtype=np.int64), np.asarray(row_ptr, dtype=np.int64)),
                      shape=(m, n))
    M.sum_duplicates()
    return M


def _exact_bound_ok(M, p) -> bool:
    """True when |sum_j a_ij x_j| < 2^62 for every row and every x in [0, p)."""
    if M.nnz == 0:
        return True
    row_abs = np.asarray(abs(M).sum(axis=1)).ravel()
    return float(row_abs.max()) * float(p) < 2.0 ** 62


def _spmm_exact(M, X, p):
    """(M X) mod p for integer sparse M and a residue block X, by exact integer sums."""
    if _exact_bound_ok(M, p):
        Y = M @ X.astype(np.int64)
        return np.mod(Y, p).astype(np.int64)
    # big-integer path (slow; only for unusually large entries)
    Mc = M.tocsr()
    out = np.zeros((M.shape[0], X.shape[1]), dtype=np.int64)
    Xo = X.astype(object)
    for i in range(M.shape[0]):
        acc = [0] * X.shape[1]
        for t in range(Mc.indptr[i], Mc.indptr[i + 1]):
            a = int(Mc.data[t])
            row = Xo[Mc.indices[t]]
            for c in range(X.shape[1]):
                acc[c] += a * int(row[c])
        out[i] = [x % p for x in acc]
    return out


def _diag_scale(d, X, p):
    """diag(d) X mod p (each product below p^2 < 2^62)."""
    if d is None:
        return X
    return (np.asarray(d, dtype=np.int64)[:, None] * X) % p


def project(U, W, p):
    """U^T W mod p for U, W in [0, p)^{n x s}; every product is reduced before summing."""
    U = np.asarray(U, dtype=np.int64)
    W = np.asarray(W, dtype=np.int64)
    n, s = U.shape
    out = np.zeros((s, W.shape[1]), dtype=np.int64)
    step = max(1, (1 << 22) // max(1, s * W.shape[1]))
    for a in range(0, n, step):
        prod = (U[a:a + step, :, None] * W[a:a + step, None, :]) % p
        out = (out + prod.sum(axis=0)) % p
    return out


class Oracle:
    """Holds A (m x n) and the diagonals; applies B = D_c A^T D_r A D_c mod p."""

    def __init__(self, m, n, row_ptr, col_idx, val, p, d_row=None, d_col=None):
        self.m, self.n, self.p = int(m), int(n), int(p)
        self.A = _csr_mod(m, n, row_ptr, col_idx, val, p)
        self.At = self.A.T.tocsr()
        self.d_row = None if d_row is None else np.asarray(d_row, dtype=np.int64) % p
        self.d_col = None if d_col is None else np.asarray(d_col, dtype=np.int64) % p

    def half(self, X):
        """Y = D_r A X mod p (the first sparse product and the row scale)."""
        return _diag_scale(self.d_row, _spmm_exact(self.A, X, self.p), self.p)

    def apply(self, W):
        """B W mod p."""
        p = self.p
        X = _diag_scale(self.d_col, np.asarray(W, dtype=np.int64) % p, p)
        Y = self.half(X)
        Z = _spmm_exact(self.At, Y, p)
        return _diag_scale(self.d_col, Z, p)

    def sequence(self, U, V, L):
        """[S_0, ..., S_{L-1}] with S_k = U^T B^k V mod p, shape (L, s, s)."""
        p = self.p
        U = np.asarray(U, dtype=np.int64) % p
        W = np.asarray(V, dtype=np.int64) % p
        out = np.zeros((L, U.shape[1], W.shape[1]), dtype=np.int64)
        for k in range(L):
            if k:
                W = self.apply(W)
            out[k] = project(U, W, p)
        return out


def sequence(A, U, V, p, L, d_row=None, d_col=None):
    """S_k = U^T (D_c A^T D_r A D_c)^k V mod p for k < L, for a CSR-like A."""
    return Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, d_row, d_col).sequence(U, V, L)


def dense_B(A_dense, p, d_row=None, d_col=None):
    """B = D_c A^T D_r A D_c mod p as a dense Python-int matrix (tiny cases only)."""
    A = [[int(x) for x in row] for row in np.asarray(A_dense).tolist()]
    m = len(A)
    n = len(A[0]) if m else 0
    dr = [1] * m if d_row is None else [int(x) for x in d_row]
    dc = [1] * n if d_col is None else [int(x) for x in d_col]
    B = [[0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            B[i][j] = (dc[i] * dc[j] * sum(A[r][i] * dr[r] * A[r][j] for r in range(m))) % p
    return B


def dense_sequence(A_dense, U, V, p, L, d_row=None, d_col=None):
    """The same sequence from explicit big-integer powers of the dense B (tiny cases only)."""
    B = dense_B(A_dense, p, d_row, d_col)
    n = len(B)
    U = [[int(x) for x in r] for r in np.asarray(U).tolist()]
    V = [[int(x) for x in r] for r in np.asarray(V).tolist()]
    s = len(U[0]) if n else 0
    W = [row[:] for row in V]
    out = []
    for k in range(L):
        if k:
            W = [[sum(B[i][t] * W[t][c] for t in range(n)) % p for c in range(s)] for i in range(n)]
        out.append([[sum(U[t][a] * W[t][c] for t in range(n)) % p for c in range(s)] for a in range(s)])
    return np.array(out, dtype=np.int64).reshape(L, s, s)
