"""Rank by Gaussian elimination: the plain definition of what the block
Wiedemann rank algorithm (Section 2.5, "Block Wiedemann Rank Algorithm")
returns with high probability.

* ``rank_sparse_modp``: sparse elimination over GF(p); every arithmetic step is
  a fresh ``% p``.  Pivot choice: shortest remaining row, then within it the
  column held by the fewest remaining rows (ties: smallest index).  The pivot
  order changes only the running time, never the rank.
* ``rank_dense_modp``: textbook dense row reduction over GF(p).
* ``rank_bareiss``: fraction-free Bareiss elimination over Z (exact big
  integers), giving the rank over Q.  rank_Q >= rank_p, with equality unless p
  divides every non-zero maximal minor.
* ``rank_over_integers``: the largest rank modulo several primes (Section 2.5:
  the rank over the integers, probabilistically, from a few random primes).

Parity pinned by: Bareiss vs dense vs sparse on random tiny matrices at two
primes, planted ranks, rank A = rank A^T <= min(m, n), invariance under
permutations and unit scalings, special cases (0, identity, entries = p,
a single non-zero row), and matrices whose determinant is a known multiple of p.
"""
from __future__ import annotations

import heapq

import numpy as np


def _rows_from_csr(m, row_ptr, col_idx, val, p):
    rows = []
    for i in range(m):
        d = {}
        for t in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            c = int(col_idx[t])
            d[c] = (d.get(c, 0) + int(val[t])) % p
        rows.append({c: v for c, v in d.items() if v})
    return rows


def rank_sparse_modp(m: int, n: int, row_ptr, col_idx, val, p: int) -> int:
    """Rank of the m x n CSR matrix over GF(p) by sparse Gaussian elimination."""
    rows = _rows_from_csr(m, row_ptr, col_idx, val, p)
    col_rows: dict[int, set[int]] = {}
    for i, r in enumerate(rows):
        for c in r:
            col_rows.setdefault(c, set()).add(i)
    active = set(i for i, r in enumerate(rows) if r)
    heap = [(len(rows[i]), i) for i in active]
    heapq.heapify(heap)
    rank = 0
    while heap:
        ln, i = heapq.heappop(heap)
        if i not in active or ln != len(rows[i]):
            continue  # stale heap entry
        row = rows[i]
        if not row:
            active.discard(i)
            continue
        # pivot column: fewest remaining rows, then smallest index
        c = min(row, key=lambda cc: (len(col_rows[cc]), cc))
        inv = pow(row[c], p - 2, p)
        active.discard(i)
        for cc in row:
            col_rows[cc].discard(i)
        rank += 1
        for j in list(col_rows[c]):
            rj = rows[j]
            f = (rj[c] * inv) % p
            for cc, v in row.items():
                nv = (rj.get(cc, 0) - f * v) % p
                if nv:
                    if cc not in rj:
                        col_rows[cc].add(j)
                    rj[cc] = nv
                elif cc in rj:
                    del rj[cc]
                    col_rows[cc].discard(j)
            if rj:
                heapq.heappush(heap, (len(rj), j))
            else:
                active.discard(j)
        rows[i] = {}
    return rank


def rank_dense_modp(M, p: int) -> int:
    """Rank over GF(p) of a dense integer matrix by plain row reduction."""
    A = [[int(x) % p for x in row] for row in np.asarray(M, dtype=object).tolist()]
    m = len(A)
    n = len(A[0]) if m else 0
    rank = 0
    for c in range(n):
        piv = next((i for i in range(rank, m) if A[i][c]), None)
        if piv is None:
            continue
        A[rank], A[piv] = A[piv], A[rank]
        inv = pow(A[rank][c], p - 2, p)
        A[rank] = [(x * inv) % p for x in A[rank]]
        for i in range(m):
            if i != rank and A[i][c]:
                f = A[i][c]
                A[i] = [(x - f * y) % p for x, y in zip(A[i], A[rank])]
        rank += 1
        if rank == m:
            break
    return rank


def rank_bareiss(M) -> int:
    """Rank over Q of an integer matrix by fraction-free Bareiss elimination."""
    A = [[int(x) for x in row] for row in np.asarray(M, dtype=object).tolist()]
    m = len(A)
    n = len(A[0]) if m else 0
    prev = 1
    rank = 0
    for c in range(n):
        piv = next((i for i in range(rank, m) if A[i][c] != 0), None)
        if piv is None:
            continue
        A[rank], A[piv] = A[piv], A[rank]
        for i in range(rank + 1, m):
            for j in range(c + 1, n):
                # exact division: the Bareiss identity keeps every entry a minor
                A[i][j] = (A[rank][c] * A[i][j] - A[i][c] * A[rank][j]) // prev
            A[i][c] = 0
        prev = A[rank][c]
        rank += 1
        if rank == m:
            break
    return rank


def rank_csr(A, p: int) -> int:
    """Sparse elimination on a ``workloads.CSR``-like object (attributes m, n, row_ptr, col_idx, val)."""
    return rank_sparse_modp(A.m, A.n, A.row_ptr, A.col_idx, A.val, p)


def rank_over_integers(A, primes) -> int:
    """Largest rank of the CSR-like ``A`` over GF(p) for p in ``primes`` (Section 2.5).  Every modular rank is at
    most the rank over Q, so the maximum is a lower bound that equals it unless every prime divides every
    non-zero maximal minor."""
    return max(rank_csr(A, int(p)) for p in primes)
