"""Seeded synthetic sparse integer matrices with a planted rank.

The paper's matrices (the boundary maps of the Voronoi complex of GL_7(Z),
Section 2.1 and Table "tab:res") are not available here, so every workload is a
synthetic stand-in with their shape traits: very sparse (below 1 %, down to
0.2 %), small integer entries that are mostly +-1 (the differential of
Section 2.1.2 has incidence-number entries), 8 to 37 million non-zeros at
paper scale.

Construction (one definition for every workload):

* ``r`` core rows in triangular order.  Core row ``i`` has a 1 in core column
  ``i`` and ``min(i, k)`` further entries in distinct earlier core columns.
  Each of those further entries moves, with probability ``(n - r) / n``, to a
  uniformly chosen padding column (columns ``r .. n-1``), so padding columns
  are populated.  Entries that land on the same padding column are summed.
* ``m - r`` dependent rows, each ``core_a +- core_b`` (``a != b`` uniform, fair
  sign), summed entrywise with zeros dropped.
* Uniform random row and column permutations.

The core restricted to the core columns is unit lower triangular, so its
determinant is 1 and the rank is exactly ``r`` over Q and modulo every prime.

This module only draws inputs.  It holds none of the method's arithmetic and is
shared by the oracle-side tests and the GPU path's callers alike.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 0x07042351


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: int64 row pointers, int32 column indices and values."""

    m: int
    n: int
    row_ptr: np.ndarray  # int64, m + 1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray  # int32, nnz
    planted_rank: int | None = None

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.m, self.n), dtype=np.int64)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        np.add.at(out, (rows, self.col_idx.astype(np.int64)), self.val.astype(np.int64))
        return out

    def transpose(self) -> "CSR":
        rows = np.repeat(np.arange(self.m, dtype=np.int64), np.diff(self.row_ptr))
        return coo_to_csr(self.n, self.m, self.col_idx.astype(np.int64), rows, self.val, self.planted_rank)


def coo_to_csr(m: int, n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray,
               planted_rank: int | None = None, coalesce: bool = True) -> CSR:
    """Sort COO triples by (row, col); sum duplicates and drop zeros if ``coalesce``."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.int64)
    key = rows * np.int64(n) + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    if coalesce and key.size:
        starts = np.flatnonzero(np.concatenate(([True], key[1:] != key[:-1])))
        vals = np.add.reduceat(vals, starts)
        key = key[starts]
        keep = vals != 0
        key = key[keep]
        vals = vals[keep]
    r = key // n
    c = key - r * n
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=m), out=row_ptr[1:])
    return CSR(m, n, row_ptr, c.astype(np.int32), vals.astype(np.int32), planted_rank)


def from_dense(M: np.ndarray) -> CSR:
    M = np.asarray(M, dtype=np.int64)
    rows, cols = np.nonzero(M)
    return coo_to_csr(M.shape[0], M.shape[1], rows, cols, M[rows, cols])


def _offdiag_values(rng: np.random.Generator, count: int, frac_pm1: float, vmax: int) -> np.ndarray:
    """``frac_pm1`` of the values are +-1 (fair sign); the rest uniform on {-vmax..vmax} \\ {0}."""
    pm1 = rng.random(count) < frac_pm1
    sign = np.where(rng.random(count) < 0.5, -1, 1)
    mag = rng.integers(1, vmax + 1, size=count)
    return np.where(pm1, sign, sign * mag).astype(np.int64)


def _distinct_earlier_columns(rng: np.random.Generator, r: int, k: int):
    """For each core row i, ``min(i, k)`` distinct columns drawn from ``[0, i)``.

    Returns (row ids, column ids) as flat int64 arrays, grouped by row.
    """
    rows_out = []
    cols_out = []
    # rows 1..k take every earlier column
    small = np.arange(1, min(k, r - 1) + 1, dtype=np.int64) if r > 1 else np.zeros(0, np.int64)
    if small.size:
        rr = np.repeat(small, small)
        starts = np.repeat(np.cumsum(small) - small, small)
        cc = np.arange(rr.size, dtype=np.int64) - starts
        rows_out.append(rr)
        cols_out.append(cc)
    big = np.arange(k + 1, r, dtype=np.int64)
    if big.size and k > 0:
        draw = np.floor(rng.random((big.size, k)) * big[:, None]).astype(np.int64)
        # redraw rows with a repeated column until none is left; only redrawn rows can change,
        # so each round re-checks just those
        idx = np.arange(big.size)
        while idx.size:
            srt = np.sort(draw[idx], axis=1)
            idx = idx[np.any(srt[:, 1:] == srt[:, :-1], axis=1)]
            if idx.size:
                draw[idx] = np.floor(rng.random((idx.size, k)) * big[idx, None]).astype(np.int64)
        rows_out.append(np.repeat(big, k))
        cols_out.append(draw.reshape(-1))
    if rows_out:
        return np.concatenate(rows_out), np.concatenate(cols_out)
    return np.zeros(0, np.int64), np.zeros(0, np.int64)


def planted(m: int, n: int, r: int, k: int, seed: int, frac_pm1: float = 0.8, vmax: int = 3,
            permute: bool = True) -> CSR:
    """Planted-rank sparse integer matrix (see the module docstring)."""
    if not (0 <= r <= min(m, n)):
        raise ValueError("need 0 <= r <= min(m, n)")
    if r < 2 and m > r:
        raise ValueError("dependent rows need at least two core rows")
    rng = np.random.default_rng(seed)
    # core rows: diagonal plus off-diagonals
    orow, ocol = _distinct_earlier_columns(rng, r, k)
    oval = _offdiag_values(rng, orow.size, frac_pm1, vmax)
    if n > r and orow.size:
        move = rng.random(orow.size) < (n - r) / n
        ocol = np.where(move, rng.integers(r, n, size=orow.size), ocol)
    drow = np.arange(r, dtype=np.int64)
    core = coo_to_csr(r, n, np.concatenate((drow, orow)), np.concatenate((drow, ocol)),
                      np.concatenate((np.ones(r, np.int64), oval)))
    # dependent rows: core_a +- core_b
    nd = m - r
    rows_list = [np.repeat(np.arange(r, dtype=np.int64), np.diff(core.row_ptr))]
    cols_list = [core.col_idx.astype(np.int64)]
    vals_list = [core.val.astype(np.int64)]
    if nd > 0:
        a = rng.integers(0, r, size=nd)
        b = rng.integers(0, r - 1, size=nd)
        b = np.where(b >= a, b + 1, b)
        sgn = np.where(rng.random(nd) < 0.5, -1, 1).astype(np.int64)
        lens = np.diff(core.row_ptr)
        for src, mult in ((a, np.ones(nd, np.int64)), (b, sgn)):
            ln = lens[src]
            dep_ids = np.repeat(np.arange(nd, dtype=np.int64), ln)
            offs = np.arange(ln.sum(), dtype=np.int64) - np.repeat(np.cumsum(ln) - ln, ln)
            pos = np.repeat(core.row_ptr[src], ln) + offs
            rows_list.append(r + dep_ids)
            cols_list.append(core.col_idx[pos].astype(np.int64))
            vals_list.append(core.val[pos].astype(np.int64) * np.repeat(mult, ln))
    rows = np.concatenate(rows_list)
    cols = np.concatenate(cols_list)
    vals = np.concatenate(vals_list)
    if permute:
        rperm = rng.permutation(m).astype(np.int64)
        cperm = rng.permutation(n).astype(np.int64)
        rows = rperm[rows]
        cols = cperm[cols]
    return coo_to_csr(m, n, rows, cols, vals, planted_rank=r)


def random_sparse(m: int, n: int, density: float, seed: int, vmax: int = 3) -> CSR:
    """Unstructured sparse matrix (no planted rank): for ragged-row and edge-case tests."""
    rng = np.random.default_rng(seed)
    cnt = rng.binomial(m * n, density) if m * n else 0
    rows = rng.integers(0, max(m, 1), size=cnt)
    cols = rng.integers(0, max(n, 1), size=cnt)
    vals = rng.integers(-vmax, vmax + 1, size=cnt)
    return coo_to_csr(m, n, rows, cols, vals)


# --- the workload configurations -------------------------------------------------

def config_seed(config: int, j: int = 0) -> int:
    return BASE_SEED + 1000 * config + j


def config1() -> CSR:
    """2000 x 1500, planted rank 1200, ~9 off-diagonals per core row."""
    return planted(2000, 1500, 1200, 9, config_seed(1))


def config2() -> CSR:
    """200 000 x 150 000, planted rank 140 000 (~20 non-zeros per dependent row)."""
    return planted(200_000, 150_000, 140_000, 9, config_seed(2))


def config3(k: int = 11) -> CSR:
    """2 000 000 x 1 000 000, planted rank 900 000, ~37 M non-zeros, 85 % +-1."""
    return planted(2_000_000, 1_000_000, 900_000, k, config_seed(3), frac_pm1=0.85, vmax=4)


def config4_shapes(count: int = 64):
    """Shapes (m, n, r) of the batched workload: n log-uniform in 5e3..2e5."""
    rng = np.random.default_rng(config_seed(4, 999_999))
    out = []
    for _ in range(count):
        n = int(round(math.exp(rng.uniform(math.log(5e3), math.log(2e5)))))
        m = int(round(n * rng.uniform(1.2, 2.0)))
        r = int(round(n * rng.uniform(0.70, 0.95)))
        out.append((m, n, r))
    return out


def config4_matrix(j: int, shapes=None) -> CSR:
    shapes = shapes or config4_shapes()
    m, n, r = shapes[j]
    return planted(m, n, r, 9, config_seed(4, j))


CONFIG4_PRIMES = (65521, 65519, 65497, 2**31 - 1)


def config5_trace(count: int = 200, rate: float = 50.0, n_lo: float = 1e3, n_hi: float = 1e6):
    """Seeded Poisson arrival trace: (arrival_s, m, n, r, prime, seed) per request."""
    rng = np.random.default_rng(config_seed(5, 999_999))
    t = 0.0
    out = []
    for j in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(round(1.5 * n))
        r = int(round(n * rng.uniform(0.70, 0.95)))
        prime = int(CONFIG4_PRIMES[rng.integers(0, len(CONFIG4_PRIMES))])
        out.append((t, m, n, r, prime, config_seed(5, j)))
    return out
