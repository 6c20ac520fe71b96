"""Planted mistakes in the oracle, on the CPU: each plausible slip (a dropped diagonal, a transposed operand or
result, a lost sign, a reversal by the wrong degree, a missing codegree) is planted into a copy of the oracle's
behaviour with monkeypatch, and the pin that guards against it must then fail.  This shows that the pins tie
the oracle to the mathematics rather than to itself (the pins themselves are in test_oracle_*.py)."""
import numpy as np
import pytest

from oracle import ge, sequence as oseq, sigma
from workloads import planted

P = 65521


def _case(seed=3, m=9, n=7, r=5, s=2, L=8):
    rng = np.random.default_rng(seed)
    A = planted(m, n, r, 2, 700 + seed)
    dr = rng.integers(1, P, size=m)
    dc = rng.integers(1, P, size=n)
    U = rng.integers(0, P, size=(n, s))
    V = rng.integers(0, P, size=(n, s))
    return A, dr, dc, U, V, L


def _sequence_pin_holds(A, dr, dc, U, V, L):
    """The pin of the sequence: sparse oracle against explicit big-integer powers of the dense B."""
    got = oseq.sequence(A, U, V, P, L, dr, dc)
    want = np.array(oseq.dense_sequence(A.to_dense(), U, V, P, L, dr, dc), dtype=np.int64)
    return np.array_equal(got, want)


def test_unmutated_sequence_passes_its_pin():
    assert _sequence_pin_holds(*_case())


def test_dropped_column_diagonal_is_caught(monkeypatch):
    orig = oseq.Oracle.__init__

    def no_dc(self, m, n, row_ptr, col_idx, val, p, d_row=None, d_col=None):
        orig(self, m, n, row_ptr, col_idx, val, p, d_row, None)

    monkeypatch.setattr(oseq.Oracle, "__init__", no_dc)
    assert not _sequence_pin_holds(*_case())


def test_dropped_row_diagonal_is_caught(monkeypatch):
    monkeypatch.setattr(oseq.Oracle, "half", lambda self, X: oseq._spmm_exact(self.A, X, self.p))
    assert not _sequence_pin_holds(*_case())


def test_transposed_projection_is_caught(monkeypatch):
    # S_k^T = V^T B^k U instead of U^T B^k V (B is symmetric, so only U != V tells them apart)
    orig = oseq.project
    monkeypatch.setattr(oseq, "project", lambda U, W, p: orig(U, W, p).T)
    assert not _sequence_pin_holds(*_case())


def test_lost_sign_of_entries_is_caught(monkeypatch):
    # entries reduced from |a| instead of a: the elimination oracle against Bareiss over Q
    M = np.array([[1, 1, 0], [1, -1, 2], [0, 0, 3]])
    assert ge.rank_dense_modp(M, P) == ge.rank_bareiss(M) == 3
    orig = ge._rows_from_csr

    def abs_rows(m, row_ptr, col_idx, val, p):
        return orig(m, row_ptr, col_idx, np.abs(np.asarray(val)), p)

    monkeypatch.setattr(ge, "_rows_from_csr", abs_rows)
    from workloads import from_dense

    B = from_dense(M)
    assert ge.rank_csr(B, P) != ge.rank_bareiss(M)


def test_reversal_by_polynomial_degree_is_caught(monkeypatch):
    # F(x) = x^deg(p) p(1/x) instead of x^delta p(1/x): for s = 1 and a singular B the factor x^codeg of the
    # minimal polynomial is lost, so the generator is no longer the minimal polynomial of B (the pin that
    # compares them fails; the read-out alone would not see it, deg det F - codeg det F being unchanged)
    A, dr, dc, U, V, _ = _case(seed=4, m=9, n=7, r=5, s=1)
    L = 2 + 2 * A.n + 4
    S = oseq.sequence(A, U, V, P, L, dr, dc)
    B = oseq.dense_B(A.to_dense(), P, dr, dc)
    mp = sigma.minpoly_dense(B, P)
    assert mp[0] == 0  # B is singular: x divides its minimal polynomial

    def monic(f):
        f = [int(x) % P for x in f]
        while len(f) > 1 and f[-1] == 0:
            f.pop()
        inv = pow(f[-1], P - 2, P)
        return [x * inv % P for x in f]

    F, _, _ = sigma.min_generator(S, P)
    assert monic(F[:, 0, 0]) == mp
    orig = sigma.min_generator

    def by_poly_degree(S_, p):
        F_, delta, Prow = orig(S_, p)
        dp = max([j for j in range(Prow.shape[0]) if Prow[j, 0, :].any()] or [0])
        G = np.zeros((dp + 1, 1, 1), dtype=np.int64)
        for j in range(dp + 1):
            G[dp - j, 0, 0] = Prow[j, 0, 0]
        return G, [dp], Prow

    monkeypatch.setattr(sigma, "min_generator", by_poly_degree)
    F, _, _ = sigma.min_generator(S, P)
    assert monic(F[:, 0, 0]) != mp


def test_missing_codegree_is_caught(monkeypatch):
    # rank = deg det F without subtracting codeg det F: wrong whenever B is singular (r < n)
    A, dr, dc, U, V, _ = _case(seed=7, m=22, n=15, r=9, s=2)
    L = 2 + -(-2 * A.n // 2)
    S = oseq.sequence(A, U, V, P, L, dr, dc)
    want = ge.rank_csr(A, P)
    assert sigma.rank_from_sequence(S, P) == want == 9
    monkeypatch.setattr(sigma, "det_valuation", lambda M, p, max_k=None: 0)
    assert sigma.rank_from_sequence(S, P) != want


def test_premature_generator_is_caught():
    # a generator taken at or before the last order where the generator rows' degrees move (a premature
    # early stop) does not annihilate the terms past it, and its read-out can even exceed the rank; three
    # orders later it annihilates them and reads out the rank
    A, dr, dc, U, V, _ = _case(seed=2, m=40, n=30, r=12, s=2)
    L = 2 + -(-2 * A.n // 2)
    S = oseq.sequence(A, U, V, P, L + 8, dr, dc)
    want = ge.rank_csr(A, P)
    G = np.zeros((L, 4, 2), dtype=np.int64)
    G[:, :2, :] = S[:L]
    G[0, 2:, :] = (-np.eye(2, dtype=np.int64)) % P
    sums = [sum(sorted(sigma.mbasis(G, c, [0, 0, 1, 1], P)[1])[:2]) for c in range(L + 1)]
    c_star = max(c for c in range(L + 1) if c == 0 or sums[c] != sums[c - 1])
    for c in (c_star - 1, c_star):
        F, _, _ = sigma.min_generator(S[:c], P)
        assert not sigma.annihilates(F, S, P)
    F, _, _ = sigma.min_generator(S[:c_star], P)
    assert sigma.rank_from_generator(F, P) > want
    F, _, _ = sigma.min_generator(S[:c_star + 3], P)
    assert sigma.annihilates(F, S, P)
    assert sigma.rank_from_generator(F, P) == want
