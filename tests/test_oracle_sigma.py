"""Pins for the generator and read-out oracle (oracle/sigma.py): steps 3 and 4
of the "Block Wiedemann Rank Algorithm" (Section 2.5) and the sigma-basis of
Section 2.4."""
import numpy as np
import pytest

from oracle import ge, sequence as oseq, sigma
from workloads import planted, from_dense

P = 65521


def monic(f, p):
    inv = pow(int(f[-1]), p - 2, p)
    return [int(x) * inv % p for x in f]


def test_bm_textbook_sequences():
    p = 101
    fib = [0, 1]
    for _ in range(10):
        fib.append((fib[-1] + fib[-2]) % p)
    ell, f = sigma.berlekamp_massey(fib, p)
    assert ell == 2 and f == [p - 1, p - 1, 1]  # x^2 - x - 1
    geo = [pow(7, k, p) for k in range(8)]
    assert sigma.berlekamp_massey(geo, p) == (1, [p - 7, 1])  # x - 7
    imp = [5, 0, 0, 0, 0, 0]
    assert sigma.berlekamp_massey(imp, p) == (1, [0, 1])  # x: codegree 1
    assert sigma.berlekamp_massey([0] * 6, p) == (0, [1])
    # a_k = k: (x - 1)^2
    assert sigma.berlekamp_massey(list(range(8)), p) == (2, [1, p - 2, 1])


def tiny_case(seed, m=9, n=7, r=5, k=2, s=1, L=None, p=P, dcol=True):
    rng = np.random.default_rng(seed)
    A = planted(m, n, r, k, 300 + seed)
    dr = rng.integers(1, p, size=m)
    dc = rng.integers(1, p, size=n) if dcol else None
    U = rng.integers(0, p, size=(n, s))
    V = rng.integers(0, p, size=(n, s))
    L = L or 2 + -(-2 * n // s) + 4
    return A, dr, dc, oseq.sequence(A, U, V, p, L, dr, dc)


@pytest.mark.parametrize("seed", range(8))
def test_scalar_generator_is_minpoly(seed):
    A, dr, dc, S = tiny_case(seed)
    B = oseq.dense_B(A.to_dense(), P, dr, dc)
    mp = sigma.minpoly_dense(B, P)
    ell, f = sigma.berlekamp_massey(S[:, 0, 0], P)
    F, delta, _ = sigma.min_generator(S, P)
    assert f == mp
    assert monic(F[:, 0, 0], P) == mp
    assert delta == [ell]


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("s", [2, 3, 4])
def test_block_generator_degrees_and_annihilation(seed, s):
    A, dr, dc, S = tiny_case(seed, m=24, n=16, r=11, k=3, s=s)
    L = S.shape[0] - 4
    F, delta, _ = sigma.min_generator(S[:L], P)
    assert sigma.annihilates(F, S, P)  # holds on 4 terms beyond those used
    Pf = sigma.popov_form(F, P)
    assert sigma.annihilates(Pf, S, P)
    assert sorted(sigma.row_degrees(Pf)) == sigma.hankel_generator_degrees(S, P, max(delta) + 1)
    assert sum(sigma.row_degrees(Pf)) == sum(delta)


def test_popov_is_unique_normal_form():
    A, dr, dc, S = tiny_case(3, m=24, n=16, r=11, k=3, s=3)
    F, _, _ = sigma.min_generator(S, P)
    Pf = sigma.popov_form(F, P)
    # a unimodular left multiple has the same Popov form
    rng = np.random.default_rng(0)
    T = np.zeros((2, 3, 3), dtype=np.int64)
    T[0] = np.eye(3, dtype=np.int64)
    T[1, 0, 2] = int(rng.integers(1, P))  # row0 += c x row2
    T[0, 1, 0] = int(rng.integers(1, P))  # row1 += c row0
    G = np.zeros((F.shape[0] + 1, 3, 3), dtype=np.int64)
    for a in range(2):
        for b in range(F.shape[0]):
            G[a + b] = (G[a + b] + sigma._matmul_mod(T[a], F[b], P)) % P
    assert np.array_equal(sigma.popov_form(G, P), Pf)
    # Popov shape: monic pivots on the diagonal, strictly smaller degrees elsewhere in the column
    degs = sigma.row_degrees(Pf)
    for i in range(3):
        assert Pf[degs[i], i, i] == 1
        for j in range(3):
            if j != i:
                assert sigma.poly_deg(Pf[:, j, i]) < degs[i]


@pytest.mark.parametrize("seed", range(6))
def test_codegree_by_local_smith_matches_interpolation(seed):
    A, dr, dc, S = tiny_case(seed, m=20, n=12, r=7, k=3, s=2)
    F, _, _ = sigma.min_generator(S, P)
    det = sigma.det_by_interpolation(F, P)
    nz = [i for i, x in enumerate(det) if x]
    assert sigma.det_valuation(F, P) == nz[0]
    assert sum(sigma.row_degrees(sigma.weak_popov(F, P))) == nz[-1]


def test_det_valuation_known():
    p = 101
    # diag(x^2, x (1 + x)) -> valuation 3
    M = np.zeros((3, 2, 2), dtype=np.int64)
    M[2, 0, 0] = 1
    M[1, 1, 1] = 1
    M[2, 1, 1] = 1
    assert sigma.det_valuation(M, p) == 3
    # [[x, 1], [0, x]] -> x^2
    M = np.zeros((2, 2, 2), dtype=np.int64)
    M[1, 0, 0] = 1
    M[0, 0, 1] = 1
    M[1, 1, 1] = 1
    assert sigma.det_valuation(M, p) == 2
    # [[1, x], [x, x^2]] is singular
    M = np.zeros((3, 2, 2), dtype=np.int64)
    M[0, 0, 0] = 1
    M[1, 0, 1] = 1
    M[1, 1, 0] = 1
    M[2, 1, 1] = 1
    assert sigma.det_valuation(M, p) is None


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_readout_matches_elimination_and_rank_of_power(seed, s):
    A, dr, dc, S = tiny_case(seed, m=22, n=15, r=9 + seed % 4, k=3, s=s)
    L = 2 + -(-2 * A.n // s)
    got = sigma.rank_from_sequence(S[:L], P)
    B = oseq.dense_B(A.to_dense(), P, dr, dc)
    assert got == sigma.rank_of_power(B, P) == ge.rank_csr(A, P) == A.planted_rank


def test_isotropic_row_space_needs_column_scaling():
    # a^2 = -1 mod 65521: the row (1, a) is isotropic, so A^T D A is nilpotent for every D
    a = 24297
    assert a * a % P == P - 1
    A = from_dense(np.array([[1, a]]))
    rng = np.random.default_rng(1)
    U = rng.integers(0, P, size=(2, 1))
    V = rng.integers(0, P, size=(2, 1))
    S = oseq.sequence(A, U, V, P, 8, [int(rng.integers(1, P))])
    assert sigma.rank_from_sequence(S, P) == 0  # wrong: the true rank is 1
    S = oseq.sequence(A, U, V, P, 8, [int(rng.integers(1, P))], rng.integers(1, P, size=2))
    assert sigma.rank_from_sequence(S, P) == 1 == ge.rank_csr(A, P)


def test_readout_big_prime():
    p = 2**31 - 1
    A, dr, dc, S = tiny_case(5, m=18, n=12, r=8, k=3, s=2, p=p)
    L = 2 + -(-2 * A.n // 2)
    assert sigma.rank_from_sequence(S[:L], p) == 8


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("s", [2, 3])
def test_early_termination_reading(seed, s):
    """The reading behind early termination (the outlook of the conclusion), on the plain M-Basis: the
    sum of the s smallest shifted degrees of the order-c basis of [S; -I] never decreases, grows over
    every two orders while the generator rows still take pivots, and is constant from an order c* close
    to 2 r / s on.  A stall over a few orders therefore marks c*, and the generator of the order where the
    stall is seen has the same Popov form and read-out as the generator of the full length."""
    A, dr, dc, S = tiny_case(seed, m=40, n=30, r=8 + seed, k=3, s=s)
    r = A.planted_rank
    L = 2 + -(-2 * A.n // s)
    G = np.zeros((S.shape[0], 2 * s, s), dtype=np.int64)
    G[:, :s, :] = S
    G[0, s:, :] = (-np.eye(s, dtype=np.int64)) % P
    shift = [0] * s + [1] * s
    sums = [sum(sorted(sigma.mbasis(G, c, shift, P)[1])[:s]) for c in range(L + 1)]
    assert all(a <= b for a, b in zip(sums, sums[1:]))
    c_star = max(c for c in range(L + 1) if c == 0 or sums[c] != sums[c - 1])
    assert c_star <= 2 * -(-(r + 1) // s) + 2, (c_star, r, s)
    assert all(sums[c + 2] > sums[c] for c in range(c_star - 1)), sums
    # the stall over v orders is first seen at c_star + v
    v = 3
    c_stop = next(c for c in range(v, L + 1) if sums[c] == sums[c - v])
    assert c_stop == c_star + v
    F_full, _, _ = sigma.min_generator(S[:L], P)
    F_early, _, _ = sigma.min_generator(S[:c_stop], P)
    assert np.array_equal(sigma.popov_form(F_early, P), sigma.popov_form(F_full, P))
    assert sigma.annihilates(F_early, S, P)
    assert sigma.rank_from_generator(F_early, P) == r == ge.rank_csr(A, P)


@pytest.mark.parametrize("p", [5, 7, 11])
def test_readout_is_one_sided_at_tiny_primes(p):
    """Each draw of the method gives at most the rank mod p (Section 2.5: the algorithm can only return less),
    which is what makes the largest rank over several draws (trials, and the batched agreement retry) a valid
    result.  At tiny primes the random diagonals and projections are often degenerate, so draws fall short
    often: none may exceed the elimination rank, some fall short, and the largest over 16 draws reaches it."""
    A = planted(20, 14, 9, 3, 77)
    want = ge.rank_csr(A, p)
    assert want == A.planted_rank == 9
    s = 2
    L = 2 + -(-2 * A.n // s)
    got = []
    for seed in range(16):
        rng = np.random.default_rng(seed)
        dr = rng.integers(1, p, size=A.m)
        dc = rng.integers(1, p, size=A.n)
        U = rng.integers(0, p, size=(A.n, s))
        V = rng.integers(0, p, size=(A.n, s))
        S = oseq.sequence(A, U, V, p, L, dr, dc)
        got.append(sigma.rank_from_sequence(S, p))
    assert max(got) == want, got
    assert all(r <= want for r in got), got
    assert min(got) < want, got


@pytest.mark.parametrize("seed", range(4))
def test_early_termination_reading_symmetric_projection(seed):
    """The same premise with the symmetric projection U = V (Section 2.3), which early termination also
    serves: the generator rows' degree sum stalls at c* <= 2 ceil((r+1)/s) + 2, and the generator at the
    first stall seen over three orders reads out the rank."""
    p, s = P, 2
    rng = np.random.default_rng(500 + seed)
    A = planted(36, 26, 7 + seed, 3, 900 + seed)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    V = rng.integers(0, p, size=(A.n, s))
    L = 2 + -(-2 * A.n // s)
    S = oseq.sequence(A, V, V, p, L, dr, dc)
    assert all(np.array_equal(S[k], S[k].T) for k in range(L))
    G = np.zeros((L, 2 * s, s), dtype=np.int64)
    G[:, :s, :] = S
    G[0, s:, :] = (-np.eye(s, dtype=np.int64)) % p
    shift = [0] * s + [1] * s
    sums = [sum(sorted(sigma.mbasis(G, c, shift, p)[1])[:s]) for c in range(L + 1)]
    c_star = max(c for c in range(L + 1) if c == 0 or sums[c] != sums[c - 1])
    assert c_star <= 2 * -(-(A.planted_rank + 1) // s) + 2
    c_stop = next(c for c in range(3, L + 1) if sums[c] == sums[c - 3])
    F, _, _ = sigma.min_generator(S[:c_stop], p)
    assert sigma.rank_from_generator(F, p) == A.planted_rank == ge.rank_csr(A, p)


@pytest.mark.parametrize("m,n,r,s", [(24, 16, 9, 2), (30, 21, 14, 3), (40, 28, 20, 4)])
def test_sparse_projection_reading(m, n, r, s):
    """The premise of sparse projections (the other outlook of the conclusion; not built on the GPU): with U
    made of stacked s x s identity blocks (one non-zero per row, U[i, i mod s] = 1) and only V, D_r and D_c
    random, the generator still annihilates the terms past L and reads out the rank, on every draw tried."""
    A = planted(m, n, r, 3, 123)
    want = ge.rank_csr(A, P)
    assert want == r
    U = np.zeros((n, s), dtype=np.int64)
    U[np.arange(n), np.arange(n) % s] = 1
    L = 2 + -(-2 * n // s)
    for seed in range(6):
        rng = np.random.default_rng(seed)
        dr = rng.integers(1, P, size=m)
        dc = rng.integers(1, P, size=n)
        V = rng.integers(0, P, size=(n, s))
        S = oseq.sequence(A, U, V, P, L + 4, dr, dc)
        F, _, _ = sigma.min_generator(S[:L], P)
        assert sigma.annihilates(F, S, P)
        assert sigma.rank_from_generator(F, P) == want
