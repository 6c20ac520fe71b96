"""Pins for the rank oracle (oracle/ge.py, oracle/ge_rank.c): the plain
definition of the rank the method returns (Section 2.5)."""
import numpy as np
import pytest

from oracle import ge, native
from workloads import planted, random_sparse, from_dense, config1, config2

PRIMES = (3, 5, 65521, 2**31 - 1)


def all_ranks(A, p):
    M = A.to_dense()
    return (ge.rank_csr(A, p), ge.rank_dense_modp(M, p), native.rank_csr_c(A, p))


@pytest.mark.parametrize("seed", range(25))
def test_eliminations_agree_and_bareiss_bounds(seed):
    rng = np.random.default_rng(seed)
    m, n = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    A = random_sparse(m, n, float(rng.uniform(0.2, 0.8)), seed, vmax=6)
    rq = ge.rank_bareiss(A.to_dense())
    rp = []
    for p in PRIMES:
        r = all_ranks(A, p)
        assert r[0] == r[1] == r[2]
        assert r[0] <= rq
        rp.append(r[0])
    # over a large prime the rank mod p equals the rank over Q unless p divides every maximal minor
    assert max(rp) == rq


def test_bareiss_known_values():
    assert ge.rank_bareiss([[1, 2], [2, 4]]) == 1
    assert ge.rank_bareiss([[0, 0], [0, 0]]) == 0
    assert ge.rank_bareiss([[2, 3, 5], [7, 11, 13], [17, 19, 23]]) == 3  # det = -78
    assert ge.rank_bareiss([[1, 2, 3], [4, 5, 6], [7, 8, 9]]) == 2


@pytest.mark.parametrize("p", [65521, 2**31 - 1, 7])
def test_determinant_multiple_of_p(p):
    # det = -p: full rank over Q, rank 1 mod p (entries fit int32)
    M = np.array([[1, 1], [1, 1 - p]])
    A = from_dense(M)
    assert ge.rank_bareiss(M) == 2
    assert set(all_ranks(A, p)) == {1}
    # det [[2,3,5],[7,11,13],[17,19,23]] = -78 = -2*3*13: rank 2 mod 13, rank 3 mod 7
    M = np.array([[2, 3, 5], [7, 11, 13], [17, 19, 23]])
    A = from_dense(M)
    assert set(all_ranks(A, 13)) == {2}
    assert set(all_ranks(A, 7)) == {3}


@pytest.mark.parametrize("shape", [(40, 30, 20, 4), (60, 45, 44, 9), (25, 25, 25, 3), (50, 20, 2, 1)])
@pytest.mark.parametrize("p", [65521, 2**31 - 1, 3])
def test_planted_rank_exact(shape, p):
    m, n, r, k = shape
    A = planted(m, n, r, k, seed=11 * m + r)
    assert set(all_ranks(A, p)) == {r}
    if m * n <= 1600:
        assert ge.rank_bareiss(A.to_dense()) == r


@pytest.mark.parametrize("seed", range(6))
def test_transpose_and_bound(seed):
    A = random_sparse(12, 7, 0.3, 100 + seed)
    for p in (5, 65521):
        r = native.rank_csr_c(A, p)
        assert r == native.rank_csr_c(A.transpose(), p) == ge.rank_csr(A.transpose(), p)
        assert r <= min(A.m, A.n)


def test_permutation_and_unit_scaling_invariance():
    p = 65521
    A = planted(30, 24, 17, 4, 5)
    M = A.to_dense()
    rng = np.random.default_rng(3)
    M2 = M[rng.permutation(30)][:, rng.permutation(24)]
    M2 = M2 * rng.choice([-1, 1], size=(30, 1)) * rng.choice([-1, 1], size=(1, 24))
    M2 = M2 * rng.integers(1, 7, size=(30, 1))  # units mod p
    assert native.rank_csr_c(from_dense(M2), p) == native.rank_csr_c(A, p) == 17


def test_special_cases():
    for p in (3, 65521):
        assert set(all_ranks(from_dense(np.zeros((4, 5), np.int64)), p)) == {0}
        assert set(all_ranks(from_dense(np.eye(6, dtype=np.int64)), p)) == {6}
        assert set(all_ranks(from_dense(np.full((4, 4), p)), p)) == {0}
        M = np.zeros((5, 6), np.int64)
        M[2] = [0, 3, 0, -1, 2, 0]
        assert set(all_ranks(from_dense(M), p)) == {1}
    # duplicate entries are summed: 2 + (-2) = 0 leaves a zero matrix
    from workloads import coo_to_csr
    A = coo_to_csr(2, 2, [0, 0], [1, 1], [2, -2], coalesce=False)
    assert native.rank_csr_c(A, 65521) == 0 == ge.rank_csr(A, 65521)
    # empty shapes
    for m, n in ((0, 3), (3, 0), (0, 0)):
        A = from_dense(np.zeros((m, n), np.int64))
        assert native.rank_csr_c(A, 65521) == 0 == ge.rank_csr(A, 65521)


def test_config1_planted_rank():
    A = config1()
    assert A.nnz > 25_000
    assert native.rank_csr_c(A, 65521) == 1200
    assert ge.rank_csr(A, 65521) == 1200


def test_config2_planted_rank_both_primes():
    A = config2()
    assert 2_500_000 < A.nnz < 2_700_000
    assert native.rank_csr_c(A, 65521) == 140_000
    assert native.rank_csr_c(A, 2**31 - 1) == 140_000


def test_rank_over_integers_is_the_largest_modular_rank():
    """Section 2.5: the rank over the integers from several primes.  Pins: each modular rank is at most the
    Bareiss rank over Q; a matrix whose determinant is -78 = -2*3*13 has rank 2 mod 3 and mod 13 and rank 3 over
    Q, recovered once a prime not dividing 78 is among the primes; random integer matrices agree with Bareiss."""
    M = np.array([[2, 3, 5], [7, 11, 13], [17, 19, 23]])
    A = from_dense(M)
    assert ge.rank_over_integers(A, (3, 13)) == 2
    assert ge.rank_over_integers(A, (3, 13, 65521)) == 3 == ge.rank_bareiss(M)
    rng = np.random.default_rng(11)
    for _ in range(20):
        m, n = int(rng.integers(2, 9)), int(rng.integers(2, 9))
        M = rng.integers(-6, 7, size=(m, n)) * (rng.random((m, n)) < 0.6)
        A = from_dense(M)
        r = ge.rank_bareiss(M.tolist())
        assert all(ge.rank_csr(A, p) <= r for p in (3, 5, 7))
        assert ge.rank_over_integers(A, (3, 5, 65521, 2**31 - 1)) == r
