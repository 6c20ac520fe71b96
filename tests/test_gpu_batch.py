"""GPU parity of the batched engine: every (matrix, prime) sequence advanced
in the batch equals the oracle's sequence with the same SplitMix64 draws
(the oracle's own implementation of the generator), a matrix's results are
the same alone and in a mix, and batched ranks equal single-matrix ranks."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge, native, splitmix
from oracle import sequence as oseq
from tests.gpu_util import announce, need_gpu
from workloads import from_dense, planted, random_sparse

pytestmark = pytest.mark.gpu
PRIMES4 = (65521, 65519, 65497, 2**31 - 1)


def oracle_batch_sequence(A, p, s, seed, length):
    """The sequence bwr_rank_modp draws for (A, p, s, seed): B on the smaller side."""
    T = A.transpose() if A.m < A.n else A
    nb, outer = T.n, T.m
    V = np.array(splitmix.block(seed, splitmix.STREAM_V, nb * s, p), dtype=np.int64).reshape(nb, s)
    U = np.array(splitmix.block(seed, splitmix.STREAM_U, nb * s, p), dtype=np.int64).reshape(nb, s)
    dr = np.array(splitmix.block(seed, splitmix.STREAM_DROW, outer, p, diag=True), dtype=np.int64)
    dc = np.array(splitmix.block(seed, splitmix.STREAM_DCOL, nb, p, diag=True), dtype=np.int64)
    return oseq.sequence(T, U, V, p, length, dr, dc)


MIX = [planted(300, 200, 150, 6, 1), planted(150, 260, 120, 5, 2), random_sparse(257, 129, 0.03, 3),
       planted(40, 30, 20, 3, 4)]


@pytest.mark.parametrize("s,primes", [(8, PRIMES4), (16, (65521, 2**31 - 1)), (4, PRIMES4), (3, (65537, 65521)),
                                      (32, (65519,)), (8, (65521, 65519, 65497)), (4, (3, 65521)),
                                      (16, (257, 40009))])
def test_batch_sequences_match_oracle(s, primes):
    """(Only 16-bit primes: the blocks are stored in 16-bit residues.)"""
    need_gpu()
    announce(f"batch sequences s={s} primes={primes}")
    lengths = [12, 7, 20, 3]
    seed = 77
    got = bw.sequence_batch(MIX, primes, s, seed, lengths)
    for j, A in enumerate(MIX):
        for t, p in enumerate(primes):
            want = oracle_batch_sequence(A, p, s, seed, lengths[j])
            assert np.array_equal(got[j][t].astype(np.int64), want), (j, p)


@pytest.mark.parametrize("graph", ["0", "1"])
def test_batch_long_run_with_graph_chunks(graph, monkeypatch):
    """Long enough for several 64-step chunks (graph replay) and jobs ending mid-run."""
    need_gpu()
    announce(f"batch long graph={graph}")
    monkeypatch.setenv("BWR_NO_GRAPH", "1" if graph == "0" else "0")
    mats = [planted(500, 350, 300, 6, 10), planted(220, 180, 150, 5, 11)]
    lengths = [301, 157]
    got = bw.sequence_batch(mats, (65521, 2**31 - 1), 8, 5, lengths)
    for j, A in enumerate(mats):
        for t, p in enumerate((65521, 2**31 - 1)):
            assert np.array_equal(got[j][t].astype(np.int64), oracle_batch_sequence(A, p, 8, 5, lengths[j]))


def test_alone_and_in_the_mix_are_identical():
    need_gpu()
    announce("batch alone vs mix")
    alone = bw.sequence_batch([MIX[0]], PRIMES4, 8, 9, [40])[0]
    mixed = bw.sequence_batch(MIX, PRIMES4, 8, 9, [40, 55, 30, 12])[0]
    assert np.array_equal(alone, mixed)


def test_batched_ranks_equal_single_ranks():
    need_gpu()
    announce("batched ranks")
    rng = np.random.default_rng(3)
    mats = []
    for j in range(6):
        n = int(rng.integers(300, 2500))
        m = int(n * rng.uniform(1.2, 2.0))
        r = int(n * rng.uniform(0.7, 0.95))
        mats.append(planted(m, n, r, 9, 4000 + j))
    mats.append(planted(400, 900, 350, 7, 4100))  # wide: transposed inside
    ranks, info = bw.rank_modp_batch(mats, PRIMES4, 8, 1)
    announce(f"  info {info}")
    for j, A in enumerate(mats):
        for t, p in enumerate(PRIMES4):
            assert ranks[j, t] == A.planted_rank, (j, p)
    # the single-matrix path gives the same numbers
    for j in (0, 6):
        for t, p in enumerate(PRIMES4[:2]):
            assert bw.rank_modp(mats[j], p, 8, 1)[0] == ranks[j, t]


@pytest.mark.parametrize("limit", ["1", "150000"])
def test_batched_ranks_with_single_matrix_share(limit, monkeypatch):
    """Matrices whose block of all primes exceeds the batched launches' budget (BWR_BATCH_BLOCK_BYTES) run
    as single-matrix solves on host threads beside the batched launches (all of them with limit 1, the
    larger ones with 150000): the ranks are those of the all-batched run and the planted ones."""
    need_gpu()
    announce(f"batched ranks with single-matrix share, limit {limit}")
    rng = np.random.default_rng(5)
    mats = []
    for j in range(6):
        n = int(rng.integers(300, 2500))
        mats.append(planted(int(n * rng.uniform(1.2, 2.0)), n, int(n * rng.uniform(0.7, 0.95)), 9, 4200 + j))
    want, _ = bw.rank_modp_batch(mats, PRIMES4, 8, 1)
    monkeypatch.setenv("BWR_BATCH_BLOCK_BYTES", limit)
    got, info = bw.rank_modp_batch(mats, PRIMES4, 8, 1)
    announce(f"  info {info}")
    assert np.array_equal(got, want)
    for j, A in enumerate(mats):
        assert (got[j] == A.planted_rank).all(), j
    if limit == "1":
        assert info["jobs"] == 0


def test_batched_ranks_with_wide_entries_and_empty():
    need_gpu()
    announce("batched ranks, wide entries and empty matrix")
    A = planted(200, 150, 110, 6, 31)
    A.val = (A.val.astype(np.int64) * 1000003 % (2**31 - 1)).astype(np.int32)
    Z = random_sparse(20, 10, 0.0, 1)
    B = planted(120, 100, 90, 5, 32)
    ranks, _ = bw.rank_modp_batch([A, Z, B], (65521, 2**31 - 1), 8, 2)
    assert ranks[1].tolist() == [0, 0]
    assert ranks[2].tolist() == [90, 90]
    for t, p in enumerate((65521, 2**31 - 1)):
        assert ranks[0, t] == native.rank_csr_c(A, p)


def test_rank_over_integers():
    """Section 2.5: the rank over the integers as the largest rank modulo several primes equals the oracle's
    and Bareiss's over Q on a 3 x 3 matrix of determinant -78 (rank 2 mod 3 and mod 13), and the planted rank
    of a planted matrix; no modular rank exceeds it."""
    need_gpu()
    announce("rank over the integers")
    M = np.array([[2, 3, 5], [7, 11, 13], [17, 19, 23]])
    A = from_dense(M)
    r, per = bw.rank_integer(A, (3, 13, 65521), 2, 4)
    assert r == ge.rank_bareiss(M) == 3
    assert per.max() == 3 and (per <= 3).all()
    B = planted(300, 220, 180, 7, 4300)
    primes = (3, 13, 65521, 2**31 - 1)
    r, per = bw.rank_integer(B, primes, 8, 2)
    assert r == ge.rank_over_integers(B, primes) == B.planted_rank
    assert (per <= B.planted_rank).all()
