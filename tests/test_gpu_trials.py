"""Independent draws (bwr_set_trials): the rank algorithm's error is one-sided
(Section 2.5: a draw may return less than the rank, never more), so the
largest rank over several draws is kept.  The case is the one matrix of the
batched configuration whose first draw misses at p = 65521 (166849 x 132620,
planted rank 122034, n > p): one draw gives at most the planted rank, two draws
give it exactly, through the single-matrix path, the batched path and the
server."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from tests.gpu_util import announce, need_gpu
from workloads import config4_matrix

pytestmark = pytest.mark.gpu

MISS_J = 46  # (166849, 132620, rank 122034) in the batched configuration's shapes


@pytest.fixture(scope="module")
def miss():
    need_gpu()
    A = config4_matrix(MISS_J)
    assert (A.m, A.n, A.planted_rank) == (166849, 132620, 122034)
    return A


@pytest.fixture
def trials():
    old = bw.get_trials()
    yield bw.set_trials
    bw.set_trials(old)


def test_single_matrix_draws(miss, trials):
    announce("trials: single-matrix path")
    trials(1)
    r1, i1 = bw.rank_modp(miss, 65521, 8, 1)
    assert r1 <= miss.planted_rank and i1["trials"] == 1
    trials(2)
    r2, i2 = bw.rank_modp(miss, 65521, 8, 1)
    assert r2 == miss.planted_rank and i2["trials"] == 2
    # a draw that reaches min(m, n) ends the draws early: the 2^31 - 1 rank of a full-rank matrix
    # is not asked here; a full-column-rank case is checked on the host path below


def test_batched_draws(miss, trials):
    announce("trials: batched path")
    trials(2)
    ranks, _ = bw.rank_modp_batch([miss], [65521, 65519, 2**31 - 1], 8, 1)
    assert np.all(ranks == miss.planted_rank)


def test_served_draws(miss, trials):
    announce("trials: server")
    trials(2)
    srv = bw.Server(8 << 30, 8, 8)
    try:
        r = srv.wait(srv.submit(miss, 65521, 1))
    finally:
        srv.close()
    assert r == miss.planted_rank


def test_full_rank_stops_after_one_draw(trials):
    """A draw that reaches min(m, n) ends the computation: more draws cannot raise it."""
    need_gpu()
    from workloads import planted

    trials(4)
    A = planted(900, 600, 600, 7, 5)
    r, info = bw.rank_modp(A, 65521, 8, 1)
    assert r == 600 and info["trials"] == 1


def test_batched_agreement_retry(miss, trials):
    """One draw, with the agreement retry: the 16-bit prime whose first draw falls short of the other primes'
    rank gets a further draw and reaches the planted rank; the primes that agreed get none."""
    announce("trials: batched agreement retry")
    trials(1)
    old = bw.get_batch_retry()
    bw.set_batch_retry(2)
    try:
        ranks, info = bw.rank_modp_batch([miss], [65521, 65519, 2**31 - 1], 8, 1)
    finally:
        bw.set_batch_retry(old)
    assert np.all(ranks == miss.planted_rank), ranks
    assert 1 <= info["retries"] <= 2
