"""Early termination (the outlook of the paper's conclusion): a single-matrix rank
whose sequence stops once the device sigma-basis beside it has converged.  The
rank must equal the planted rank (exact over every field) and the elimination
oracle's, the generator must be taken at an order near 2 r / s + O(1) rather
than at L = 2 + ceil(2 min(m, n) / s), and, when the rank is well below
min(m, n), fewer terms must be computed than the full sequence has."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import native
from tests.gpu_util import announce, need_gpu
from workloads import planted

pytestmark = pytest.mark.gpu


@pytest.fixture
def early():
    need_gpu()
    old = bw.get_early_termination()
    bw.set_early_termination(True)
    yield
    bw.set_early_termination(old)


def _full_len(A, s):
    return bw.sequence_length(min(A.m, A.n), s)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_low_rank_stops_early(early, p):
    # r = 0.3 n: the generator's degree is about r / s, so about 2 r / s terms suffice
    m, n, r, s = 90000, 60000, 18000, 8
    announce(f"early termination: {m}x{n} rank {r}, s={s}, p={p}")
    A = planted(m, n, r, 9, 20260 + (p & 7))
    rank, info = bw.rank_modp(A, p, s, 1)
    L = _full_len(A, s)
    assert rank == r
    assert info["len"] < L // 2, (info["len"], L)
    assert info["len"] >= 2 * r // s, info["len"]
    assert info["check_terms"] == 4
    # terms computed: at least the generator's order plus the terms it was checked on, fewer than L
    assert info["len"] + 4 <= info["terms"] < L, (info["len"], info["terms"], L)


def test_equal_to_elimination_and_to_full_sequence(early):
    # rank close to min(m, n): the stall comes late or not at all; the result must not change
    m, n, r, s, p = 30000, 20000, 19000, 8, 65521
    announce(f"early termination: {m}x{n} rank {r} against elimination and the full sequence")
    A = planted(m, n, r, 9, 4242)
    r_early, i_early = bw.rank_modp(A, p, s, 3)
    bw.set_early_termination(False)
    r_full, i_full = bw.rank_modp(A, p, s, 3)
    bw.set_early_termination(True)
    assert r_early == r_full == native.rank_csr_c(A, p) == r
    assert i_full["len"] == _full_len(A, s) and i_full["terms"] == i_full["len"] + 4
    assert i_early["len"] <= i_full["len"]


def test_transposed_and_device_input(early):
    # m < n: B acts on the row side; the device-pointer entry point shares the path
    m, n, r, s, p = 40000, 60000, 12000, 8, 65521
    announce(f"early termination: transposed {m}x{n} rank {r}, s={s}, device input")
    A = planted(m, n, r, 9, 777)
    Ad = bw.csr_to_device(A, "cuda:0")
    rank, info = bw.rank_modp_dev(Ad, p, s, 5)
    assert rank == r
    assert info["transposed"] == 1
    assert info["len"] < _full_len(A, s) // 2


@pytest.mark.parametrize("gram", [False, True])
def test_symmetric_projection(early, gram):
    m, n, r, s, p = 60000, 40000, 10000, 8, 65521
    announce(f"early termination: symmetric projection, gram={gram}")
    A = planted(m, n, r, 9, 99 + int(gram))
    rank, info = bw.rank_modp_sym(A, p, s, 1, gram=gram)
    assert rank == r
    assert info["len"] < _full_len(A, s) // 2


def test_short_sequences_unchanged(early):
    # under 4096 terms the basis runs after the sequence: early termination does not apply
    A = planted(3000, 2000, 1200, 9, 5)
    rank, info = bw.rank_modp(A, 65521, 4, 1)
    assert rank == 1200 and info["len"] == _full_len(A, 4)



def test_batched_call_with_early_termination(early):
    # with early termination on, the batched call sends the matrices whose sequence can stop early to its
    # single-matrix lanes and batches the rest; every rank must still be the planted one
    mats = [planted(3000, 2000, 1500, 9, 11), planted(30000, 20000, 14000, 9, 12), planted(45000, 30000, 9000, 9, 13)]
    announce("early termination: batched call, 3 matrices x 3 primes")
    primes = [65521, 65519, 2**31 - 1]
    ranks, _ = bw.rank_modp_batch(mats, primes, 8, 1)
    want = np.array([[A.planted_rank] * len(primes) for A in mats])
    assert np.array_equal(ranks, want), (ranks, want)


def test_with_trials(early):
    # two draws, each stopping early; the larger rank is kept (both equal the planted rank here)
    old = bw.get_trials()
    bw.set_trials(2)
    try:
        A = planted(60000, 40000, 16000, 9, 31)
        announce("early termination: two draws")
        rank, info = bw.rank_modp(A, 65521, 8, 1)
    finally:
        bw.set_trials(old)
    assert rank == 16000 and info["trials"] == 2
    assert info["len"] < _full_len(A, 8) // 2


def test_workspace_form_runs_full_length(early):
    # inside a caller's workspace the generator is computed after the sequence (on the host), so early
    # termination does not apply there; the rank is the same
    A = planted(30000, 20000, 8000, 9, 41)
    announce("early termination: workspace form")
    Ad = bw.csr_to_device(A, "cuda:0")
    rank, info = bw.rank_modp_dev_ws(Ad, 65521, 8, 1)
    assert rank == 8000 and info["len"] == _full_len(A, 8)


def test_server_solo_lane(early):
    # a request of at least 2^20 non-zeros runs on the server's single-matrix lane, which stops early
    A = planted(105000, 70000, 42000, 9, 51)
    assert A.nnz >= 1 << 20
    announce(f"early termination: server solo lane, {A.m}x{A.n}, {A.nnz} non-zeros")
    srv = bw.Server(8 << 30, 8, 8)
    try:
        r = srv.wait(srv.submit(A, 65521, 1))
    finally:
        srv.close()
    assert r == 42000


def test_short_confirmation_still_right(early, monkeypatch):
    # confirmation over a single order with short chunks: while the sequence still looks generic the
    # generator rows take pivots at every order or two, so even this confirms only a true stall
    monkeypatch.setenv("BWR_EARLY_STEP", "64")
    monkeypatch.setenv("BWR_EARLY_VERIFY", "1")
    A = planted(30000, 20000, 9000, 9, 61)
    announce("early termination: step 64, confirmation over 1 order")
    for seed in (1, 2, 3):
        rank, info = bw.rank_modp(A, 65521, 8, seed)
        assert rank == 9000 and 2 * 9000 // 8 <= info["len"] < _full_len(A, 8), (seed, rank, info["len"])


def test_premature_stop_falls_back_to_full_length(early, monkeypatch):
    # the basis kept (by force) at the cut 1137, long before the generator is complete (about 2 r / s =
    # 2250): the kept generator fails its check on the terms past its order, and the draw is made again at
    # the full length, so the rank is right and no error reaches the caller
    monkeypatch.setenv("BWR_EARLY_FORCE_AT", "700")
    A = planted(30000, 20000, 9000, 9, 61)
    announce("early termination: forced premature stop, fallback to the full length")
    rank, info = bw.rank_modp(A, 65521, 8, 1)
    assert rank == 9000
    assert info["len"] == _full_len(A, 8) and info["terms"] == info["len"] + 4
