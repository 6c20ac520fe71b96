"""GPU tests of the continuous-batching server: ranks equal the planted ranks
and the single-matrix path, a request's result is the same alone and in the
mix, requests that arrive while others run join the running batch, and
admission respects the HBM budget."""
import threading
import time

import numpy as np
import pytest

import paper_0704_2351_amd as bw
from tests.gpu_util import announce, need_gpu
from workloads import CONFIG4_PRIMES, planted

pytestmark = pytest.mark.gpu


def requests(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(np.exp(rng.uniform(np.log(150), np.log(2500))))
        m = int(1.5 * n)
        r = int(n * rng.uniform(0.7, 0.95))
        p = int(CONFIG4_PRIMES[rng.integers(0, 4)])
        out.append((planted(m, n, r, 9, 7000 + seed * 100 + j), p, 11 + j))
    return out


def test_server_ranks_and_alone_vs_mix():
    need_gpu()
    announce("server mix")
    reqs = requests(10, 1)
    srv = bw.Server(4 << 30, 16, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    ranks = [srv.wait(t) for t in tickets]
    st = srv.stats()
    announce(f"  stats {st}")
    srv.close()
    for (A, p, sd), r in zip(reqs, ranks):
        assert r == A.planted_rank
    assert st["completed"] == 10 and st["max_active"] > 1
    # alone: a fresh server with one request
    srv = bw.Server(4 << 30, 16, 8)
    A, p, sd = reqs[3]
    assert srv.wait(srv.submit(A, p, sd)) == ranks[3]
    srv.close()
    assert bw.rank_modp(A, p, 8, sd)[0] == ranks[3]


def test_server_continuous_arrivals():
    """Requests arrive while earlier ones are on the device; they join at step boundaries."""
    need_gpu()
    announce("server staggered arrivals")
    reqs = requests(12, 2)
    srv = bw.Server(4 << 30, 32, 8)
    tickets = [None] * len(reqs)

    def feeder():
        for i, (A, p, sd) in enumerate(reqs):
            tickets[i] = srv.submit(A, p, sd)
            time.sleep(0.02)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    ranks = [srv.wait(t) for t in tickets]
    st = srv.stats()
    announce(f"  stats {st}")
    srv.close()
    assert ranks == [A.planted_rank for A, _, _ in reqs]
    assert st["p99_ms"] >= st["p50_ms"] > 0
    assert st["solves_per_s"] > 0


def test_server_admission_by_budget():
    """The device bytes of the requests admitted at once (encoded matrices, blocks, sequences, and the upload
    of the one being encoded) never exceed the budget, which bounds how many run together."""
    need_gpu()
    announce("server budget")
    reqs = [(planted(2250, 1500, 1200, 9, 6600 + j), CONFIG4_PRIMES[j % 4], 3 + j) for j in range(8)]
    # unconstrained: all eight admitted together
    srv = bw.Server(4 << 30, 64, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    assert [srv.wait(t) for t in tickets] == [A.planted_rank for A, _, _ in reqs]
    free = srv.stats()
    srv.close()
    announce(f"  unconstrained stats {free}")
    # half of that peak: fewer requests at once, every rank still right, the peak within the budget
    budget = free["peak_bytes"] // 2
    srv = bw.Server(budget, 64, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    ranks = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    announce(f"  budget {budget} stats {st}")
    assert ranks == [A.planted_rank for A, _, _ in reqs]
    assert st["max_active"] < len(reqs)
    assert 0 < st["peak_bytes"] <= budget
    # a request larger than the whole budget is refused
    srv = bw.Server(1 << 20, 4, 8)
    with pytest.raises(bw.BwrError) as ei:
        srv.submit(planted(30000, 20000, 15000, 9, 5), 65521, 1)
    assert ei.value.code == -3
    srv.close()


@pytest.mark.parametrize("ahead", ["0", "1", "2"])
def test_server_readouts_beside_captures(monkeypatch, ahead):
    """Many requests of staggered lengths: the active sets change often, so each batch captures new graphs
    while read-outs of finished requests wait for their sequences on other threads.  A read-out's wait must
    never meet a capture (HIP would refuse it and invalidate the capture); every answer is the planted rank,
    with and without the bound on queued advances."""
    need_gpu()
    announce(f"server read-outs beside captures, BWR_SERVER_AHEAD={ahead}")
    monkeypatch.setenv("BWR_SERVER_AHEAD", ahead)
    rng = np.random.default_rng(40 + int(ahead))
    reqs = []
    for j in range(40):
        n = int(rng.integers(600, 4000))
        r = int(n * rng.uniform(0.7, 0.95))
        p = int(CONFIG4_PRIMES[j % 4])
        reqs.append((planted(int(1.5 * n), n, r, 9, 9100 + j), p, 21 + j))
    srv = bw.Server(4 << 30, 24, 8)
    tickets = []
    for w in range(4):
        tickets += [srv.submit(A, p, sd) for A, p, sd in reqs[10 * w:10 * w + 10]]
        time.sleep(0.015)
    ranks = [srv.wait(t) for t in tickets]
    st = srv.stats()
    announce(f"  stats {st}")
    srv.close()
    assert ranks == [A.planted_rank for A, _, _ in reqs]
    assert st["completed"] == 40 and st["max_active"] > 4


def test_server_failed_advance_answers_and_recovers(monkeypatch):
    """An advance that reports an error (forced from the host, no kernel is launched) answers every request in
    the batch with that error and releases its job; requests submitted afterwards are answered correctly."""
    need_gpu()
    announce("server failed advance")
    monkeypatch.setenv("BWR_SERVER_FAIL_ADVANCE", "1")
    # 252 terms each: several advances of 64 steps, so the second advance finds them all in the batch
    reqs = [(planted(1500, 1000, 800, 9, 8800 + j), CONFIG4_PRIMES[j % 4], 5 + j) for j in range(4)]
    srv = bw.Server(4 << 30, 16, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    codes = []
    for t in tickets:
        try:
            codes.append(srv.wait(t))
        except bw.BwrError as e:
            codes.append(e.code)
    assert -4 in codes  # at least the requests in the failed batch carry BWR_EDEVICE
    later = requests(3, 6)
    ranks = [srv.wait(srv.submit(A, p, sd)) for A, p, sd in later]
    st = srv.stats()
    srv.close()
    assert ranks == [A.planted_rank for A, _, _ in later]
    assert st["completed"] == 7


def test_server_solo_lane(monkeypatch):
    """Requests of at least BWR_SERVER_SOLO_NNZ non-zeros run through the single-matrix path on the server's
    solo lane while the batches run the others: every answer equals the planted rank and the plain
    single-matrix rank, also with two draws per request and with a budget that admits one request at a time."""
    need_gpu()
    announce("server solo lane")
    monkeypatch.setenv("BWR_SERVER_SOLO_NNZ", "20000")
    reqs = requests(8, 4) + [(planted(24000, 16000, 13000, 9, 7777), 65521, 5),
                             (planted(30000, 20000, 15000, 9, 7778), 2**31 - 1, 6)]
    assert sum(A.nnz >= 20000 for A, _, _ in reqs) >= 3 and sum(A.nnz < 20000 for A, _, _ in reqs) >= 3
    srv = bw.Server(4 << 30, 16, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    ranks = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    announce(f"  stats {st}")
    assert ranks == [A.planted_rank for A, _, _ in reqs]
    assert st["completed"] == len(reqs)
    for A, p, sd in reqs[-2:]:
        assert bw.rank_modp(A, p, 8, sd)[0] == A.planted_rank
    bw.set_trials(2)
    try:
        srv = bw.Server(4 << 30, 16, 8)
        tickets = [srv.submit(A, p, sd) for A, p, sd in reqs[-3:]]
        assert [srv.wait(t) for t in tickets] == [A.planted_rank for A, _, _ in reqs[-3:]]
        srv.close()
    finally:
        bw.set_trials(1)
    # a budget near the largest single request: the lanes take turns, every answer still right
    big = max(st["peak_bytes"] // 3, 64 << 20)
    srv = bw.Server(big, 16, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    assert [srv.wait(t) for t in tickets] == [A.planted_rank for A, _, _ in reqs]
    st2 = srv.stats()
    srv.close()
    announce(f"  budget {big} stats {st2}")
    assert 0 < st2["peak_bytes"] <= big


def test_server_solo_lane_releases_its_budget(monkeypatch):
    """A budget that holds exactly one solo request: three of them, submitted together, run one after the other
    (each releases all it held, the upload included, when answered); polled with a deadline, not waited on."""
    need_gpu()
    announce("server solo lane budget release")
    monkeypatch.setenv("BWR_SERVER_SOLO_NNZ", "20000")
    reqs = [(planted(24000, 16000, 13000, 9, 7790 + j), 65521, 5 + j) for j in range(3)]
    reqs.sort(key=lambda q: -q[0].nnz)  # the budget is measured on the largest
    srv = bw.Server(4 << 30, 16, 8)
    assert srv.wait(srv.submit(*reqs[0])) == reqs[0][0].planted_rank
    one = srv.stats()["peak_bytes"]
    srv.close()
    assert one > 0
    srv = bw.Server(one, 16, 8)
    tickets = [srv.submit(A, p, sd) for A, p, sd in reqs]
    deadline = time.time() + 120
    ranks = [None] * len(tickets)
    while time.time() < deadline and any(r is None for r in ranks):
        for i, t in enumerate(tickets):
            if ranks[i] is None:
                done, r = srv.poll(t)
                if done:
                    ranks[i] = r
        time.sleep(0.05)
    st = srv.stats()
    srv.close()
    announce(f"  budget {one} stats {st}")
    assert ranks == [A.planted_rank for A, _, _ in reqs], ranks
    assert st["peak_bytes"] <= one
