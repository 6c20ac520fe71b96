"""GPU rank parity: the block Wiedemann rank (Section 2.5) equals the rank by
Gaussian elimination (the plain definition) bit for bit."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge, native
from tests.gpu_util import announce, need_gpu
from workloads import coo_to_csr, config1, config2, from_dense, planted, random_sparse

pytestmark = pytest.mark.gpu


def test_rank_config1():
    need_gpu()
    announce("rank config1 2000x1500 s=4 p=65521")
    A = config1()
    r, info = bw.rank_modp(A, 65521, 4, 1)
    assert r == native.rank_csr_c(A, 65521) == 1200
    assert info["len"] == 752 and info["s"] == 4


@pytest.mark.parametrize("seed", range(12))
def test_rank_small_random_cases(seed):
    need_gpu()
    rng = np.random.default_rng(seed)
    m = int(rng.integers(20, 400))
    n = int(rng.integers(20, 400))
    r = int(rng.integers(1, min(m, n)))
    k = int(rng.integers(1, 9))
    s = int(rng.choice([1, 2, 3, 4, 7, 8, 16]))
    p = int(rng.choice([65521, 65519, 65497, 2**31 - 1, 65537, 1000003]))
    announce(f"rank random m={m} n={n} r={r} s={s} p={p}")
    A = planted(m, n, r, k, 900 + seed)
    got, info = bw.rank_modp(A, p, s, 1 + seed)
    assert got == native.rank_csr_c(A, p) == r
    assert info["transposed"] == (1 if m < n else 0)


@pytest.mark.parametrize("seed", range(6))
def test_rank_unstructured(seed):
    need_gpu()
    announce(f"rank random_sparse seed={seed}")
    A = random_sparse(150 + 10 * seed, 120, 0.02 + 0.01 * seed, 70 + seed, vmax=4)
    p = 65521
    got, _ = bw.rank_modp(A, p, 4, 5)
    assert got == ge.rank_csr(A, p)


def test_rank_isotropic_row_space():
    """The row (1, a) with a^2 = -1 mod p is isotropic; the column scaling makes the rank come out."""
    need_gpu()
    announce("rank isotropic")
    A = from_dense(np.array([[1, 24297]]))
    got, _ = bw.rank_modp(A, 65521, 1, 3)
    assert got == 1


def test_rank_degenerate():
    need_gpu()
    announce("rank degenerate")
    assert bw.rank_modp(coo_to_csr(5, 7, [], [], []), 65521, 4, 1)[0] == 0
    assert bw.rank_modp(coo_to_csr(0, 7, [], [], []), 65521, 4, 1)[0] == 0
    assert bw.rank_modp(from_dense(np.full((4, 4), 65521)), 65521, 4, 1)[0] == 0  # entries = p
    assert bw.rank_modp(from_dense(np.eye(9, dtype=np.int64)), 65521, 4, 1)[0] == 9
    assert bw.rank_modp(from_dense(np.eye(9, dtype=np.int64)), 65521, 64, 1)[0] == 9
    M = np.zeros((6, 5), np.int64)
    M[3] = [0, 2, 0, -1, 5]
    assert bw.rank_modp(from_dense(M), 65521, 2, 1)[0] == 1


def test_rank_large_values():
    need_gpu()
    announce("rank wide encoding")
    rng = np.random.default_rng(8)
    A = planted(200, 150, 110, 6, 31)
    A.val = (A.val.astype(np.int64) * 1000003 % (2**31 - 1)).astype(np.int32)  # scale entries by a unit
    for p in (65521, 2**31 - 1):
        want = native.rank_csr_c(A, p)
        got, _ = bw.rank_modp(A, p, 8, 2)
        assert got == want


def test_rank_dev_entry_point():
    need_gpu()
    announce("rank_modp_dev")
    A = planted(500, 400, 333, 8, 5)
    Ad = bw.csr_to_device(A)
    got, info = bw.rank_modp_dev(Ad, 65521, 8, 9)
    assert got == 333


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_rank_config2(p):
    """200k x 150k, planted rank 140k, s = 8: the rank equals elimination's at both primes."""
    need_gpu()
    announce(f"rank config2 p={p}")
    A = config2()
    got, info = bw.rank_modp(A, p, 8, 1)
    announce(f"  info {info}")
    assert got == native.rank_csr_c(A, p) == 140_000


def test_concurrent_calls_from_host_threads():
    """Solves issued from several host threads (each on its own library stream) give the ranks and the
    sequences that the same calls give one after another."""
    import threading

    need_gpu()
    announce("concurrent host threads")
    mats = [planted(3000, 2200, 1900, 9, 70), planted(2500, 2000, 1500, 9, 71)]
    primes = [65521, 2**31 - 1]
    want = {(j, p): bw.rank_modp(A, p, 8, 3)[0] for j, A in enumerate(mats) for p in primes}
    rng = np.random.default_rng(0)
    A0 = mats[0]
    U = rng.integers(0, 65521, size=(A0.n, 4))
    V = rng.integers(0, 65521, size=(A0.n, 4))
    S_want = bw.sequence(A0, U, V, 65521, 300)
    got, seqs, errors = {}, [], []

    def solve(j, p):
        try:
            got[(j, p)] = bw.rank_modp(mats[j], p, 8, 3)[0]
            seqs.append(bw.sequence(A0, U, V, 65521, 300))
        except Exception as e:  # surfaced below
            errors.append(e)

    threads = [threading.Thread(target=solve, args=key) for key in want]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    assert got == want
    assert all(np.array_equal(S, S_want) for S in seqs) and len(seqs) == len(want)
