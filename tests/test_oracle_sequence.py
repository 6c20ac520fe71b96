"""Pins for the sequence oracle (oracle/sequence.py): S_k = U^T B^k V with
B = D_c A^T D_r A D_c (Sections 2.2, 2.3 and step 2 of Section 2.5)."""
import numpy as np
import pytest

from oracle import sequence as oseq
from workloads import planted, random_sparse, from_dense

PR = (65521, 2**31 - 1, 65537)


def rnd(rng, shape, p):
    return rng.integers(0, p, size=shape, dtype=np.int64)


@pytest.mark.parametrize("p", PR)
def test_s0_is_utv(p):
    rng = np.random.default_rng(1)
    A = random_sparse(9, 7, 0.3, 1)
    U, V = rnd(rng, (7, 3), p), rnd(rng, (7, 3), p)
    S = oseq.sequence(A, U, V, p, 1)
    want = [[sum(int(U[t, i]) * int(V[t, j]) for t in range(7)) % p for j in range(3)] for i in range(3)]
    assert S[0].tolist() == want


@pytest.mark.parametrize("p", PR)
def test_identity_closed_form(p):
    rng = np.random.default_rng(2)
    n, s = 6, 2
    A = from_dense(np.eye(n, dtype=np.int64))
    dr = rng.integers(1, p, size=n)
    dc = rng.integers(1, p, size=n)
    U, V = rnd(rng, (n, s), p), rnd(rng, (n, s), p)
    S = oseq.sequence(A, U, V, p, 5, dr, dc)
    lam = [int(dc[t]) * int(dc[t]) * int(dr[t]) % p for t in range(n)]
    for k in range(5):
        want = [[sum(int(U[t, i]) * pow(lam[t], k, p) * int(V[t, j]) for t in range(n)) % p
                 for j in range(s)] for i in range(s)]
        assert S[k].tolist() == want


def test_zero_matrix():
    p = 65521
    rng = np.random.default_rng(3)
    A = from_dense(np.zeros((5, 4), np.int64))
    S = oseq.sequence(A, rnd(rng, (4, 2), p), rnd(rng, (4, 2), p), p, 4)
    assert not S[1:].any()


@pytest.mark.parametrize("p", PR)
def test_one_row_closed_form(p):
    # A = a (1 x n), D_r = d: B = d D_c a^T a D_c, so for k >= 1
    # S_k = d^k (a D_c^2 a^T)^(k-1) (U^T D_c a^T)(a D_c V)
    rng = np.random.default_rng(4)
    n, s = 7, 3
    a = rng.integers(-3, 4, size=n)
    A = from_dense(a[None, :])
    d = int(rng.integers(1, p))
    dc = rng.integers(1, p, size=n)
    U, V = rnd(rng, (n, s), p), rnd(rng, (n, s), p)
    S = oseq.sequence(A, U, V, p, 5, [d], dc)
    aa = sum(int(a[t]) * int(dc[t]) ** 2 * int(a[t]) for t in range(n)) % p
    ua = [sum(int(U[t, i]) * int(dc[t]) * int(a[t]) for t in range(n)) for i in range(s)]
    av = [sum(int(a[t]) * int(dc[t]) * int(V[t, j]) for t in range(n)) for j in range(s)]
    for k in range(1, 5):
        want = [[pow(d, k, p) * pow(aa, k - 1, p) * ua[i] * av[j] % p for j in range(s)] for i in range(s)]
        assert S[k].tolist() == want


def test_symmetric_projection():
    p = 65521
    rng = np.random.default_rng(5)
    A = planted(20, 15, 10, 3, 5)
    V = rnd(rng, (15, 4), p)
    S = oseq.sequence(A, V, V, p, 8, rng.integers(1, p, size=20), rng.integers(1, p, size=15))
    for k in range(8):
        assert (S[k] == S[k].T).all()


def test_linearity_in_v():
    p = 2**31 - 1
    rng = np.random.default_rng(6)
    A = planted(20, 15, 10, 3, 6)
    U, V1, V2 = rnd(rng, (15, 3), p), rnd(rng, (15, 3), p), rnd(rng, (15, 3), p)
    c = int(rng.integers(1, p))
    dr = rng.integers(1, p, size=20)
    S1 = oseq.sequence(A, U, V1, p, 6, dr)
    S2 = oseq.sequence(A, U, V2, p, 6, dr)
    S3 = oseq.sequence(A, U, (V1 + c * V2) % p, p, 6, dr)
    assert ((S1 + c * S2) % p == S3).all()


@pytest.mark.parametrize("p", PR)
@pytest.mark.parametrize("seed", range(3))
def test_dense_power_agrees(p, seed):
    rng = np.random.default_rng(10 + seed)
    A = random_sparse(8, 6, 0.35, 20 + seed, vmax=5)
    U, V = rnd(rng, (6, 3), p), rnd(rng, (6, 3), p)
    dr, dc = rng.integers(1, p, size=8), rng.integers(1, p, size=6)
    S = oseq.sequence(A, U, V, p, 7, dr, dc)
    S2 = oseq.dense_sequence(A.to_dense(), U, V, p, 7, dr, dc)
    assert (S == S2).all()


def test_large_entries_take_exact_path():
    p = 2**31 - 1
    rng = np.random.default_rng(7)
    M = rng.integers(-(2**31) + 1, 2**31 - 1, size=(5, 4))
    M[rng.random((5, 4)) < 0.4] = 0
    A = from_dense(M)
    U, V = rnd(rng, (4, 2), p), rnd(rng, (4, 2), p)
    S = oseq.sequence(A, U, V, p, 4)
    S2 = oseq.dense_sequence(M, U, V, p, 4)
    assert (S == S2).all()
