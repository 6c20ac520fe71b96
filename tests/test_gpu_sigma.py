"""GPU parity of the device sigma-basis (Section 2.4) and of the rank read-out
that uses it (Section 2.5): the device generator equals the host PM-Basis
generator entry for entry, its Popov form equals the oracle's, and ranks
agree with elimination whether the sigma-basis runs on the device or the host."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge, native
from oracle import sequence as oseq
from oracle import sigma
from tests.gpu_util import announce, blocks, need_gpu
from workloads import planted

pytestmark = pytest.mark.gpu


def to_dev(torch, S):
    return torch.from_numpy(np.ascontiguousarray(S, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


def reversed_generator(delta, P, s):
    D = max(delta)
    F = np.zeros((D + 1, s, s), dtype=np.int64)
    for i in range(s):
        for j in range(min(P.shape[0], delta[i] + 1)):
            F[delta[i] - j, i, :] = P[j, i, :]
    return F


@pytest.mark.parametrize("p", [65521, 2**31 - 1, 65537])
@pytest.mark.parametrize("s", [1, 2, 3, 4, 8, 16])
def test_device_generator_matches_host_and_oracle(s, p):
    torch = need_gpu()
    announce(f"device sigma-basis s={s} p={p}")
    rng = np.random.default_rng(s + p % 101)
    A = planted(90, 70, 50, 4, 60 + s)
    U, V = blocks(rng, A.n, s, p)
    dr, dc = rng.integers(1, p, size=A.m), rng.integers(1, p, size=A.n)
    L = sigma.sequence_length(A.n, s)
    S = oseq.sequence(A, U, V, p, L + 4, dr, dc)
    d_dev, P_dev = bw.min_generator_dev(to_dev(torch, S[:L]), p)
    d_host, P_host = bw.min_generator(S[:L], p)
    assert np.array_equal(d_dev, d_host)
    assert np.array_equal(P_dev, P_host)
    F = reversed_generator(d_dev.tolist(), P_dev.astype(np.int64), s)
    assert sigma.annihilates(F, S, p)
    Fo, delta_o, _ = sigma.min_generator(S[:L], p)
    assert sorted(d_dev.tolist()) == sorted(delta_o)
    if s <= 4:
        assert np.array_equal(sigma.popov_form(F, p), sigma.popov_form(Fo, p))


@pytest.mark.parametrize("L,s,p", [(2000, 8, 65521), (4100, 4, 2**31 - 1), (1500, 16, 65521), (37502, 8, 65521)])
def test_device_generator_long_random_sequences(L, s, p):
    """Random sequences of generic linear complexity: device = host PM-Basis, entry for entry."""
    torch = need_gpu()
    announce(f"device sigma-basis random L={L} s={s} p={p}")
    rng = np.random.default_rng(L)
    S = rng.integers(0, p, size=(L, s, s), dtype=np.int64)
    d_dev, P_dev = bw.min_generator_dev(to_dev(torch, S), p)
    d_host, P_host = bw.min_generator(S, p)
    assert np.array_equal(d_dev, d_host)
    assert np.array_equal(P_dev, P_host)


@pytest.mark.parametrize("L,s,p,min_chunk", [(2000, 8, 65521, 1), (2000, 8, 65521, 300), (701, 4, 2**31 - 1, 7),
                                             (1500, 16, 65521, 64), (90, 3, 65537, 2)])
def test_chunked_generator_equals_one_call(L, s, p, min_chunk, monkeypatch):
    """The online order (chunks [c_{i-1}, c_i) halving down to min_chunk, each chunk's basis composed onto
    the product of the earlier ones) gives the one-call PM-Basis generator entry for entry."""
    torch = need_gpu()
    announce(f"chunked device sigma-basis L={L} s={s} p={p} min_chunk={min_chunk}")
    rng = np.random.default_rng(L + min_chunk)
    S = rng.integers(0, p, size=(L, s, s), dtype=np.int64)
    d_host, P_host = bw.min_generator(S, p)
    monkeypatch.setenv("BWR_SIGMA_MIN_CHUNK", str(min_chunk))
    d_dev, P_dev = bw.min_generator_dev(to_dev(torch, S), p)
    assert np.array_equal(d_dev, d_host)
    assert np.array_equal(P_dev, P_host)


@pytest.mark.parametrize("primes,L,s", [((65521, 65519, 65497), 900, 8), ((2**31 - 1, 2147483629), 700, 4),
                                         ((65521, 65519, 65497, 40009), 300, 3), ((2**31 - 1,), 260, 8),
                                         ((40009, 3), 150, 16), ((65537, 1000003), 120, 16)])
def test_batched_generators_equal_single(primes, L, s):
    """Several sequences of one shape, one prime each, through one batched recursion: each generator equals
    the one the single-sequence device sigma-basis gives, entry for entry."""
    torch = need_gpu()
    announce(f"batched device sigma-basis primes={primes} L={L} s={s}")
    rng = np.random.default_rng(L + s)
    seqs = [rng.integers(0, p, size=(L, s, s), dtype=np.int64) for p in primes]
    devs = [to_dev(torch, S) for S in seqs]
    got = bw.min_generators_dev(devs, primes)
    for (d, P), S_dev, p in zip(got, devs, primes):
        d1, P1 = bw.min_generator_dev(S_dev, p)
        assert np.array_equal(d, d1)
        assert np.array_equal(P, P1)


def test_batched_generators_refuse_mixed_classes():
    torch = need_gpu()
    announce("batched device sigma-basis mixed prime classes")
    S = to_dev(torch, np.ones((40, 2, 2), dtype=np.int64))
    with pytest.raises(bw.BwrError):
        bw.min_generators_dev([S, S], (65521, 2**31 - 1))


def test_device_generator_zero_sequence():
    torch = need_gpu()
    announce("device sigma-basis zero sequence")
    S = np.zeros((12, 3, 3), dtype=np.int64)
    d, P = bw.min_generator_dev(to_dev(torch, S), 65521)
    assert d.tolist() == [0, 0, 0]


@pytest.mark.parametrize("where", ["device", "host"])
@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_rank_with_sigma_on_device_or_host(where, p, monkeypatch):
    need_gpu()
    announce(f"rank sigma on {where} p={p}")
    if where == "host":
        monkeypatch.setenv("BWR_HOST_SIGMA", "1")
    A = planted(3000, 2200, 1900, 9, 808)
    r, info = bw.rank_modp(A, p, 8, 4)
    assert r == native.rank_csr_c(A, p) == 1900
    assert (info["sigma_threads"] == 0) == (where == "device")


@pytest.mark.parametrize("min_chunk", [0, 1, 16, 100])
@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_rank_with_sigma_beside_sequence(min_chunk, p, monkeypatch):
    """The sigma-basis chunks that run on a second stream while the sequence is computed (each waits on
    an event after the terms it needs) give the rank of elimination; min_chunk 0 runs it afterwards."""
    need_gpu()
    announce(f"rank with online sigma min_chunk={min_chunk} p={p}")
    monkeypatch.setenv("BWR_SIGMA_MIN_CHUNK", str(min_chunk))
    A = planted(3000, 2200, 1900, 9, 809)
    r, info = bw.rank_modp(A, p, 8, 5)
    assert r == native.rank_csr_c(A, p) == 1900
