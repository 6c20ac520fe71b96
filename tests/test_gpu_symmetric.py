"""GPU parity of the symmetric projection U = V (Section 2.3): S_k = V^T B^k V
element by element against the oracle's sequence with U = V, formed as the
independent projection with its symmetry check, and in Gram form (two terms per
application of B, the identities S_2k = W_k^T W_k, S_2k+1 = (A D_c W_k)^T D_r
(A D_c W_k); not in the paper), over block sizes, both residue widths, even and
odd lengths, graph-captured chunks, the tiled and row-split products, identity
and zero-containing diagonals; then ranks against elimination."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge
from oracle import sequence as oseq
from tests.gpu_util import announce, need_gpu
from workloads import config1, config2, planted

pytestmark = pytest.mark.gpu


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


def _run(torch, A, V, p, L, dr, dc, gram):
    Ad = bw.csr_to_device(A)
    S = bw.sequence_sym_dev(Ad, _t(torch, V), p, L, None if dr is None else _t(torch, dr),
                            None if dc is None else _t(torch, dc), gram=gram)
    torch.cuda.synchronize()
    return S.cpu().numpy().view(np.uint32).astype(np.int64)


@pytest.mark.parametrize("tiled", ["0", "1"])
@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("s", [1, 3, 8, 16])
@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_symmetric_terms(gram, s, p, tiled, monkeypatch):
    """tiled = 1: both products tiled (small row blocks and slabs), the Gram terms formed in their epilogues."""
    torch = need_gpu()
    announce(f"symmetric gram={gram} s={s} p={p} tiled={tiled}")
    monkeypatch.setenv("BWR_TILED", tiled)
    monkeypatch.setenv("BWR_TILED_R", "64")
    monkeypatch.setenv("BWR_TILED_SLAB", "1024")
    A = planted(700, 500, 420, 7, 100 + s)
    rng = np.random.default_rng(s)
    V = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    for L in (9, 10):
        got = _run(torch, A, V, p, L, dr, dc, gram)
        want = oseq.sequence(A, V, V, p, L, dr, dc)
        assert np.array_equal(got, want), L
        assert np.array_equal(got, np.transpose(got, (0, 2, 1)))


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("tiled", ["1", "0"])
def test_symmetric_graph_chunks_and_kernels(gram, tiled, monkeypatch):
    """601 terms (graph chunks of the Gram loop and a ragged tail), tiled or row-split products."""
    torch = need_gpu()
    announce(f"symmetric long gram={gram} tiled={tiled}")
    monkeypatch.setenv("BWR_TILED", tiled)
    if tiled == "1":
        monkeypatch.setenv("BWR_TILED_R", "128")
        monkeypatch.setenv("BWR_TILED_SLAB", "2048")
    p = 65521
    A = planted(1500, 1000, 900, 8, 55)
    rng = np.random.default_rng(2)
    V = rng.integers(0, p, size=(A.n, 8), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = _run(torch, A, V, p, 601, dr, dc, gram)
    assert np.array_equal(got, oseq.sequence(A, V, V, p, 601, dr, dc))


@pytest.mark.parametrize("gram", [False, True])
def test_symmetric_identity_and_zero_diagonals(gram):
    """No diagonals (identity), and a row diagonal with entries divisible by p (those rows weigh 0)."""
    torch = need_gpu()
    announce(f"symmetric diagonals gram={gram}")
    p = 65521
    A = planted(400, 300, 250, 6, 7)
    rng = np.random.default_rng(9)
    V = rng.integers(0, p, size=(A.n, 4), dtype=np.int64)
    assert np.array_equal(_run(torch, A, V, p, 12, None, None, gram), oseq.sequence(A, V, V, p, 12))
    dr = rng.integers(1, p, size=A.m)
    dr[::7] = p
    dc = rng.integers(1, p, size=A.n)
    assert np.array_equal(_run(torch, A, V, p, 12, dr, dc, gram), oseq.sequence(A, V, V, p, 12, dr, dc))


@pytest.mark.parametrize("gram", [False, True])
@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_symmetric_ranks_equal_elimination(gram, p):
    """The 2000 x 1500 and 200000 x 150000 matrices, and a wide matrix (A and A^T swap roles)."""
    need_gpu()
    announce(f"symmetric ranks gram={gram} p={p}")
    A = config1()
    assert bw.rank_modp_sym(A, p, 4, 1, gram)[0] == 1200 == ge.rank_csr(A, p)
    B = planted(900, 1300, 700, 6, 31)
    r, info = bw.rank_modp_sym(B, p, 8, 1, gram)
    assert info["transposed"] == 1 and r == 700
    C = config2()
    assert bw.rank_modp_sym(C, p, 8, 1, gram)[0] == C.planted_rank
