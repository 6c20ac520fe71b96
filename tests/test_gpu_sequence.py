"""GPU parity of the sequence path against the oracle, element by element:
S_k = U^T B^k V and single applications of B = D_c A^T D_r A D_c
(Sections 2.2, 2.3 and step 2 of the rank algorithm in Section 2.5).
Integer work: the bar is bit-exact equality."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import coo_to_csr, config1, config2, planted, random_sparse

pytestmark = pytest.mark.gpu
PRIMES = (65521, 2**31 - 1, 65537, 3)


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8, 16, 32, 64])
def test_sequence_block_widths(s, p):
    need_gpu()
    announce(f"sequence planted(300,200) s={s} p={p}")
    rng = np.random.default_rng(s * 7 + p % 97)
    A = planted(300, 200, 150, 6, 1000 + s)
    U, V = blocks(rng, A.n, s, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 7, dr, dc)
    want = oseq.sequence(A, U, V, p, 7, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("sorted_enc", ["1", "0"])
@pytest.mark.parametrize("shape", [(700, 500, 420), (500, 700, 420)])
def test_sequence_with_and_without_length_sort(shape, sorted_enc, monkeypatch):
    """The rank path relabels rows and columns by length (and permutes the draws to match); the terms equal
    the oracle's either way, and so does the rank in both orientations."""
    need_gpu()
    announce(f"sequence length-sorted={sorted_enc} shape={shape}")
    if sorted_enc == "0":
        monkeypatch.setenv("BWR_NO_SORT", "1")
    p = 2**31 - 1
    m, n, r = shape
    A = planted(m, n, r, 9, 9100 + m)
    rng = np.random.default_rng(m)
    U, V = blocks(rng, A.n, 8, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 9, dr, dc)
    assert np.array_equal(got.astype(np.int64), oseq.sequence(A, U, V, p, 9, dr, dc))
    assert bw.rank_modp(A, p, 8, 3)[0] == r


@pytest.mark.parametrize("diag", ["none", "row", "col", "both"])
def test_sequence_diagonal_options(diag):
    need_gpu()
    announce(f"sequence diagonals={diag}")
    p = 65521
    rng = np.random.default_rng(3)
    A = planted(400, 250, 200, 7, 77)
    U, V = blocks(rng, A.n, 8, p)
    dr = rng.integers(1, p, size=A.m) if diag in ("row", "both") else None
    dc = rng.integers(1, p, size=A.n) if diag in ("col", "both") else None
    got = bw.sequence(A, U, V, p, 9, dr, dc)
    want = oseq.sequence(A, U, V, p, 9, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("shape", [(257, 129, 0.03), (1000, 3000, 0.002), (64, 64, 0.5), (1, 50, 0.3), (50, 1, 0.3),
                                   (2049, 1023, 0.004)])
def test_sequence_ragged_and_empty_rows(shape):
    need_gpu()
    m, n, dens = shape
    announce(f"sequence random_sparse {shape}")
    p = 65521
    rng = np.random.default_rng(m + n)
    A = random_sparse(m, n, dens, m * 31 + n, vmax=5)
    U, V = blocks(rng, n, 4, p)
    dr = rng.integers(1, p, size=m)
    got = bw.sequence(A, U, V, p, 6, dr)
    want = oseq.sequence(A, U, V, p, 6, dr)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
@pytest.mark.parametrize("vmax", [127, 128, 10**6, 2**31 - 1])
def test_sequence_large_values(p, vmax):
    """Values beyond int8 take the wide encoding (residues per prime)."""
    need_gpu()
    announce(f"sequence large values vmax={vmax} p={p}")
    rng = np.random.default_rng(vmax % 1000)
    m, n = 120, 90
    cnt = 900
    rows = rng.integers(0, m, cnt)
    cols = rng.integers(0, n, cnt)
    vals = rng.integers(-vmax, vmax, cnt, endpoint=True)
    A = coo_to_csr(m, n, rows, cols, vals)
    U, V = blocks(rng, n, 4, p)
    dc = rng.integers(1, p, size=n)
    got = bw.sequence(A, U, V, p, 5, None, dc)
    want = oseq.sequence(A, U, V, p, 5, None, dc)
    assert np.array_equal(got.astype(np.int64), want)


def test_sequence_duplicates_and_unsorted_columns():
    need_gpu()
    announce("sequence duplicate entries")
    p = 65521
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 40, 400)
    cols = rng.integers(0, 30, 400)
    vals = rng.integers(-3, 4, 400)
    A = coo_to_csr(40, 30, rows, cols, vals, coalesce=False)
    # shuffle the order inside each row
    for i in range(A.m):
        b, e = A.row_ptr[i], A.row_ptr[i + 1]
        perm = rng.permutation(e - b) + b
        A.col_idx[b:e] = A.col_idx[perm]
        A.val[b:e] = A.val[perm]
    U, V = blocks(rng, 30, 4, p)
    got = bw.sequence(A, U, V, p, 6)
    want = oseq.sequence(A, U, V, p, 6)
    assert np.array_equal(got.astype(np.int64), want)


def test_sequence_degenerate_shapes():
    need_gpu()
    announce("sequence degenerate shapes")
    p = 65521
    rng = np.random.default_rng(5)
    # all-zero matrix: S_k = 0 for k >= 1
    A = coo_to_csr(20, 10, [], [], [])
    U, V = blocks(rng, 10, 3, p)
    got = bw.sequence(A, U, V, p, 4)
    assert np.array_equal(got.astype(np.int64), oseq.sequence(A, U, V, p, 4))
    assert not got[1:].any()
    # no rows
    A = coo_to_csr(0, 10, [], [], [])
    got = bw.sequence(A, U, V, p, 3)
    assert np.array_equal(got.astype(np.int64), oseq.sequence(A, U, V, p, 3))
    # len 0 and len 1
    A = planted(30, 20, 15, 3, 3)
    U, V = blocks(rng, 20, 2, p)
    assert bw.sequence(A, U, V, p, 0).shape == (0, 2, 2)
    assert np.array_equal(bw.sequence(A, U, V, p, 1).astype(np.int64), oseq.sequence(A, U, V, p, 1))


def test_sequence_rejects_zero_column_scale():
    need_gpu()
    announce("sequence d_col with a zero entry")
    p = 65521
    A = planted(30, 20, 15, 3, 3)
    rng = np.random.default_rng(1)
    U, V = blocks(rng, 20, 2, p)
    dc = rng.integers(1, p, size=20)
    dc[4] = p  # = 0 mod p
    with pytest.raises(bw.BwrError) as ei:
        bw.sequence(A, U, V, p, 3, None, dc)
    assert ei.value.code == -1


def test_sequence_config1_all_terms():
    """2000 x 1500, planted rank 1200, s = 4, p = 65521: every one of the 756 terms."""
    need_gpu()
    announce("sequence config1 all terms")
    p = 65521
    A = config1()
    rng = np.random.default_rng(1)
    U, V = blocks(rng, A.n, 4, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    L = bw.sequence_length(A.n, 4) + 4
    got = bw.sequence(A, U, V, p, L, dr, dc)
    want = oseq.sequence(A, U, V, p, L, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_apply_config2_full_output(p):
    """One application of B at the 200k x 150k size, s = 8: all 1.2 M outputs."""
    torch = need_gpu()
    announce(f"apply config2 p={p}")
    A = config2()
    rng = np.random.default_rng(2)
    X = rng.integers(0, p, size=(A.n, 8), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    Ad = bw.csr_to_device(A)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()
    Z = bw.apply_dev(Ad, t(X), p, t(dr), t(dc))
    torch.cuda.synchronize()
    got = Z.cpu().numpy().view(np.uint32).astype(np.int64)
    want = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, dr, dc).apply(X)
    assert np.array_equal(got, want)


def test_sequence_dev_config2_first_terms():
    """Device entry point at the 200k x 150k size: first 4 terms."""
    torch = need_gpu()
    announce("sequence_dev config2")
    p = 65521
    A = config2()
    rng = np.random.default_rng(4)
    U, V = blocks(rng, A.n, 8, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    Ad = bw.csr_to_device(A)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()
    S = bw.sequence_dev(Ad, t(U), t(V), p, 4, t(dr), t(dc))
    torch.cuda.synchronize()
    got = S.cpu().numpy().view(np.uint32).astype(np.int64)
    want = oseq.sequence(A, U, V, p, 4, dr, dc)
    assert np.array_equal(got, want)
