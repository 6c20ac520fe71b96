"""GPU parity of the two-dimensional tiled sparse x block product (row blocks
accumulated in LDS, the gathered block read slab by slab), forced through
BWR_TILED=1: sequence terms and one application of B against the oracle,
element by element, for every block width, both residue widths and both
accumulator forms (int32 sums for p <= 2^16, 16-bit halves above), with small
row blocks, small slabs and fewer workgroups than row blocks so that every
tile boundary, the ragged last row block and the grid-stride loop are hit;
then the default geometry and ranks against elimination."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import coo_to_csr, config1, planted

pytestmark = pytest.mark.gpu


def skewed_matrix(m, n, seed):
    """Rows of very different lengths (0 .. ~3n/4), a few empty rows and empty columns."""
    rng = np.random.default_rng(seed)
    lens = np.minimum(rng.geometric(0.08, size=m) - 1, (3 * n) // 4)
    lens[rng.integers(0, m, 5)] = min(n - 1, 150)
    lens[rng.integers(0, m, 5)] = 0
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([rng.choice(n - 7, size=l, replace=False) for l in lens]) if lens.sum() else np.zeros(0)
    vals = rng.choice([-3, -2, -1, 1, 2, 3], size=rows.size)
    return coo_to_csr(m, n, rows, cols, vals)


def small_tiles(monkeypatch, W, esize):
    monkeypatch.setenv("BWR_TILED", "1")
    monkeypatch.setenv("BWR_TILED_R", "64")
    monkeypatch.setenv("BWR_TILED_SLAB", str(16 * W * esize))  # 16 block rows per slab
    monkeypatch.setenv("BWR_TILED_GRID", "3")


@pytest.mark.parametrize("s", [3, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("p,e32", [(65521, "0"), (65521, "1"), (2**31 - 1, "0")])
def test_tiled_small_tiles(s, p, e32, monkeypatch):
    need_gpu()
    announce(f"tiled small tiles s={s} p={p} e32={e32}")
    W = 4 if s <= 4 else s
    esize = 2 if (p <= 65536 and e32 == "0") else 4
    small_tiles(monkeypatch, W, esize)
    monkeypatch.setenv("BWR_E32", e32)
    A = skewed_matrix(700, 300, 31 * s + (p & 7))
    rng = np.random.default_rng(s)
    U, V = blocks(rng, A.n, s, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 5, dr, dc)
    want = oseq.sequence(A, U, V, p, 5, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


def sparse_blocks_matrix(m, n, row_step, col_step, seed):
    """Entries only in rows r = 0 mod row_step and columns c = 0 mod col_step: with row_step a multiple of the
    number of row blocks, every row block but the first has no entries."""
    rng = np.random.default_rng(seed)
    rs = np.arange(0, m, row_step)
    cs = np.arange(0, n, col_step)
    rows = np.repeat(rs, 6)
    cols = rng.choice(cs, size=rows.size)
    vals = rng.choice([-2, -1, 1, 3], size=rows.size)
    return coo_to_csr(m, n, rows, cols, vals)


@pytest.mark.parametrize("p,s", [(65521, 16), (65521, 8), (2**31 - 1, 16)])
@pytest.mark.parametrize("shape", ["empty-row-blocks", "rowless-row-block", "many-slabs"])
def test_tiled_row_block_edges(shape, p, s, monkeypatch):
    """Row-block starts: row blocks with no entries (700 x 300, entries in rows 0 mod 12 and columns 0 mod 6, 12
    and 6 row blocks), a row block with no rows (2 x 40: 3 row blocks for 2 rows), and more slabs than threads
    of a workgroup (600 x 20000, 16 block rows a slab: 1250 slabs in the first product), each over several row
    blocks per workgroup; 5 terms against the oracle."""
    need_gpu()
    announce(f"tiled row-block edges {shape} s={s} p={p}")
    W = s
    small_tiles(monkeypatch, W, 2 if p <= 65536 else 4)
    if shape == "empty-row-blocks":
        A = sparse_blocks_matrix(700, 300, 12, 6, 5)
    elif shape == "rowless-row-block":
        A = sparse_blocks_matrix(2, 40, 1, 1, 6)
    else:
        A = sparse_blocks_matrix(600, 20000, 1, 1, 7)
    rng = np.random.default_rng(s + 1)
    U, V = blocks(rng, A.n, s, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 5, dr, dc)
    want = oseq.sequence(A, U, V, p, 5, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_tiled_graph_chunks(p, monkeypatch):
    """600 terms: captured 256-step graphs replayed with the tiled kernels, then a tail."""
    need_gpu()
    announce(f"tiled graph chunks p={p}")
    small_tiles(monkeypatch, 8, 2 if p <= 65536 else 4)
    A = planted(900, 600, 500, 7, 77)
    rng = np.random.default_rng(9)
    U, V = blocks(rng, A.n, 8, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 600, dr, dc)
    want = oseq.sequence(A, U, V, p, 600, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
@pytest.mark.parametrize("s", [8, 16])
def test_tiled_apply_full_output(p, s, monkeypatch):
    """One application of B through the tiled kernels (32-bit residues): every output entry."""
    torch = need_gpu()
    announce(f"tiled apply p={p} s={s}")
    monkeypatch.setenv("BWR_TILED", "1")
    monkeypatch.setenv("BWR_TILED_R", "128")
    monkeypatch.setenv("BWR_TILED_SLAB", str(64 * s * 4))
    A = planted(30000, 20000, 17000, 9, 4242)
    rng = np.random.default_rng(3)
    X = rng.integers(0, p, size=(A.n, s), dtype=np.int64)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    Ad = bw.csr_to_device(A)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()
    Z = bw.apply_dev(Ad, t(X), p, t(dr), t(dc))
    torch.cuda.synchronize()
    got = Z.cpu().numpy().view(np.uint32).astype(np.int64)
    want = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, dr, dc).apply(X)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_tiled_default_geometry(p, monkeypatch):
    """Default geometry (one round of row blocks over every CU, slabs of 128 KB of the block) on a matrix
    with fewer rows than one LDS-sized row block per CU holds: 6 terms."""
    need_gpu()
    announce(f"tiled default geometry p={p}")
    monkeypatch.setenv("BWR_TILED", "1")
    A = planted(120000, 90000, 80000, 9, 99)
    rng = np.random.default_rng(5)
    U, V = blocks(rng, A.n, 16, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 6, dr, dc)
    want = oseq.sequence(A, U, V, p, 6, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_tiled_ranks_equal_elimination(p, monkeypatch):
    """Ranks through the tiled kernels: the 2000 x 1500 matrix and a wide matrix (A and A^T swap roles)."""
    need_gpu()
    announce(f"tiled ranks p={p}")
    monkeypatch.setenv("BWR_TILED", "1")
    monkeypatch.setenv("BWR_TILED_R", "256")
    A = config1()
    r, _ = bw.rank_modp(A, p, 4, 1)
    assert r == 1200 == ge.rank_csr(A, p)
    B = planted(900, 1300, 700, 6, 31)  # m < n: B acts on the row side
    r2, info = bw.rank_modp(B, p, 8, 1)
    assert info["transposed"] == 1
    assert r2 == 700 == ge.rank_csr(B, p)


@pytest.mark.parametrize("un,stage", [(1, "1"), (2, "1"), (3, "0"), (4, "1"), (4, "0")])
@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_tiled_entries_in_flight(un, stage, p, monkeypatch):
    """1 .. 4 entries per lane per pass, the projection's operands staged in LDS or loaded directly
    (BWR_TILED_NO_STAGE): row blocks of about 64 rows, 96 workgroups over 512 row blocks (grid-stride rounds
    of unequal length); 6 terms and one application of B against the oracle, then a graph-replayed 300-term
    run with row blocks of 16 rows."""
    torch = need_gpu()
    announce(f"tiled entries per pass un={un} stage={stage} p={p}")
    if stage == "0":
        monkeypatch.setenv("BWR_TILED_NO_STAGE", "1")
    monkeypatch.setenv("BWR_TILED", "1")
    monkeypatch.setenv("BWR_TILED_R", "64")
    monkeypatch.setenv("BWR_TILED_SLAB", str(256 * 16 * 4))
    monkeypatch.setenv("BWR_TILED_GRID", "96")
    monkeypatch.setenv("BWR_TILED_UN", str(un))
    A = planted(30000, 20000, 17000, 9, 4343)
    rng = np.random.default_rng(un)
    U, V = blocks(rng, A.n, 16, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 6, dr, dc)
    orc = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, p, dr, dc)
    assert np.array_equal(got.astype(np.int64), orc.sequence(U, V, 6))
    Ad = bw.csr_to_device(A)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()
    Z = bw.apply_dev(Ad, t(V), p, t(dr), t(dc))
    torch.cuda.synchronize()
    assert np.array_equal(Z.cpu().numpy().view(np.uint32).astype(np.int64), orc.apply(V))
    B = planted(3000, 2200, 1900, 7, 4444)
    monkeypatch.setenv("BWR_TILED_R", "16")
    monkeypatch.setenv("BWR_TILED_SLAB", str(16 * 8 * 4))
    U8, V8 = blocks(rng, B.n, 8, p)
    got = bw.sequence(B, U8, V8, p, 300)
    assert np.array_equal(got.astype(np.int64), oseq.sequence(B, U8, V8, p, 300))
