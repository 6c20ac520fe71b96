"""GPU parity of every row-split configuration of the sparse x block kernel
(lanes per row slice G, fused projection or not), forced through the
BWR_G1 / BWR_G2 overrides, and of the graph-captured step loop."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import coo_to_csr, planted

pytestmark = pytest.mark.gpu


def skewed_matrix(m, n, seed):
    """Rows of very different lengths (0 .. ~3n/4), including rows longer than 64 entries."""
    rng = np.random.default_rng(seed)
    lens = np.minimum(rng.geometric(0.08, size=m) - 1, (3 * n) // 4)
    lens[rng.integers(0, m, 5)] = min(n - 1, 150)
    lens[rng.integers(0, m, 5)] = 0
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([rng.choice(n, size=l, replace=False) for l in lens]) if lens.sum() else np.zeros(0)
    vals = rng.choice([-3, -2, -1, 1, 2, 3], size=rows.size)
    return coo_to_csr(m, n, rows, cols, vals)


CASES = []
for s in (3, 4, 8, 16, 32, 64):
    W = 4 if s <= 4 else s
    for g in (1, 2, 4, 8, 16):
        if (W // 4) * g > 64:
            continue
        fused = W % g == 0 and W // g <= 4
        CASES.append((s, g, fused))


@pytest.mark.parametrize("s,g,fused", CASES)
@pytest.mark.parametrize("p,e32", [(65521, "0"), (65521, "1"), (2**31 - 1, "0")])
def test_split_configurations(s, g, fused, p, e32, monkeypatch):
    """p = 65521 runs with 16-bit (e32 = 0) and 32-bit (e32 = 1) storage of the iterated blocks."""
    need_gpu()
    announce(f"split s={s} G={g} fused={fused} p={p} e32={e32}")
    monkeypatch.setenv("BWR_G1", str(g))
    monkeypatch.setenv("BWR_G2", str(g))
    monkeypatch.setenv("BWR_E32", e32)
    A = skewed_matrix(700, 300, s * 100 + g)
    rng = np.random.default_rng(g)
    U, V = blocks(rng, A.n, s, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 5, dr, dc)
    want = oseq.sequence(A, U, V, p, 5, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("graph", ["1", "0"])
def test_graph_and_stream_paths_agree(graph, monkeypatch):
    """1100 terms: the step loop is captured into a graph in chunks of 256 steps plus a tail."""
    need_gpu()
    announce(f"graph={graph} 1100 terms")
    monkeypatch.setenv("BWR_NO_GRAPH", "0" if graph == "1" else "1")
    p = 65521
    A = planted(900, 600, 500, 6, 44)
    rng = np.random.default_rng(9)
    U, V = blocks(rng, A.n, 8, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    got = bw.sequence(A, U, V, p, 1100, dr, dc)
    want = oseq.sequence(A, U, V, p, 1100, dr, dc)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("s,g", [(3, 1), (8, 2), (8, 4), (16, 4), (32, 1)])
@pytest.mark.parametrize("p,e32", [(2**31 - 1, "0"), (65537, "0"), (65521, "1")])
def test_two_column_passes(s, g, p, e32, monkeypatch):
    """Both products in two passes over the column halves (32-bit residues): same terms as the oracle,
    on rows of very different lengths, wide and tall shapes."""
    need_gpu()
    announce(f"column passes s={s} G={g} p={p} e32={e32}")
    monkeypatch.setenv("BWR_PARTS", "2")
    monkeypatch.setenv("BWR_G1", str(g))
    monkeypatch.setenv("BWR_G2", str(g))
    monkeypatch.setenv("BWR_E32", e32)
    for (m, n, seed) in ((700, 300, s + g), (301, 500, 7 * s + g)):
        A = skewed_matrix(m, n, seed)
        rng = np.random.default_rng(seed)
        U, V = blocks(rng, A.n, s, p)
        dr = rng.integers(1, p, size=A.m)
        dc = rng.integers(1, p, size=A.n)
        got = bw.sequence(A, U, V, p, 7, dr, dc)
        want = oseq.sequence(A, U, V, p, 7, dr, dc)
        assert np.array_equal(got.astype(np.int64), want), (m, n)
