"""GPU parity at the paper-scale shape: the planted 2 000 000 x 1 000 000
matrix (37.2 M non-zeros, rank 900 000), block 16, p = 65521 (step 2 of the
block Wiedemann rank algorithm, Section 2.5, at the size of the paper's largest
matrices).  Sequence terms S_0 .. S_3 element by element against the oracle
under explicit U, V, D_r, D_c, through the autotuned plan of a kept matrix
(bwr_matrix_sequence_dev), the forced tiled products and the row-split
products; one application of B on all 16 M outputs through the tiled kernels;
and the whole rank, which must equal the planted rank exactly."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import config3

pytestmark = pytest.mark.gpu

P = 65521
S_BLOCK = 16


@pytest.fixture(scope="module")
def c3():
    torch = need_gpu()
    announce("paper scale: generating the 2000000 x 1000000 matrix and the oracle's first terms")
    A = config3()
    rng = np.random.default_rng(33)
    U, V = blocks(rng, A.n, S_BLOCK, P)
    dr = rng.integers(1, P, size=A.m)
    dc = rng.integers(1, P, size=A.n)
    orc = oseq.Oracle(A.m, A.n, A.row_ptr, A.col_idx, A.val, P, dr, dc)
    S = orc.sequence(U, V, 4)
    Ad = bw.csr_to_device(A)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()
    return {"A": A, "orc": orc, "S": S, "Ad": Ad, "U": U, "V": V, "dU": t(U), "dV": t(V), "ddr": t(dr), "ddc": t(dc),
            "torch": torch}


def _got(S):
    return S.cpu().numpy().view(np.uint32).astype(np.int64)


def test_c3_terms_autotuned_kept_matrix(c3):
    """66 terms with the plan the autotuner picks (the benchmark's kernels); the first 4 against the oracle."""
    announce("paper scale: autotuned plan, kept matrix")
    M = bw.Matrix(c3["Ad"], P)
    try:
        S = M.sequence_dev(c3["dU"], c3["dV"], P, 66, c3["ddr"], c3["ddc"])
        c3["torch"].cuda.synchronize()
        got = _got(S)
    finally:
        M.close()
    assert np.array_equal(got[:4], c3["S"])


@pytest.mark.parametrize("tiled", ["1", "0"])
def test_c3_terms_tiled_and_row_split(c3, tiled, monkeypatch):
    """S_0 .. S_3 with both products forced tiled (default geometry), and with the row-split kernels."""
    announce(f"paper scale: 4 terms, BWR_TILED={tiled}")
    monkeypatch.setenv("BWR_TILED", tiled)
    S = bw.sequence_dev(c3["Ad"], c3["dU"], c3["dV"], P, 4, c3["ddr"], c3["ddc"])
    c3["torch"].cuda.synchronize()
    assert np.array_equal(_got(S), c3["S"])


def test_c3_apply_full_output_tiled(c3, monkeypatch):
    """One application of B through the tiled kernels: all 1 000 000 x 16 outputs."""
    announce("paper scale: one application of B, tiled")
    monkeypatch.setenv("BWR_TILED", "1")
    Z = bw.apply_dev(c3["Ad"], c3["dV"], P, c3["ddr"], c3["ddc"])
    c3["torch"].cuda.synchronize()
    want = c3["orc"].apply(c3["V"])
    assert np.array_equal(_got(Z), want)


@pytest.mark.timeout(900)
def test_c3_rank_equals_planted(c3):
    """The whole rank (2 + 2n/16 + 4 = 125006 terms, sigma-basis, read-out) equals the planted 900000."""
    announce("paper scale: whole rank")
    r, info = bw.rank_modp_dev(c3["Ad"], P, S_BLOCK, 1)
    print(f"[gpu-case] paper-scale rank {r} in {info['t_sequence']:.1f} s sequence + {info['t_sigma']:.2f} s "
          f"sigma-basis + {info['t_readout']:.2f} s read-out", flush=True)
    assert r == 900000 == c3["A"].planted_rank
