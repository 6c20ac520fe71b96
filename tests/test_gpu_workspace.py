"""GPU parity of the caller-workspace forms (bwr_sequence_dev_ws,
bwr_rank_modp_dev_ws; Sections 2.2-2.3 and 2.5): every device buffer comes
from a torch-allocated workspace of the size bwr_*_workspace returns, the
library makes no device allocation during the call (its allocation count is
unchanged), and the results equal the oracle's element by element (sequence
terms) and elimination (ranks).  A workspace one byte short of what a call
needs fails cleanly with BWR_ENOMEM; a misaligned one with BWR_EINVAL."""
import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import ge
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import config1, coo_to_csr, planted

pytestmark = pytest.mark.gpu


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


def _ws(torch, nbytes):
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def big_values(m, n, seed):
    rng = np.random.default_rng(seed)
    nnz = 6 * m
    rows = rng.integers(0, m, nnz)
    cols = rng.integers(0, n, nnz)
    vals = rng.integers(-5000, 5000, nnz)
    return coo_to_csr(m, n, rows, cols, vals)


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
@pytest.mark.parametrize("case", ["planted", "wide", "config1"])
def test_sequence_workspace_equals_oracle(p, case):
    torch = need_gpu()
    announce(f"workspace sequence {case} p={p}")
    A = {"planted": lambda: planted(3000, 2000, 1700, 9, 71), "wide": lambda: big_values(1500, 1100, 72),
         "config1": config1}[case]()
    s = 8
    rng = np.random.default_rng(3)
    U, V = blocks(rng, A.n, s, p)
    dr = rng.integers(1, p, size=A.m)
    dc = rng.integers(1, p, size=A.n)
    Ad = bw.csr_to_device(A)
    need = bw.sequence_workspace(A.m, A.n, A.nnz, s)
    assert need > 0
    ws = _ws(torch, need)
    torch.cuda.synchronize()
    before = bw.device_allocations()
    S = bw.sequence_dev_ws(Ad, _t(torch, U), _t(torch, V), p, 70, _t(torch, dr), _t(torch, dc), workspace=ws)
    torch.cuda.synchronize()
    assert bw.device_allocations() == before
    got = S.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(got, oseq.sequence(A, U, V, p, 70, dr, dc))


def test_sequence_workspace_too_small_and_misaligned():
    torch = need_gpu()
    announce("workspace too small / misaligned")
    p, s = 65521, 4
    A = planted(600, 400, 300, 6, 9)
    rng = np.random.default_rng(1)
    U, V = blocks(rng, A.n, s, p)
    Ad = bw.csr_to_device(A)
    with pytest.raises(bw.BwrError) as ei:
        bw.sequence_dev_ws(Ad, _t(torch, U), _t(torch, V), p, 10, workspace=_ws(torch, 4096))
    assert ei.value.code == -3
    big = _ws(torch, bw.sequence_workspace(A.m, A.n, A.nnz, s) + 512)
    with pytest.raises(bw.BwrError) as ei:
        bw.sequence_dev_ws(Ad, _t(torch, U), _t(torch, V), p, 10, workspace=big[1:])
    assert ei.value.code == -1


@pytest.mark.parametrize("p", [65521, 2**31 - 1])
def test_rank_workspace_equals_elimination(p):
    """Both orientations (A and A^T swap roles when m < n), and a matrix with a large planted deficiency."""
    torch = need_gpu()
    announce(f"workspace rank p={p}")
    for A in (planted(2500, 1800, 1500, 9, 41), planted(1300, 1900, 1000, 8, 42), config1()):
        Ad = bw.csr_to_device(A)
        ws = _ws(torch, bw.rank_workspace(A.m, A.n, A.nnz, 8))
        torch.cuda.synchronize()
        before = bw.device_allocations()
        r, info = bw.rank_modp_dev_ws(Ad, p, 8, 1, workspace=ws)
        torch.cuda.synchronize()
        assert bw.device_allocations() == before
        assert r == A.planted_rank == ge.rank_csr(A, p)
        assert info["transposed"] == (1 if A.m < A.n else 0)
