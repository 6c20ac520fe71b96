"""The sequence entry point that allocates nothing (bwr_sequence_dev_noalloc):
two calls in a row through the C-ABI, the second on a smaller matrix, each
equal to the allocating bwr_sequence_dev element by element (and to the
oracle), with the library's device allocation count unchanged; and a matrix
beyond the static scratch refused before any device work."""
import ctypes

import numpy as np
import pytest

import paper_0704_2351_amd as bw
from oracle import sequence as oseq
from tests.gpu_util import announce, blocks, need_gpu
from workloads import planted

pytestmark = pytest.mark.gpu


def _t(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64).astype(np.uint32).view(np.int32)).cuda()


def test_noalloc_two_calls_match_allocating_entry():
    torch = need_gpu()
    cases = [(planted(3000, 2200, 1900, 9, 5), 8, 65521, 40), (planted(800, 600, 500, 7, 6), 4, 2**31 - 1, 25)]
    for A, s, p, L in cases:
        announce(f"no-alloc sequence {A.m}x{A.n} s={s} p={p}")
        rng = np.random.default_rng(s)
        U, V = blocks(rng, A.n, s, p)
        dr = rng.integers(1, p, size=A.m)
        dc = rng.integers(1, p, size=A.n)
        Ad = bw.csr_to_device(A)
        dU, dV, ddr, ddc = _t(torch, U), _t(torch, V), _t(torch, dr), _t(torch, dc)
        out = torch.empty((L, s, s), dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        before = bw.device_allocations()
        bw.sequence_dev_noalloc(Ad, dU, dV, p, L, ddr, ddc, out=out)
        torch.cuda.synchronize()
        assert bw.device_allocations() == before
        got = out.cpu().numpy().view(np.uint32).astype(np.int64)
        ref = bw.sequence_dev(Ad, dU, dV, p, L, ddr, ddc)
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.cpu().numpy().view(np.uint32).astype(np.int64))
        assert np.array_equal(got, oseq.sequence(A, U, V, p, L, dr, dc))


def test_noalloc_refuses_matrices_beyond_the_scratch():
    """The size check runs on the host from the CSR's sizes, before anything touches the device arrays."""
    need_gpu()
    announce("no-alloc size limit")
    big = bw.binding.CSRStruct(20_000_000, 10_000_000, 300_000_000, None, None, None)
    code = bw.lib().bwr_sequence_dev_noalloc(ctypes.byref(big), None, None, None, None, 65521, 8, 10, None, None)
    assert code == -1
    assert "too large" in bw.lib().bwr_last_error().decode()
