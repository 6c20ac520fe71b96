"""ctypes binding of libbwrank.so: argument marshalling only.

Every function forwards to the C-ABI of the same name (include/bwrank.h).
Host variants take numpy arrays; ``*_dev`` variants take torch tensors that
live on a HIP device and use torch's current stream.  There is no Python or
CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbwrank.so")

BWR_OK, BWR_EINVAL, BWR_EPRIME, BWR_ENOMEM, BWR_EDEVICE, BWR_EBUSY, BWR_ESHORT = 0, -1, -2, -3, -4, -5, -6
EXPORTED = ("bwr_version", "bwr_last_error", "bwr_is_prime", "bwr_sequence_length", "bwr_set_threads",
            "bwr_random_block", "bwr_sequence", "bwr_sequence_dev", "bwr_apply_dev", "bwr_rank_modp",
            "bwr_rank_modp_dev", "bwr_min_generator", "bwr_rank_from_sequence", "bwr_time_step_kernels_dev",
            "bwr_min_generator_dev", "bwr_min_generators_dev", "bwr_rank_modp_batch", "bwr_rank_integer", "bwr_sequence_batch", "bwr_server_create",
            "bwr_server_submit", "bwr_server_poll", "bwr_server_wait", "bwr_server_get_stats", "bwr_server_destroy",
            "bwr_matrix_create_dev", "bwr_matrix_sequence_dev", "bwr_matrix_destroy", "bwr_set_trials",
            "bwr_get_trials", "bwr_sequence_workspace", "bwr_rank_workspace", "bwr_sequence_dev_ws",
            "bwr_rank_modp_dev_ws", "bwr_device_allocations", "bwr_sequence_sym_dev", "bwr_rank_modp_sym",
            "bwr_rank_modp_sym_dev", "bwr_matrix_sequence_sym_dev", "bwr_sequence_dev_noalloc",
            "bwr_set_early_termination", "bwr_get_early_termination", "bwr_set_batch_retry",
            "bwr_get_batch_retry")


class BwrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bwrank error {code}: {msg}")
        self.code = code


class CSRStruct(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("t_encode", ctypes.c_double), ("t_sequence", ctypes.c_double), ("t_sigma", ctypes.c_double),
                ("t_total", ctypes.c_double), ("steps", ctypes.c_int64), ("jobs", ctypes.c_int32),
                ("width", ctypes.c_int32), ("g1", ctypes.c_int32), ("g2", ctypes.c_int32),
                ("retries", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RankInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("nb", ctypes.c_int64), ("s", ctypes.c_int32),
                ("transposed", ctypes.c_int32), ("len", ctypes.c_int64), ("check_terms", ctypes.c_int64),
                ("sum_delta", ctypes.c_int64), ("t_encode", ctypes.c_double), ("t_sequence", ctypes.c_double),
                ("t_sigma", ctypes.c_double), ("t_readout", ctypes.c_double), ("sigma_threads", ctypes.c_int32),
                ("trials", ctypes.c_int32), ("terms", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libbwrank.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0704_2351_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "bwr_version": (ctypes.c_int, []),
            "bwr_last_error": (ctypes.c_char_p, []),
            "bwr_is_prime": (ctypes.c_int, [u32]),
            "bwr_sequence_length": (i64, [i64, i32]),
            "bwr_set_threads": (ctypes.c_int, [i32]),
            "bwr_set_trials": (ctypes.c_int, [i32]),
            "bwr_get_trials": (i32, []),
            "bwr_set_early_termination": (ctypes.c_int, [i32]),
            "bwr_get_early_termination": (i32, []),
            "bwr_set_batch_retry": (ctypes.c_int, [i32]),
            "bwr_get_batch_retry": (i32, []),
            "bwr_random_block": (ctypes.c_int, [u64, i32, i64, i32, u32, i32, vp]),
            "bwr_sequence": (ctypes.c_int, [vp, vp, vp, vp, vp, u32, i32, i64, vp]),
            "bwr_sequence_dev": (ctypes.c_int, [vp, vp, vp, vp, vp, u32, i32, i64, vp, vp]),
            "bwr_apply_dev": (ctypes.c_int, [vp, vp, vp, vp, u32, i32, vp, vp]),
            "bwr_rank_modp": (ctypes.c_int, [vp, u32, i32, u64, vp, vp]),
            "bwr_rank_modp_dev": (ctypes.c_int, [vp, u32, i32, u64, vp, vp, vp]),
            "bwr_min_generator": (ctypes.c_int, [vp, i64, i32, u32, vp, vp, i64, vp]),
            "bwr_rank_from_sequence": (ctypes.c_int, [vp, i64, i64, i32, u32, vp]),
            "bwr_time_step_kernels_dev": (ctypes.c_int, [vp, u32, i32, i32, i32, vp, vp, vp]),
            "bwr_min_generator_dev": (ctypes.c_int, [vp, i64, i32, u32, vp, vp, vp, i64, vp]),
            "bwr_min_generators_dev": (ctypes.c_int, [vp, i32, i64, i32, vp, vp, vp, vp, i64, vp]),
            "bwr_rank_integer": (ctypes.c_int, [vp, vp, i32, i32, u64, vp, vp]),
            "bwr_rank_modp_batch": (ctypes.c_int, [vp, i32, vp, i32, i32, u64, vp, vp]),
            "bwr_sequence_batch": (ctypes.c_int, [vp, i32, vp, i32, i32, u64, vp, vp]),
            "bwr_server_create": (ctypes.c_int, [u64, i32, i32, vp]),
            "bwr_server_submit": (ctypes.c_int, [vp, vp, u32, u64, vp]),
            "bwr_server_poll": (ctypes.c_int, [vp, u64, vp, vp]),
            "bwr_server_wait": (ctypes.c_int, [vp, u64, vp]),
            "bwr_server_get_stats": (ctypes.c_int, [vp, vp]),
            "bwr_server_destroy": (None, [vp]),
            "bwr_matrix_create_dev": (ctypes.c_int, [vp, u32, vp, vp]),
            "bwr_matrix_sequence_dev": (ctypes.c_int, [vp, vp, vp, vp, vp, u32, i32, i64, vp, vp]),
            "bwr_matrix_destroy": (None, [vp]),
            "bwr_sequence_workspace": (ctypes.c_size_t, [i64, i64, i64, i32]),
            "bwr_device_allocations": (i64, []),
            "bwr_sequence_sym_dev": (ctypes.c_int, [vp, vp, vp, vp, u32, i32, i64, i32, vp, vp]),
            "bwr_rank_modp_sym": (ctypes.c_int, [vp, u32, i32, u64, i32, vp, vp]),
            "bwr_rank_modp_sym_dev": (ctypes.c_int, [vp, u32, i32, u64, i32, vp, vp, vp]),
            "bwr_matrix_sequence_sym_dev": (ctypes.c_int, [vp, vp, vp, vp, u32, i32, i64, i32, vp, vp]),
            "bwr_sequence_dev_noalloc": (ctypes.c_int, [vp, vp, vp, vp, vp, u32, i32, i64, vp, vp]),
            "bwr_rank_workspace": (ctypes.c_size_t, [i64, i64, i64, i32]),
            "bwr_sequence_dev_ws": (ctypes.c_int, [vp, vp, vp, vp, vp, u32, i32, i64, vp, vp, ctypes.c_size_t, vp]),
            "bwr_rank_modp_dev_ws": (ctypes.c_int, [vp, u32, i32, u64, vp, ctypes.c_size_t, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int):
    if code != BWR_OK:
        raise BwrError(code, lib().bwr_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data


def _u32(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.uint32)
    if shape is not None and a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} entries, got {a.shape}")
    return a


def _host_csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col_idx, dtype=np.int32)
    vv = np.ascontiguousarray(A.val, dtype=np.int32)
    st = CSRStruct(int(A.m), int(A.n), int(rp[-1]) if rp.size else 0, rp.ctypes.data, ci.ctypes.data,
                   vv.ctypes.data)
    return st, (rp, ci, vv)


# ------------------------------------------------------------------ host-side helpers
def version() -> int:
    return lib().bwr_version()


def is_prime(p: int) -> bool:
    return bool(lib().bwr_is_prime(int(p)))


def sequence_length(nb: int, s: int) -> int:
    return int(lib().bwr_sequence_length(int(nb), int(s)))


def set_threads(n: int) -> None:
    _check(lib().bwr_set_threads(int(n)))


def set_trials(n: int) -> None:
    """Independent draws per rank computation (the largest rank over the draws is kept)."""
    _check(lib().bwr_set_trials(int(n)))


def get_trials() -> int:
    return int(lib().bwr_get_trials())


def set_early_termination(on: bool) -> None:
    """Stop single-matrix rank sequences once the device sigma-basis beside them has converged."""
    _check(lib().bwr_set_early_termination(1 if on else 0))


def get_early_termination() -> bool:
    return bool(lib().bwr_get_early_termination())


def set_batch_retry(n: int) -> None:
    """Further draws (up to n) for a batched (matrix, prime) whose rank is below the matrix's largest rank."""
    _check(lib().bwr_set_batch_retry(int(n)))


def get_batch_retry() -> int:
    return int(lib().bwr_get_batch_retry())


def random_block(seed: int, stream: int, rows: int, s: int, p: int, diag: bool = False) -> np.ndarray:
    out = np.zeros(max(rows * s, 1), dtype=np.uint32)
    _check(lib().bwr_random_block(int(seed), int(stream), int(rows), int(s), int(p), int(diag), out.ctypes.data))
    return out[: rows * s].reshape(rows, s)


# ------------------------------------------------------------------ host-pointer entry points
def sequence(A, U, V, p: int, length: int, d_row=None, d_col=None) -> np.ndarray:
    """S_k = U^T (D_c A^T D_r A D_c)^k V mod p, k < length; returns (length, s, s) uint32."""
    st, keep = _host_csr(A)
    U = _u32(U)
    s = U.shape[1]
    V = _u32(V, (A.n, s))
    U = _u32(U, (A.n, s))
    dr = _u32(d_row, (A.m,))
    dc = _u32(d_col, (A.n,))
    out = np.zeros(max(length * s * s, 1), dtype=np.uint32)
    _check(lib().bwr_sequence(ctypes.byref(st), _ptr(dr), _ptr(dc), _ptr(U), _ptr(V), int(p), int(s),
                              int(length), out.ctypes.data))
    return out[: length * s * s].reshape(length, s, s)


def rank_modp(A, p: int, block: int, seed: int):
    """(rank, info dict) of A over GF(p) by block Wiedemann (host CSR input)."""
    st, keep = _host_csr(A)
    r = ctypes.c_int64(0)
    info = RankInfo()
    _check(lib().bwr_rank_modp(ctypes.byref(st), int(p), int(block), int(seed), ctypes.byref(r), ctypes.byref(info)))
    return int(r.value), info.as_dict()


def min_generator(S, p: int):
    """(delta, P) of the minimal generator of S (len, s, s); P has shape (max_deg + 1, s, s)."""
    S = _u32(S)
    L, s, _ = S.shape
    delta = np.zeros(s, dtype=np.int64)
    P = np.zeros((L + 2) * s * s, dtype=np.uint32)
    md = ctypes.c_int64(0)
    _check(lib().bwr_min_generator(S.ctypes.data, int(L), int(s), int(p), delta.ctypes.data, P.ctypes.data,
                                   int(L + 2), ctypes.byref(md)))
    return delta, P[: (md.value + 1) * s * s].reshape(md.value + 1, s, s)


def rank_from_sequence(S, length: int, check: int, p: int) -> int:
    S = _u32(S)
    s = S.shape[1]
    if S.shape[0] < length + check:
        raise ValueError("S holds fewer than length + check terms")
    r = ctypes.c_int64(0)
    _check(lib().bwr_rank_from_sequence(S.ctypes.data, int(length), int(check), int(s), int(p), ctypes.byref(r)))
    return int(r.value)


# ------------------------------------------------------------------ device entry points (torch tensors)
def _torch():
    import torch
    return torch


def csr_to_device(A, device="cuda"):
    """Copy a host CSR to device tensors: dict(m, n, nnz, row_ptr, col_idx, val)."""
    torch = _torch()
    return {
        "m": int(A.m), "n": int(A.n), "nnz": int(A.row_ptr[-1]) if len(A.row_ptr) else 0,
        "row_ptr": torch.from_numpy(np.ascontiguousarray(A.row_ptr, dtype=np.int64)).to(device),
        "col_idx": torch.from_numpy(np.ascontiguousarray(A.col_idx, dtype=np.int32)).to(device),
        "val": torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.int32)).to(device),
    }


def _dev_csr(Ad):
    for k in ("row_ptr", "col_idx", "val"):
        t = Ad[k]
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{k} must be a contiguous device tensor")
    return CSRStruct(Ad["m"], Ad["n"], Ad["nnz"], Ad["row_ptr"].data_ptr(), Ad["col_idx"].data_ptr(),
                     Ad["val"].data_ptr())


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def sequence_dev(Ad, U, V, p: int, length: int, d_row=None, d_col=None, out=None):
    """Device sequence: U, V (n, s) uint32/int32 device tensors; returns (length, s, s) device tensor."""
    torch = _torch()
    st = _dev_csr(Ad)
    s = U.shape[1]
    if out is None:
        out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=U.device)
    _check(lib().bwr_sequence_dev(ctypes.byref(st), _dptr(d_row), _dptr(d_col), _dptr(U), _dptr(V), int(p), int(s),
                                  int(length), _dptr(out), _stream()))
    return out[:length]


class Matrix:
    """A device CSR encoded once (bwr_matrix_create_dev) for several sequences (bwr_matrix_sequence_dev)."""

    def __init__(self, Ad, p: int):
        st = _dev_csr(Ad)
        h = ctypes.c_void_p()
        _check(lib().bwr_matrix_create_dev(ctypes.byref(st), int(p), _stream(), ctypes.byref(h)))
        self._h = h

    def sequence_dev(self, U, V, p: int, length: int, d_row=None, d_col=None, out=None):
        torch = _torch()
        s = U.shape[1]
        if out is None:
            out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=U.device)
        _check(lib().bwr_matrix_sequence_dev(self._h, _dptr(d_row), _dptr(d_col), _dptr(U), _dptr(V), int(p), int(s),
                                             int(length), _dptr(out), _stream()))
        return out[:length]

    def sequence_sym_dev(self, V, p: int, length: int, d_row=None, d_col=None, gram: bool = False, out=None):
        torch = _torch()
        s = V.shape[1]
        if out is None:
            out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=V.device)
        _check(lib().bwr_matrix_sequence_sym_dev(self._h, _dptr(d_row), _dptr(d_col), _dptr(V), int(p), int(s),
                                                 int(length), int(bool(gram)), _dptr(out), _stream()))
        return out[:length]

    def close(self):
        if self._h:
            lib().bwr_matrix_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_allocations() -> int:
    """Device allocations the library has made in this process (bwr_device_allocations)."""
    return int(lib().bwr_device_allocations())


def sequence_workspace(m: int, n: int, nnz: int, s: int) -> int:
    """Device bytes bwr_sequence_dev_ws needs (0: invalid arguments)."""
    return int(lib().bwr_sequence_workspace(int(m), int(n), int(nnz), int(s)))


def rank_workspace(m: int, n: int, nnz: int, block: int) -> int:
    """Device bytes bwr_rank_modp_dev_ws needs (0: invalid arguments)."""
    return int(lib().bwr_rank_workspace(int(m), int(n), int(nnz), int(block)))


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def sequence_dev_ws(Ad, U, V, p: int, length: int, d_row=None, d_col=None, workspace=None, out=None):
    """bwr_sequence_dev_ws: the sequence with every device buffer carved from `workspace` (a torch uint8 device
    tensor; allocated here with bwr_sequence_workspace bytes when None)."""
    torch = _torch()
    st = _dev_csr(Ad)
    s = U.shape[1]
    if workspace is None:
        workspace = _workspace(sequence_workspace(Ad["m"], Ad["n"], Ad["nnz"], s), U.device)
    if out is None:
        out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=U.device)
    _check(lib().bwr_sequence_dev_ws(ctypes.byref(st), _dptr(d_row), _dptr(d_col), _dptr(U), _dptr(V), int(p),
                                     int(s), int(length), _dptr(out), _dptr(workspace), int(workspace.numel()),
                                     _stream()))
    return out[:length]


def rank_modp_dev_ws(Ad, p: int, block: int, seed: int, workspace=None):
    """bwr_rank_modp_dev_ws: (rank, info) with every device buffer carved from `workspace`."""
    st = _dev_csr(Ad)
    if workspace is None:
        workspace = _workspace(rank_workspace(Ad["m"], Ad["n"], Ad["nnz"], block), Ad["row_ptr"].device)
    r = ctypes.c_int64(0)
    info = RankInfo()
    _check(lib().bwr_rank_modp_dev_ws(ctypes.byref(st), int(p), int(block), int(seed), _dptr(workspace),
                                      int(workspace.numel()), _stream(), ctypes.byref(r), ctypes.byref(info)))
    return int(r.value), info.as_dict()


def sequence_sym_dev(Ad, V, p: int, length: int, d_row=None, d_col=None, gram: bool = False, out=None):
    """Symmetric sequence S_k = V^T B^k V (bwr_sequence_sym_dev); gram: two terms per application of B."""
    torch = _torch()
    st = _dev_csr(Ad)
    s = V.shape[1]
    if out is None:
        out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=V.device)
    _check(lib().bwr_sequence_sym_dev(ctypes.byref(st), _dptr(d_row), _dptr(d_col), _dptr(V), int(p), int(s),
                                      int(length), int(bool(gram)), _dptr(out), _stream()))
    return out[:length]


def rank_modp_sym(A, p: int, block: int, seed: int, gram: bool = False):
    """(rank, info) with the symmetric projection U = V (bwr_rank_modp_sym)."""
    st, keep = _host_csr(A)
    r = ctypes.c_int64(0)
    info = RankInfo()
    _check(lib().bwr_rank_modp_sym(ctypes.byref(st), int(p), int(block), int(seed), int(bool(gram)), ctypes.byref(r),
                                   ctypes.byref(info)))
    return int(r.value), info.as_dict()


def rank_modp_sym_dev(Ad, p: int, block: int, seed: int, gram: bool = False):
    st = _dev_csr(Ad)
    r = ctypes.c_int64(0)
    info = RankInfo()
    _check(lib().bwr_rank_modp_sym_dev(ctypes.byref(st), int(p), int(block), int(seed), int(bool(gram)), _stream(),
                                       ctypes.byref(r), ctypes.byref(info)))
    return int(r.value), info.as_dict()


def sequence_dev_noalloc(Ad, U, V, p: int, length: int, d_row=None, d_col=None, out=None):
    """bwr_sequence_dev_noalloc: the device sequence with no device allocation by the library (its buffers come
    from the library's static per-GPU scratch); `out` may be given to avoid torch's allocation too."""
    torch = _torch()
    st = _dev_csr(Ad)
    s = U.shape[1]
    if out is None:
        out = torch.empty((max(length, 1), s, s), dtype=torch.int32, device=U.device)
    _check(lib().bwr_sequence_dev_noalloc(ctypes.byref(st), _dptr(d_row), _dptr(d_col), _dptr(U), _dptr(V), int(p),
                                          int(s), int(length), _dptr(out), _stream()))
    return out[:length]


def apply_dev(Ad, X, p: int, d_row=None, d_col=None, out=None):
    torch = _torch()
    st = _dev_csr(Ad)
    s = X.shape[1]
    if out is None:
        out = torch.empty_like(X)
    _check(lib().bwr_apply_dev(ctypes.byref(st), _dptr(d_row), _dptr(d_col), _dptr(X), int(p), int(s), _dptr(out),
                               _stream()))
    return out


def rank_modp_dev(Ad, p: int, block: int, seed: int):
    st = _dev_csr(Ad)
    r = ctypes.c_int64(0)
    info = RankInfo()
    _check(lib().bwr_rank_modp_dev(ctypes.byref(st), int(p), int(block), int(seed), _stream(), ctypes.byref(r),
                                   ctypes.byref(info)))
    return int(r.value), info.as_dict()


def time_step_kernels_dev(Ad, p: int, s: int, transpose: bool = False, iters: int = 20, with_plan: bool = False):
    """Average microseconds of [first product, second product, projection] (HIP events on torch's stream);
    with_plan=True also returns the launch plan {W, G1, G2, fused, NB, esize, parts1, parts2, and the tiling of
    each product: T1R, T1cb, T1grid, T2R, T2cb, T2grid (rows per row block, 0 = not tiled; log2 slab rows;
    workgroups), T1un, T2un (entries in flight per lane)}."""
    st = _dev_csr(Ad)
    us = np.zeros(3, dtype=np.float64)
    plan = np.zeros(16, dtype=np.int32)
    _check(lib().bwr_time_step_kernels_dev(ctypes.byref(st), int(p), int(s), int(transpose), int(iters), _stream(),
                                           us.ctypes.data, plan.ctypes.data))
    if with_plan:
        keys = ("W", "G1", "G2", "fused", "NB", "esize", "parts1", "parts2", "T1R", "T1cb", "T1grid", "T2R",
                "T2cb", "T2grid", "T1un", "T2un")
        return us, {k: int(v) for k, v in zip(keys, plan)}
    return us


def min_generator_dev(S_dev, p: int):
    """Device sigma-basis of a device sequence tensor (len, s, s): (delta, P) on the host."""
    L, s, _ = S_dev.shape
    delta = np.zeros(s, dtype=np.int64)
    P = np.zeros((L + 2) * s * s, dtype=np.uint32)
    md = ctypes.c_int64(0)
    _check(lib().bwr_min_generator_dev(_dptr(S_dev), int(L), int(s), int(p), _stream(), delta.ctypes.data,
                                       P.ctypes.data, int(L + 2), ctypes.byref(md)))
    return delta, P[: (md.value + 1) * s * s].reshape(md.value + 1, s, s)


def min_generators_dev(S_devs, primes):
    """Batched device sigma-basis of device sequence tensors (len, s, s) of one shape, one prime each:
    a list of (delta, P) on the host."""
    n = len(S_devs)
    L, s, _ = S_devs[0].shape
    ptrs = (ctypes.c_void_p * n)(*[_dptr(S) for S in S_devs])
    pr = np.ascontiguousarray(primes, dtype=np.uint32)
    delta = np.zeros(n * s, dtype=np.int64)
    cap = L + 2
    P = np.zeros(n * cap * s * s, dtype=np.uint32)
    md = np.zeros(n, dtype=np.int64)
    _check(lib().bwr_min_generators_dev(ptrs, int(n), int(L), int(s), pr.ctypes.data, _stream(), delta.ctypes.data,
                                        P.ctypes.data, int(cap), md.ctypes.data))
    out = []
    for b in range(n):
        Pb = P[b * cap * s * s:(b + 1) * cap * s * s]
        out.append((delta[b * s:(b + 1) * s].copy(), Pb[: (md[b] + 1) * s * s].reshape(md[b] + 1, s, s).copy()))
    return out


def rank_integer(A, primes, block: int, seed: int):
    """(rank over the integers = the largest modular rank, ranks per prime) (Section 2.5)."""
    st, keep = _host_csr(A)
    pr = np.ascontiguousarray(primes, dtype=np.uint32)
    ranks = np.zeros(len(pr), dtype=np.int64)
    r = ctypes.c_int64(0)
    _check(lib().bwr_rank_integer(ctypes.byref(st), pr.ctypes.data, int(len(pr)), int(block), int(seed),
                                  ctypes.byref(r), ranks.ctypes.data))
    del keep
    return r.value, ranks


def _csr_array(mats):
    structs, keep = [], []
    for A in mats:
        st, k = _host_csr(A)
        structs.append(st)
        keep.append(k)
    arr = (CSRStruct * max(len(structs), 1))(*structs)
    ptrs = (ctypes.c_void_p * max(len(structs), 1))(*[ctypes.addressof(arr[i]) for i in range(len(structs))])
    return ptrs, (arr, keep)


def rank_modp_batch(mats, primes, block: int, seed: int):
    """(ranks (len(mats), len(primes)), info dict): all sequences advanced together."""
    ptrs, keep = _csr_array(mats)
    pr = np.ascontiguousarray(primes, dtype=np.uint32)
    out = np.zeros(max(len(mats) * len(pr), 1), dtype=np.int64)
    info = BatchInfo()
    _check(lib().bwr_rank_modp_batch(ptrs, len(mats), pr.ctypes.data, len(pr), int(block), int(seed),
                                     out.ctypes.data, ctypes.byref(info)))
    return out[: len(mats) * len(pr)].reshape(len(mats), len(pr)), info.as_dict()


def sequence_batch(mats, primes, s: int, seed: int, lengths):
    """Batched sequences: list over matrices of arrays (len(primes), length, s, s)."""
    ptrs, keep = _csr_array(mats)
    pr = np.ascontiguousarray(primes, dtype=np.uint32)
    ln = np.ascontiguousarray(lengths, dtype=np.int64)
    outs = [np.zeros(len(pr) * int(l) * s * s, dtype=np.uint32) for l in ln]
    optrs = (ctypes.c_void_p * max(len(outs), 1))(*[o.ctypes.data for o in outs])
    _check(lib().bwr_sequence_batch(ptrs, len(mats), pr.ctypes.data, len(pr), int(s), int(seed), ln.ctypes.data,
                                    optrs))
    return [o.reshape(len(pr), int(l), s, s) for o, l in zip(outs, ln)]


class ServerStats(ctypes.Structure):
    _fields_ = [("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("busy_s", ctypes.c_double), ("completed", ctypes.c_int64), ("max_queue", ctypes.c_int64),
                ("max_active", ctypes.c_int64), ("steps", ctypes.c_int64), ("peak_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """Continuous-batching rank server (bwr_server_*): submit host CSR requests, wait for ranks."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 64, block: int = 8):
        h = ctypes.c_void_p()
        _check(lib().bwr_server_create(int(hbm_budget_bytes), int(max_slots), int(block), ctypes.byref(h)))
        self._h = h

    def submit(self, A, p: int, seed: int) -> int:
        st, keep = _host_csr(A)
        t = ctypes.c_uint64(0)
        _check(lib().bwr_server_submit(self._h, ctypes.byref(st), int(p), int(seed), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        d = ctypes.c_int32(0)
        r = ctypes.c_int64(0)
        _check(lib().bwr_server_poll(self._h, int(ticket), ctypes.byref(d), ctypes.byref(r)))
        return (True, int(r.value)) if d.value else (False, None)

    def wait(self, ticket: int) -> int:
        r = ctypes.c_int64(0)
        _check(lib().bwr_server_wait(self._h, int(ticket), ctypes.byref(r)))
        return int(r.value)

    def stats(self):
        st = ServerStats()
        _check(lib().bwr_server_get_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._h:
            lib().bwr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
