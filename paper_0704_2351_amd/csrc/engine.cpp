// Device runtime: matrix store (validation + encoding, step 1 of the path) and
// the sequence driver (steps 2-3: the L-1 applications of B with the U^T
// projection after each, Section 2.2 and step 2 of the rank algorithm in
// Section 2.5).
#include "engine.h"

#include <algorithm>
#include <cstring>

#include "kernels.h"

namespace bwr {

Error Error::device(hipError_t e, const char* where) {
    return {EDEVICE_, std::string(where) + ": " + hipGetErrorString(e)};
}

#define BWR_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return Error::device(e_, #call);     \
    } while (0)

#define BWR_TRY(expr)                 \
    do {                              \
        Error er_ = (expr);           \
        if (!er_.ok()) return er_;    \
    } while (0)

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
    if (this != &o) {
        release();
        ptr_ = o.ptr_;
        bytes_ = o.bytes_;
        st_ = o.st_;
        o.ptr_ = nullptr;
        o.bytes_ = 0;
    }
    return *this;
}

Error DevBuf::alloc(size_t bytes, hipStream_t st) {
    release();
    st_ = st;
    bytes_ = bytes;
    if (bytes == 0) return {};
    hipError_t e = hipMallocAsync(&ptr_, bytes, st);
    if (e != hipSuccess) {
        ptr_ = nullptr;
        bytes_ = 0;
        (void)hipGetLastError();
        return {ENOMEM_, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    return {};
}

void DevBuf::release() {
    if (ptr_) (void)hipFreeAsync(ptr_, st_);
    ptr_ = nullptr;
    bytes_ = 0;
}

int padded_width(int32_t s) {
    if (s < 1) return 0;
    int w = 1;
    while (w < s) w <<= 1;
    return w <= 64 ? w : 0;
}

Error check_host_csr(const CsrView& A) {
    if (A.m < 0 || A.n < 0) return Error::inval("negative dimension");
    if (A.m > 0 && !A.row_ptr) return Error::inval("row_ptr is NULL");
    if (A.nnz > 0 && (!A.col_idx || !A.val)) return Error::inval("col_idx or val is NULL");
    if (A.m == 0) return A.nnz == 0 ? Error{} : Error::inval("nnz > 0 with no rows");
    if (A.row_ptr[0] != 0) return Error::inval("row_ptr[0] must be 0");
    if (A.row_ptr[A.m] != A.nnz) return Error::inval("row_ptr[m] must equal nnz");
    for (int64_t i = 0; i < A.m; ++i)
        if (A.row_ptr[i + 1] < A.row_ptr[i]) return Error::inval("row_ptr is not non-decreasing");
    for (int64_t t = 0; t < A.nnz; ++t)
        if (A.col_idx[t] < 0 || A.col_idx[t] >= A.n) return Error::inval("column index out of range");
    return {};
}

Error encode_matrix(const CsrView& A, uint32_t p, hipStream_t st, DeviceMatrix* M) {
    if (A.m < 0 || A.n < 0 || A.nnz < 0) return Error::inval("negative size");
    if (A.m >= (1LL << 31) - 1 || A.n >= (1LL << 31) - 1) return Error::inval("dimension must be below 2^31 - 1");
    if (A.nnz >= (1LL << 31)) return Error::inval("nnz must be below 2^31");
    if (A.m > 0 && !A.row_ptr) return Error::inval("row_ptr is NULL");
    if (A.nnz > 0 && (!A.col_idx || !A.val)) return Error::inval("col_idx or val is NULL");
    M->m = A.m;
    M->n = A.n;
    M->nnz = A.nnz;
    if (A.m == 0) {
        if (A.nnz) return Error::inval("nnz > 0 with no rows");
    }
    DevBuf small;
    BWR_TRY(small.alloc(sizeof(CsrStats) + 16, st));
    CsrStats* stats = small.as<CsrStats>();
    int32_t* flag = reinterpret_cast<int32_t*>(stats + 1);
    CsrStats h{};
    if (A.m > 0) {
        BWR_HIP(launch_rowptr_check(A.m, A.nnz, A.row_ptr, flag, st));
        int32_t bad = 0;
        BWR_HIP(hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st));
        BWR_HIP(hipStreamSynchronize(st));
        if (bad) return Error::inval("row_ptr must start at 0, be non-decreasing and end at nnz");
        BWR_HIP(launch_csr_stats(A.m, A.n, A.row_ptr, A.col_idx, A.val, stats, st));
        BWR_HIP(hipMemcpyAsync(&h, stats, sizeof(h), hipMemcpyDeviceToHost, st));
        BWR_HIP(hipStreamSynchronize(st));
        if (h.bad & BAD_COL) return Error::inval("column index out of range");
        if (h.bad) return Error::inval("malformed row_ptr");
    }
    M->max_len_a = h.max_len;
    M->max_abs = h.max_abs;
    M->packed = A.m <= (1LL << 24) && A.n <= (1LL << 24) && h.max_abs <= 127;
    ModP mp = ModP::make(p);
    M->wide_p = M->packed ? 0 : p;

    const size_t nnz = (size_t)A.nnz;
    BWR_TRY(M->rp_a.alloc(sizeof(int32_t) * (size_t)(A.m + 1), st));
    BWR_TRY(M->ent_a.alloc(sizeof(uint32_t) * nnz, st));
    BWR_TRY(M->rp_t.alloc(sizeof(int32_t) * (size_t)(A.n + 1), st));
    BWR_TRY(M->ent_t.alloc(sizeof(uint32_t) * nnz, st));
    if (!M->packed) {
        BWR_TRY(M->val_a.alloc(sizeof(uint32_t) * nnz, st));
        BWR_TRY(M->val_t.alloc(sizeof(uint32_t) * nnz, st));
    }
    if (A.m == 0) {
        BWR_HIP(hipMemsetAsync(M->rp_a.as<int32_t>(), 0, sizeof(int32_t), st));
    } else if (M->packed) {
        BWR_HIP(launch_pack_rows(A.m, A.row_ptr, A.col_idx, A.val, M->rp_a.as<int32_t>(), M->ent_a.as<uint32_t>(), st));
    } else {
        BWR_HIP(launch_wide_rows(A.m, A.row_ptr, A.col_idx, A.val, mp, M->rp_a.as<int32_t>(), M->ent_a.as<int32_t>(),
                                 M->val_a.as<uint32_t>(), st));
    }
    // CSR of A^T: column histogram, exclusive scan, scatter, per-row sort
    DevBuf cnt, cursor, tmp, mx;
    BWR_TRY(cnt.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_TRY(cursor.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_TRY(tmp.alloc(sizeof(int32_t) * (size_t)scan_tmp_words(A.n), st));
    BWR_TRY(mx.alloc(sizeof(int32_t), st));
    BWR_HIP(hipMemsetAsync(cnt.as<int32_t>(), 0, sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_HIP(hipMemsetAsync(cursor.as<int32_t>(), 0, sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_HIP(launch_col_count(A.m, A.row_ptr, A.col_idx, cnt.as<int32_t>(), st));
    BWR_HIP(launch_exclusive_scan(A.n, cnt.as<int32_t>(), M->rp_t.as<int32_t>(), tmp.as<int32_t>(), st));
    if (M->packed) {
        BWR_HIP(launch_scatter_packed_t(A.m, A.row_ptr, A.col_idx, A.val, M->rp_t.as<int32_t>(), cursor.as<int32_t>(),
                                        M->ent_t.as<uint32_t>(), st));
        BWR_HIP(launch_sort_rows_packed(A.n, M->rp_t.as<int32_t>(), M->ent_t.as<uint32_t>(), st));
    } else {
        BWR_HIP(launch_scatter_wide_t(A.m, A.row_ptr, A.col_idx, A.val, mp, M->rp_t.as<int32_t>(),
                                      cursor.as<int32_t>(), M->ent_t.as<int32_t>(), M->val_t.as<uint32_t>(), st));
        BWR_HIP(launch_sort_rows_wide(A.n, M->rp_t.as<int32_t>(), M->ent_t.as<int32_t>(), M->val_t.as<uint32_t>(),
                                      st));
    }
    BWR_HIP(launch_max_i32(A.n, cnt.as<int32_t>(), mx.as<int32_t>(), st));
    int32_t mlt = 0;
    BWR_HIP(hipMemcpyAsync(&mlt, mx.as<int32_t>(), sizeof(mlt), hipMemcpyDeviceToHost, st));
    BWR_HIP(hipStreamSynchronize(st));
    M->max_len_t = mlt;
    return {};
}

namespace {

bool use_acc32(const DeviceMatrix& M, int32_t max_len, uint32_t p) {
    if (!M.packed || p > 65536u) return false;
    return (int64_t)max_len * (int64_t)M.max_abs * (int64_t)(p - 1) < (1LL << 31);
}

Error spmm(const DeviceMatrix& M, const Operand& op, int W, ModP mp, const uint32_t* X, const uint32_t* scale,
           uint32_t* Y, hipStream_t st) {
    hipError_t e;
    if (M.packed)
        e = launch_spmm_packed(W, use_acc32(M, op.max_len, mp.p), mp.p <= 65536u, op.rows, op.rp, op.ent, X, scale, Y,
                               mp, st);
    else
        e = launch_spmm_wide(W, op.rows, op.rp, reinterpret_cast<const int32_t*>(op.ent), op.val, X, scale, Y, mp, st);
    if (e != hipSuccess) return Error::device(e, "spmm launch");
    return {};
}

void operands(const DeviceMatrix& M, bool transpose, Operand* first, Operand* second) {
    Operand a{M.m, M.max_len_a, M.rp_a.as<int32_t>(), M.ent_a.as<uint32_t>(), M.val_a.as<uint32_t>()};
    Operand t{M.n, M.max_len_t, M.rp_t.as<int32_t>(), M.ent_t.as<uint32_t>(), M.val_t.as<uint32_t>()};
    *first = transpose ? t : a;
    *second = transpose ? a : t;
}

}  // namespace

Error run_sequence(const SequenceArgs& a, hipStream_t st) {
    const DeviceMatrix& M = *a.M;
    if (a.M->packed == false && a.M->wide_p != a.mp.p) return Error::inval("matrix was encoded for another prime");
    const int W = padded_width(a.s);
    if (!W) return Error::inval("block size must be in 1..64");
    if (a.len <= 0) return {};
    Operand op1, op2;
    operands(M, a.transpose, &op1, &op2);
    const int64_t nb = op2.rows;     // iterated dimension
    const int64_t outer = op1.rows;  // intermediate dimension
    const ModP mp = a.mp;
    const bool smallp = mp.p <= 65536u;

    DevBuf Ut, X0, X1, Y, dr, dc2, part, flag;
    BWR_TRY(Ut.alloc(sizeof(uint32_t) * (size_t)(nb * W), st));
    BWR_TRY(X0.alloc(sizeof(uint32_t) * (size_t)(nb * W), st));
    BWR_TRY(X1.alloc(sizeof(uint32_t) * (size_t)(nb * W), st));
    BWR_TRY(Y.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer * W, 1), st));
    BWR_TRY(flag.alloc(sizeof(int32_t), st));
    BWR_HIP(hipMemsetAsync(flag.as<int32_t>(), 0, sizeof(int32_t), st));
    const uint32_t* drp = nullptr;
    const uint32_t* dc2p = nullptr;
    if (a.d_row && outer > 0) {
        BWR_TRY(dr.alloc(sizeof(uint32_t) * (size_t)outer, st));
        BWR_HIP(launch_reduce_vec(outer, a.d_row, mp, dr.as<uint32_t>(), st));
        drp = dr.as<uint32_t>();
    }
    if (a.d_col && nb > 0) {
        BWR_TRY(dc2.alloc(sizeof(uint32_t) * (size_t)nb, st));
        BWR_HIP(launch_square_diag(nb, a.d_col, mp, dc2.as<uint32_t>(), flag.as<int32_t>(), st));
        dc2p = dc2.as<uint32_t>();
    }
    // X_0 = D_c V and U~ = D_c^{-1} U, so that S_k = U~^T X_k with X_{k+1} = D_c^2 A^T D_r A X_k
    BWR_HIP(launch_pad_scale(nb, a.s, W, a.U, a.d_col, a.d_col ? 2 : 0, mp, Ut.as<uint32_t>(), st));
    BWR_HIP(launch_pad_scale(nb, a.s, W, a.V, a.d_col, a.d_col ? 1 : 0, mp, X0.as<uint32_t>(), st));

    const int NB = proj_blocks(nb, W);
    const size_t per_step = (size_t)NB * W * W;
    int64_t CH = std::min<int64_t>(a.len, 1024);
    CH = std::max<int64_t>(1, std::min<int64_t>(CH, (int64_t)((256u << 20) / (per_step * 4))));
    BWR_TRY(part.alloc(sizeof(uint32_t) * per_step * (size_t)CH, st));

    uint32_t* cur = X0.as<uint32_t>();
    uint32_t* nxt = X1.as<uint32_t>();
    int64_t k0 = 0;
    for (int64_t k = 0; k < a.len; ++k) {
        if (k > 0) {
            BWR_TRY(spmm(M, op1, W, mp, cur, drp, Y.as<uint32_t>(), st));
            BWR_TRY(spmm(M, op2, W, mp, Y.as<uint32_t>(), dc2p, nxt, st));
            std::swap(cur, nxt);
        }
        uint32_t* slot = part.as<uint32_t>() + per_step * (size_t)(k - k0);
        if (nb > 0) {
            hipError_t e = launch_project(W, smallp, nb, Ut.as<uint32_t>(), cur, slot, NB, mp, st);
            if (e != hipSuccess) return Error::device(e, "project launch");
        } else {
            BWR_HIP(hipMemsetAsync(slot, 0, sizeof(uint32_t) * per_step, st));
        }
        if (k - k0 + 1 == CH || k == a.len - 1) {
            BWR_HIP(launch_reduce_partials(W, a.s, NB, k - k0 + 1, part.as<uint32_t>(),
                                           a.S_out + (size_t)k0 * a.s * a.s, mp, st));
            k0 = k + 1;
        }
    }
    int32_t bad = 0;
    BWR_HIP(hipMemcpyAsync(&bad, flag.as<int32_t>(), sizeof(bad), hipMemcpyDeviceToHost, st));
    BWR_HIP(hipStreamSynchronize(st));
    if (bad) return Error::inval("d_col has an entry divisible by p");
    return {};
}

Error apply_once(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, const uint32_t* d_row,
                 const uint32_t* d_col, const uint32_t* X, uint32_t* Z, hipStream_t st) {
    if (!M.packed && M.wide_p != mp.p) return Error::inval("matrix was encoded for another prime");
    const int W = padded_width(s);
    if (!W) return Error::inval("block size must be in 1..64");
    Operand op1, op2;
    operands(M, transpose, &op1, &op2);
    const int64_t nb = op2.rows, outer = op1.rows;
    DevBuf Xp, Y, Zp, dr, dc;
    BWR_TRY(Xp.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Zp.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Y.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer * W, 1), st));
    const uint32_t* drp = nullptr;
    const uint32_t* dcp = nullptr;
    if (d_row && outer > 0) {
        BWR_TRY(dr.alloc(sizeof(uint32_t) * (size_t)outer, st));
        BWR_HIP(launch_reduce_vec(outer, d_row, mp, dr.as<uint32_t>(), st));
        drp = dr.as<uint32_t>();
    }
    if (d_col && nb > 0) {
        BWR_TRY(dc.alloc(sizeof(uint32_t) * (size_t)nb, st));
        BWR_HIP(launch_reduce_vec(nb, d_col, mp, dc.as<uint32_t>(), st));
        dcp = dc.as<uint32_t>();
    }
    // Z = D_c A^T D_r A D_c X
    BWR_HIP(launch_pad_scale(nb, s, W, X, dcp, dcp ? 1 : 0, mp, Xp.as<uint32_t>(), st));
    BWR_TRY(spmm(M, op1, W, mp, Xp.as<uint32_t>(), drp, Y.as<uint32_t>(), st));
    BWR_TRY(spmm(M, op2, W, mp, Y.as<uint32_t>(), dcp, Zp.as<uint32_t>(), st));
    BWR_HIP(launch_unpad(nb, s, W, Zp.as<uint32_t>(), Z, st));
    BWR_HIP(hipStreamSynchronize(st));
    return {};
}

Error time_step_kernels(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, int iters, hipStream_t st,
                        double us[3]) {
    const int W = padded_width(s);
    if (!W || iters < 1) return Error::inval("bad block size or iteration count");
    Operand op1, op2;
    operands(M, transpose, &op1, &op2);
    const int64_t nb = op2.rows, outer = op1.rows;
    DevBuf X, Y, Z, U, d1, d2, part;
    BWR_TRY(X.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Z.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(U.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Y.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer * W, 1), st));
    BWR_TRY(d1.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer, 1), st));
    BWR_TRY(d2.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb, 1), st));
    const int NB = proj_blocks(nb, W);
    BWR_TRY(part.alloc(sizeof(uint32_t) * (size_t)NB * W * W, st));
    BWR_HIP(launch_rng_block(12345, 0, nb, W, W, mp, 0, X.as<uint32_t>(), st));
    BWR_HIP(launch_rng_block(12345, 1, nb, W, W, mp, 0, U.as<uint32_t>(), st));
    BWR_HIP(launch_rng_block(12345, 2, outer, 1, 1, mp, 1, d1.as<uint32_t>(), st));
    BWR_HIP(launch_rng_block(12345, 3, nb, 1, 1, mp, 1, d2.as<uint32_t>(), st));
    hipEvent_t ev[2];
    BWR_HIP(hipEventCreate(&ev[0]));
    BWR_HIP(hipEventCreate(&ev[1]));
    Error err;
    for (int which = 0; which < 3 && err.ok(); ++which) {
        // one untimed launch, then `iters` timed ones
        for (int it = 0; it <= iters && err.ok(); ++it) {
            if (it == 1) (void)hipEventRecord(ev[0], st);
            if (which == 0) err = spmm(M, op1, W, mp, X.as<uint32_t>(), d1.as<uint32_t>(), Y.as<uint32_t>(), st);
            else if (which == 1) err = spmm(M, op2, W, mp, Y.as<uint32_t>(), d2.as<uint32_t>(), Z.as<uint32_t>(), st);
            else if (nb > 0) {
                hipError_t e = launch_project(W, mp.p <= 65536u, nb, U.as<uint32_t>(), Z.as<uint32_t>(),
                                              part.as<uint32_t>(), NB, mp, st);
                if (e != hipSuccess) err = Error::device(e, "project");
            }
        }
        (void)hipEventRecord(ev[1], st);
        hipError_t e = hipEventSynchronize(ev[1]);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess && err.ok()) err = Error::device(e, "event timing");
        us[which] = 1000.0 * ms / iters;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return err;
}

}  // namespace bwr
