// Device runtime: matrix store (validation + encoding, step 1 of the path) and
// the sequence driver (steps 2-3: the L-1 applications of B with the U^T
// projection after each, Section 2.2 and step 2 of the rank algorithm in
// Section 2.5).
#include "engine.h"

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <tuple>
#include <mutex>
#include <map>

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

namespace {
thread_local Arena* t_arena = nullptr;
std::atomic<int64_t> g_device_allocs{0};  // hipMallocAsync calls made by DevBuf
}  // namespace

int64_t device_allocations() { return g_device_allocs.load(); }

ArenaScope::ArenaScope(Arena* a) : prev_(t_arena) { t_arena = a; }
ArenaScope::~ArenaScope() { t_arena = prev_; }
Arena* current_arena() { return t_arena; }

DevBuf& DevBuf::operator=(DevBuf&& o) noexcept {
    if (this != &o) {
        release();
        ptr_ = o.ptr_;
        bytes_ = o.bytes_;
        st_ = o.st_;
        arena_ = o.arena_;
        o.ptr_ = nullptr;
        o.bytes_ = 0;
        o.arena_ = nullptr;
    }
    return *this;
}

Error DevBuf::alloc(size_t bytes, hipStream_t st) {
    release();
    st_ = st;
    bytes_ = bytes;
    if (bytes == 0) return {};
    if (Arena* a = t_arena) {
        const size_t off = (a->used + 255) & ~(size_t)255;
        const size_t want = (bytes + 255) & ~(size_t)255;
        if (off + want > a->size) {
            bytes_ = 0;
            return {ENOMEM_, "workspace too small: " + std::to_string(off + want) + " bytes needed so far, " +
                                 std::to_string(a->size) + " given"};
        }
        ptr_ = a->base + off;
        a->used = off + want;
        a->peak = std::max(a->peak, a->used);
        arena_ = a;
        return {};
    }
    g_device_allocs.fetch_add(1);
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
    if (ptr_ && arena_) {
        // the topmost carving returns its bytes (stream order keeps earlier readers ahead of later writers)
        const size_t want = (bytes_ + 255) & ~(size_t)255;
        if ((char*)ptr_ + want == arena_->base + arena_->used) arena_->used = (size_t)((char*)ptr_ - arena_->base);
    } else if (ptr_) {
        (void)hipFreeAsync(ptr_, st_);
    }
    ptr_ = nullptr;
    bytes_ = 0;
    arena_ = nullptr;
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

namespace {

Error encode_plain(const CsrView& A, uint32_t p, hipStream_t st, DeviceMatrix* M) {
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
        BWR_HIP(launch_fill_zero(M->rp_a.as<int32_t>(), sizeof(int32_t), st));
    } else if (M->packed) {
        BWR_HIP(launch_pack_rows(A.m, A.row_ptr, A.col_idx, A.val, M->rp_a.as<int32_t>(), M->ent_a.as<uint32_t>(), st));
    } else {
        BWR_HIP(launch_wide_rows(A.m, A.row_ptr, A.col_idx, A.val, mp, M->rp_a.as<int32_t>(), M->ent_a.as<int32_t>(),
                                 M->val_a.as<uint32_t>(), st));
    }
    // CSR of A^T: column histogram, exclusive scan, scatter (the order inside a
    // row of A^T is that of the atomics; sums do not depend on it)
    DevBuf cnt, cursor, tmp, mx;
    BWR_TRY(cnt.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_TRY(cursor.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_TRY(tmp.alloc(sizeof(int32_t) * (size_t)scan_tmp_words(A.n), st));
    BWR_TRY(mx.alloc(sizeof(int32_t), st));
    BWR_HIP(launch_fill_zero(cnt.as<int32_t>(), sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_HIP(launch_fill_zero(cursor.as<int32_t>(), sizeof(int32_t) * (size_t)std::max<int64_t>(A.n, 1), st));
    BWR_HIP(launch_col_count(A.m, A.row_ptr, A.col_idx, cnt.as<int32_t>(), st));
    BWR_HIP(launch_exclusive_scan(A.n, cnt.as<int32_t>(), M->rp_t.as<int32_t>(), tmp.as<int32_t>(), st));
    if (M->packed) {
        BWR_HIP(launch_scatter_packed_t(A.m, A.row_ptr, A.col_idx, A.val, M->rp_t.as<int32_t>(), cursor.as<int32_t>(),
                                        M->ent_t.as<uint32_t>(), st));
    } else {
        BWR_HIP(launch_scatter_wide_t(A.m, A.row_ptr, A.col_idx, A.val, mp, M->rp_t.as<int32_t>(),
                                      cursor.as<int32_t>(), M->ent_t.as<int32_t>(), M->val_t.as<uint32_t>(), st));
    }
    BWR_HIP(launch_max_i32(A.n, cnt.as<int32_t>(), mx.as<int32_t>(), st));
    int32_t mlt = 0;
    BWR_HIP(hipMemcpyAsync(&mlt, mx.as<int32_t>(), sizeof(mlt), hipMemcpyDeviceToHost, st));
    BWR_HIP(hipStreamSynchronize(st));
    M->max_len_t = mlt;
    return {};
}

// Indices 0 .. count-1 in order of decreasing length (stable; lengths above 4095 count as 4095).
std::vector<int32_t> by_decreasing_length(const std::vector<int32_t>& len) {
    constexpr int KMAX = 4095;
    std::vector<int64_t> start(KMAX + 2, 0);
    for (int32_t l : len) ++start[KMAX - std::min(std::max(l, 0), KMAX) + 1];
    for (int k = 0; k <= KMAX; ++k) start[k + 1] += start[k];
    std::vector<int32_t> order(len.size());
    for (size_t i = 0; i < len.size(); ++i) order[start[KMAX - std::min(std::max(len[i], 0), KMAX)]++] = (int32_t)i;
    return order;
}

}  // namespace

Error encode_matrix(const CsrView& A, uint32_t p, hipStream_t st, DeviceMatrix* M, bool sort) {
    BWR_TRY(encode_plain(A, p, st, M));
    const char* ns = getenv("BWR_NO_SORT");
    if (!sort || (ns && atoi(ns) != 0) || A.m < 2 || A.n < 1 || A.nnz == 0) return {};
    // row lengths of A and of A^T from the encoding just built
    std::vector<int32_t> rpa((size_t)A.m + 1), rpt((size_t)A.n + 1);
    BWR_HIP(hipMemcpyAsync(rpa.data(), M->rp_a.as<void>(), sizeof(int32_t) * rpa.size(), hipMemcpyDeviceToHost, st));
    BWR_HIP(hipMemcpyAsync(rpt.data(), M->rp_t.as<void>(), sizeof(int32_t) * rpt.size(), hipMemcpyDeviceToHost, st));
    BWR_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> lr((size_t)A.m), lc((size_t)A.n);
    for (int64_t i = 0; i < A.m; ++i) lr[i] = rpa[i + 1] - rpa[i];
    for (int64_t j = 0; j < A.n; ++j) lc[j] = rpt[j + 1] - rpt[j];
    const std::vector<int32_t> perm_r = by_decreasing_length(lr), perm_c = by_decreasing_length(lc);
    std::vector<int32_t> inv_c((size_t)A.n);
    for (int64_t j = 0; j < A.n; ++j) inv_c[perm_c[j]] = (int32_t)j;
    std::vector<int64_t> rp_new((size_t)A.m + 1, 0);
    for (int64_t i = 0; i < A.m; ++i) rp_new[i + 1] = rp_new[i] + lr[perm_r[i]];
    // declared after the host vectors, so destroyed before them: an error return below must not free them
    // while their asynchronous (possibly staged) copies are still pending
    struct DrainOnExit {
        hipStream_t st;
        ~DrainOnExit() { (void)hipStreamSynchronize(st); }
    } drain_before_free{st};
    DevBuf d_pr, d_pc, d_ic, d_rp, d_col, d_val;
    BWR_TRY(d_pr.alloc(sizeof(int32_t) * perm_r.size(), st));
    BWR_TRY(d_pc.alloc(sizeof(int32_t) * perm_c.size(), st));
    BWR_TRY(d_ic.alloc(sizeof(int32_t) * inv_c.size(), st));
    BWR_TRY(d_rp.alloc(sizeof(int64_t) * rp_new.size(), st));
    BWR_TRY(d_col.alloc(sizeof(int32_t) * (size_t)A.nnz, st));
    BWR_TRY(d_val.alloc(sizeof(int32_t) * (size_t)A.nnz, st));
    BWR_HIP(hipMemcpyAsync(d_pr.as<void>(), perm_r.data(), sizeof(int32_t) * perm_r.size(), hipMemcpyHostToDevice, st));
    BWR_HIP(hipMemcpyAsync(d_pc.as<void>(), perm_c.data(), sizeof(int32_t) * perm_c.size(), hipMemcpyHostToDevice, st));
    BWR_HIP(hipMemcpyAsync(d_ic.as<void>(), inv_c.data(), sizeof(int32_t) * inv_c.size(), hipMemcpyHostToDevice, st));
    BWR_HIP(hipMemcpyAsync(d_rp.as<void>(), rp_new.data(), sizeof(int64_t) * rp_new.size(), hipMemcpyHostToDevice, st));
    BWR_HIP(launch_permute_csr(A.m, d_rp.as<int64_t>(), d_pr.as<int32_t>(), A.row_ptr, A.col_idx, A.val,
                               d_ic.as<int32_t>(), d_col.as<int32_t>(), d_val.as<int32_t>(), st));
    const CsrView B{A.m, A.n, A.nnz, d_rp.as<int64_t>(), d_col.as<int32_t>(), d_val.as<int32_t>()};
    DeviceMatrix S;
    BWR_TRY(encode_plain(B, p, st, &S));  // synchronizes st, so the host vectors above have been read
    S.sorted = true;
    S.perm_r = std::move(d_pr);
    S.perm_c = std::move(d_pc);
    *M = std::move(S);
    return {};
}

namespace {

bool use_acc32(const DeviceMatrix& M, int32_t max_len, uint32_t p) {
    if (!M.packed || p > 65536u) return false;
    return (int64_t)max_len * (int64_t)M.max_abs * (int64_t)(p - 1) < (1LL << 31);
}

// accumulator mode of the row-split kernel for G lanes per row slice (see launch_spmm_split)
int acc_mode(const DeviceMatrix& M, int32_t max_len, uint32_t p, int G) {
    if (use_acc32(M, max_len, p)) return 1;
    if (M.packed && p > 65536u && G >= 1) {
        const int64_t per_lane = ((int64_t)max_len + G - 1) / G;
        if (per_lane * (int64_t)M.max_abs * 65535 < (1LL << 31)) return 2;
    }
    return 0;
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

// The two column parts of a packed operand (entries gathering from the first and the second half of
// the block) and the carry buffer between their passes.
struct SplitOp {
    DevBuf rp0, rp1, ent0, ent1, carry;
    Operand p0{}, p1{};
    bool on = false;
};

Error build_split(const Operand& op, int64_t cols, int64_t nnz, int W, hipStream_t st, SplitOp* so) {
    const int64_t rows = op.rows;
    DevBuf cnt0, cnt1, tmp;
    BWR_TRY(so->rp0.alloc(sizeof(int32_t) * (size_t)(rows + 1), st));
    BWR_TRY(so->rp1.alloc(sizeof(int32_t) * (size_t)(rows + 1), st));
    BWR_TRY(so->ent0.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nnz, 1), st));
    BWR_TRY(so->ent1.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nnz, 1), st));
    BWR_TRY(so->carry.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(rows * W, 1), st));
    BWR_TRY(cnt0.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(rows, 1), st));
    BWR_TRY(cnt1.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(rows, 1), st));
    BWR_TRY(tmp.alloc(sizeof(int32_t) * (size_t)scan_tmp_words(rows), st));
    BWR_HIP(launch_split_operand(rows, op.rp, op.ent, (uint32_t)(cols / 2), cnt0.as<int32_t>(), cnt1.as<int32_t>(),
                                 tmp.as<int32_t>(), so->rp0.as<int32_t>(), so->rp1.as<int32_t>(),
                                 so->ent0.as<uint32_t>(), so->ent1.as<uint32_t>(), st));
    so->p0 = Operand{rows, op.max_len, so->rp0.as<int32_t>(), so->ent0.as<uint32_t>(), nullptr};
    so->p1 = Operand{rows, op.max_len, so->rp1.as<int32_t>(), so->ent1.as<uint32_t>(), nullptr};
    so->on = true;
    return {};
}

// ---- two-dimensional tiled products ----

int device_attr(hipDeviceAttribute_t a, int dflt) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, a, dev) != hipSuccess || v <= 0) return dflt;
    return v;
}

// bits of the two's-complement value field holding -max_abs .. max_abs
int value_bits(int32_t max_abs) {
    int b = 1;
    while (b < 31 && (1LL << (b - 1)) <= (int64_t)max_abs) ++b;
    return std::max(b, 2);
}

int bit_length(int64_t x) {
    int b = 0;
    while (x > 0) {
        ++b;
        x >>= 1;
    }
    return b;
}

// int32 accumulation over a whole row (all its slabs): see launch_spmm_tiled
bool tiled_acc_ok(const DeviceMatrix& M, int32_t max_len, uint32_t p) {
    if (!M.packed) return false;
    const int64_t f = p <= 65536u ? (int64_t)(p - 1) : 65535;
    return (int64_t)max_len * (int64_t)std::max(M.max_abs, 1) * f < (1LL << 31);
}

TiledOperand tiled_view(int64_t rows, int64_t cols, const StepPlan::Tile& t, int32_t max_abs) {
    TiledOperand v;
    v.rows = rows;
    v.R = t.R;
    v.cb = t.cb;
    v.vb = value_bits(max_abs);
    v.rb = bit_length(t.R - 1);
    v.nrb = t.nrb;
    v.K = (int)std::max<int64_t>(1, (cols + (1LL << t.cb) - 1) >> t.cb);
    return v;
}

// Row blocks for at most Rmax rows each and `slots` resident workgroups: whole rounds of grid blocks, each
// block as small as that count allows; with fill, at least one block per slot while there are rows for them,
// so that a single round still occupies every CU.
void finish_tile(int64_t rows, int64_t Rmax, int64_t slots, StepPlan::Tile* t, bool fill = true) {
    int64_t nrb0 = (rows + Rmax - 1) / Rmax;
    if (fill) nrb0 = std::max(nrb0, std::min(slots, rows));
    const int64_t grid = std::max<int64_t>(1, std::min(nrb0, slots));
    t->nrb = grid * ((nrb0 + grid - 1) / grid);
    t->R = (int)((rows + t->nrb - 1) / t->nrb);
    t->grid = (int)grid;
}

// Geometry of a tiled product with `rows` outputs gathering from `cols` block rows: slabs of about
// slab_bytes of the block (fewer when the 32-bit entry needs the bits), row blocks as large as wgs
// workgroups per CU leave LDS for, one persistent workgroup per (CU, wgs) slot.
bool tile_geometry(int64_t rows, int64_t cols, int W, int esize, bool split, bool proj, int32_t max_abs,
                   size_t slab_bytes, int wgs, StepPlan::Tile* t) {
    if (rows < 1 || cols < 1 || W < 4) return false;
    wgs = std::min(std::max(wgs, 1), 2);
    const int lds = device_attr(hipDeviceAttributeMaxSharedMemoryPerBlock, 65536) / wgs;
    const int nacc = split ? 2 * W : W;
    const int vb = value_bits(max_abs);
    int cb = std::min(24, bit_length((int64_t)(slab_bytes / ((size_t)W * esize))) - 1);
    cb = std::max(4, std::min<int>(cb, std::max(4, bit_length(cols - 1))));
    for (; cb >= 4; --cb) {
        const int64_t K = (cols + (1LL << cb) - 1) >> cb;
        if (K > 8192) return false;
        int64_t R = ((int64_t)lds / 4 - K - 2) / nacc - 1;
        R = std::min<int64_t>(R, rows);
        if (R < 1) return false;
        if (bit_length(R - 1) + cb + vb > 32) continue;
        if (tiled_lds_bytes(W, split, proj, (int)R, (int)K) > (size_t)lds) continue;
        const int cus = device_attr(hipDeviceAttributeMultiprocessorCount, 256);
        t->cb = cb;
        finish_tile(rows, R, (int64_t)cus * wgs, t);
        return true;
    }
    return false;
}

// Tiled geometries the autotuner tries: row blocks for one or two workgroups per CU, slabs of 128 to 512 KB of
// the block (measured at the 2M x 1M size: larger slabs lose, 256 and 128 KB are within a few per cent), one, two
// or four entries per lane per pass (a pass of fewer entries spans fewer slabs; more entries load more entry
// words ahead).  BWR_TILED_WGS, BWR_TILED_SLAB (bytes), BWR_TILED_R (cap on the row block), BWR_TILED_GRID (cap
// on the workgroups) and BWR_TILED_UN (entries per lane per pass) pin one geometry.
std::vector<StepPlan::Tile> tile_candidates(int64_t rows, int64_t cols, int W, int esize, bool split, bool proj,
                                            int32_t max_abs) {
    std::vector<StepPlan::Tile> out;
    const char* ew = getenv("BWR_TILED_WGS");
    const char* es = getenv("BWR_TILED_SLAB");
    const char* er = getenv("BWR_TILED_R");
    std::vector<int> wgs = ew ? std::vector<int>{atoi(ew)} : std::vector<int>{1, 2};
    std::vector<size_t> slabs = es ? std::vector<size_t>{(size_t)atoll(es)}
                                   : std::vector<size_t>{(size_t)128 << 10, (size_t)256 << 10, (size_t)512 << 10};
    for (int w : wgs)
        for (size_t sl : slabs) {
            StepPlan::Tile t;
            if (!tile_geometry(rows, cols, W, esize, split, proj, max_abs, sl, w, &t)) continue;
            const int64_t slots = (int64_t)device_attr(hipDeviceAttributeMultiprocessorCount, 256) * std::min(2, std::max(1, w));
            if (er && atoi(er) >= 1 && t.R > atoi(er)) finish_tile(rows, atoi(er), slots, &t, false);
            if (const char* eg = getenv("BWR_TILED_GRID")) {
                if (atoi(eg) >= 1) t.grid = (int)std::min<int64_t>(t.grid, atoi(eg));
                if (atoi(eg) == -1) t.grid = (int)t.nrb;  // one workgroup per row block
            }
            const char* eu = getenv("BWR_TILED_UN");
            for (int un : eu ? std::vector<int>{std::min(4, std::max(1, atoi(eu)))} : std::vector<int>{1, 2, 4}) {
                t.un = un;
                bool dup = false;
                for (const auto& o : out)
                    dup |= (o.R == t.R && o.cb == t.cb && o.grid == t.grid && o.nrb == t.nrb && o.un == t.un);
                if (!dup) out.push_back(t);
            }
        }
    return out;
}

struct TiledOp {
    DevBuf tp, ent;
    TiledOperand v;
    bool on = false;
};

// launch shape of geometry t over the tiled encoding o
TiledLaunch tiled_launch(const TiledOp&, const StepPlan::Tile& t) {
    TiledLaunch L;
    L.grid = t.grid;
    L.un = t.un;
    return L;
}

// Tiled encoding of a packed operand for the geometry cfg (see launch_tiled_build).
Error build_tiled(const Operand& op, int64_t cols, int64_t nnz, int32_t max_abs, const StepPlan::Tile& cfg,
                  hipStream_t st, TiledOp* to) {
    to->v = tiled_view(op.rows, cols, cfg, max_abs);
    const int64_t ntiles = to->v.nrb * to->v.K;
    const int64_t count = ntiles * cfg.R;
    if (count >= (1LL << 31)) return Error::inval("tiled encoding too large");
    DevBuf cnt, pos, tmp;
    BWR_TRY(cnt.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(count, 1), st));
    BWR_TRY(pos.alloc(sizeof(int32_t) * (size_t)(count + 1), st));
    BWR_TRY(tmp.alloc(sizeof(int32_t) * (size_t)scan_tmp_words(count), st));
    BWR_TRY(to->tp.alloc(sizeof(uint32_t) * (size_t)(ntiles + 1), st));
    BWR_TRY(to->ent.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nnz, 1), st));
    BWR_HIP(launch_tiled_build(op.rows, to->v.nrb, op.rp, op.ent, to->v.K, cfg.R, cfg.cb, to->v.vb, cnt.as<int32_t>(),
                               pos.as<int32_t>(), tmp.as<int32_t>(), to->tp.as<uint32_t>(), to->ent.as<uint32_t>(),
                               st));
    to->v.tile_ptr = to->tp.as<uint32_t>();
    to->v.ent = to->ent.as<uint32_t>();
    to->on = true;
    return {};
}

}  // namespace

struct TiledStore {
    hipStream_t home = nullptr;
    std::mutex mu;
    struct Ent {
        int which;  // 0: rows of A, 1: rows of A^T
        StepPlan::Tile cfg;
        TiledOp op;
    };
    std::vector<std::unique_ptr<Ent>> v;
};

std::shared_ptr<TiledStore> make_tiled_store(hipStream_t home) {
    auto s = std::make_shared<TiledStore>();
    s->home = home;
    return s;
}

void rehome(DeviceMatrix& M, hipStream_t home) {
    for (DevBuf* b : {&M.rp_a, &M.ent_a, &M.rp_t, &M.ent_t, &M.val_a, &M.val_t, &M.perm_r, &M.perm_c})
        b->set_stream(home);
}

namespace {

// The tiled encoding of operand op (rows of A or of A^T) for geometry cfg: from the matrix's store when it
// has one (built there on first use), else built into *scratch.
Error get_tiled(const DeviceMatrix& M, const Operand& op, int64_t cols, const StepPlan::Tile& cfg, hipStream_t st,
                TiledOp* scratch, const TiledOp** out) {
    if (!M.tiled) {
        BWR_TRY(build_tiled(op, cols, M.nnz, M.max_abs, cfg, st, scratch));
        *out = scratch;
        return {};
    }
    const int which = op.rp == M.rp_a.as<int32_t>() ? 0 : 1;
    TiledStore& S = *M.tiled;
    std::lock_guard<std::mutex> lk(S.mu);
    for (auto& e : S.v)
        if (e->which == which && e->cfg.R == cfg.R && e->cfg.cb == cfg.cb && e->cfg.nrb == cfg.nrb) {
            e->op.v.rows = op.rows;
            *out = &e->op;
            return {};
        }
    auto e = std::make_unique<TiledStore::Ent>();
    e->which = which;
    e->cfg = cfg;
    BWR_TRY(build_tiled(op, cols, M.nnz, M.max_abs, cfg, st, &e->op));
    BWR_HIP(hipStreamSynchronize(st));  // built before its buffers change owner stream
    e->op.tp.set_stream(S.home);
    e->op.ent.set_stream(S.home);
    *out = &e->op;
    S.v.push_back(std::move(e));
    return {};
}

}  // namespace

namespace {

int env_int(const char* name, int dflt) {
    const char* v = getenv(name);
    return (v && *v) ? atoi(v) : dflt;
}

int pow2_ceil(double x) {
    int g = 1;
    while (g < x && g < 16) g <<= 1;
    return g;
}

// Lanes per row slice: about a quarter of the average row length, so that one
// unrolled pass (4 non-zeros per lane) covers a typical row.
int heuristic_g(const Operand& op, int64_t nnz, int W, bool proj) {
    double avg = op.rows > 0 ? (double)nnz / (double)op.rows : 1.0;
    int g = pow2_ceil(avg / 4.0);
    if (proj && g < W / 4) g = W / 4;
    while (g > 1 && !split_supported(W, g, proj)) g >>= 1;
    if (!split_supported(W, g, proj)) {
        for (g = 1; g <= 16 && !split_supported(W, g, proj); g <<= 1) {
        }
    }
    return split_supported(W, g, proj) ? g : 0;
}

// First product of a step: Y = D_r (A X) (row-split kernel, in two column passes when so is set).
hipError_t first_product(const DeviceMatrix& M, const Operand& op1, const SplitOp* so, int G, const StepPlan& pl,
                         ModP mp, const void* X, const uint32_t* dr, void* Y, hipStream_t st,
                         const TiledOp* to = nullptr) {
    const bool smallp = mp.p <= 65536u;
    if (to && to->on)
        return launch_spmm_tiled(to->v, pl.W, 0, !smallp, pl.esize, X, dr, Y, nullptr, nullptr, nullptr,
                                 tiled_launch(*to, pl.t1), mp, st);
    if (so && so->on) {
        hipError_t e = launch_spmm_split(pl.W, G, false, acc_mode(M, op1.max_len, mp.p, G), smallp, pl.esize,
                                         op1.rows, so->p0.rp, so->p0.ent, X, nullptr, nullptr, nullptr, nullptr, 0, mp,
                                         st, 1, so->carry.as<uint32_t>());
        if (e != hipSuccess) return e;
        return launch_spmm_split(pl.W, G, false, acc_mode(M, op1.max_len, mp.p, G), smallp, pl.esize, op1.rows,
                                 so->p1.rp, so->p1.ent, X, dr, Y, nullptr, nullptr, 0, mp, st, 2,
                                 so->carry.as<uint32_t>());
    }
    return launch_spmm_split(pl.W, G, false, acc_mode(M, op1.max_len, mp.p, G), smallp, pl.esize, op1.rows, op1.rp,
                             op1.ent, X, dr, Y, nullptr, nullptr, 0, mp, st);
}

// Second product: Z = D_c^2 (A^T Y), with the projection partials when fused (nblocks persistent blocks).
hipError_t second_product(const DeviceMatrix& M, const Operand& op2, const SplitOp* so, int G, bool fused,
                          int nblocks, const StepPlan& pl, ModP mp, const void* Yin, const uint32_t* dc2, void* Z,
                          const void* Ut, uint32_t* partial, hipStream_t st, const TiledOp* to = nullptr) {
    const bool smallp = mp.p <= 65536u;
    if (to && to->on)
        return launch_spmm_tiled(to->v, pl.W, 1, !smallp, pl.esize, Yin, dc2, Z, Ut, nullptr, partial,
                                 tiled_launch(*to, pl.t2), mp, st);
    if (so && so->on) {
        hipError_t e = launch_spmm_split(pl.W, G, false, acc_mode(M, op2.max_len, mp.p, G), smallp, pl.esize,
                                         op2.rows, so->p0.rp, so->p0.ent, Yin, nullptr, nullptr, nullptr, nullptr, 0,
                                         mp, st, 1, so->carry.as<uint32_t>());
        if (e != hipSuccess) return e;
        return launch_spmm_split(pl.W, G, fused, acc_mode(M, op2.max_len, mp.p, G), smallp, pl.esize, op2.rows,
                                 so->p1.rp, so->p1.ent, Yin, dc2, Z, fused ? Ut : nullptr, fused ? partial : nullptr,
                                 fused ? nblocks : 0, mp, st, 2, so->carry.as<uint32_t>());
    }
    return launch_spmm_split(pl.W, G, fused, acc_mode(M, op2.max_len, mp.p, G), smallp, pl.esize, op2.rows, op2.rp,
                             op2.ent, Yin, dc2, Z, fused ? Ut : nullptr, fused ? partial : nullptr, fused ? nblocks : 0,
                             mp, st);
}

struct Bufs {
    const uint32_t* dr;
    const uint32_t* dc2;
    const void* Ut;  // pl.esize-byte residues
    void* Y;
};

Error launch_step(const DeviceMatrix& M, const Operand& op1, const Operand& op2, const SplitOp* so1,
                  const SplitOp* so2, const StepPlan& pl, ModP mp, const Bufs& b, const void* cur, void* nxt,
                  uint32_t* slot, hipStream_t st, const TiledOp* to1 = nullptr, const TiledOp* to2 = nullptr) {
    const bool smallp = mp.p <= 65536u;
    const int64_t nb = op2.rows;
    hipError_t e;
    if (pl.G1 > 0 || (to1 && to1->on)) {
        e = first_product(M, op1, so1, pl.G1, pl, mp, cur, b.dr, b.Y, st, to1);
        if (e != hipSuccess) return Error::device(e, "sparse product (first)");
    } else {
        BWR_TRY(spmm(M, op1, pl.W, mp, (const uint32_t*)cur, b.dr, (uint32_t*)b.Y, st));
    }
    if (pl.G2 > 0 || (to2 && to2->on)) {
        e = second_product(M, op2, so2, pl.G2, pl.fused, pl.NB, pl, mp, b.Y, b.dc2, nxt, b.Ut, slot, st, to2);
        if (e != hipSuccess) return Error::device(e, "sparse product (second)");
        if (pl.fused) return {};
    } else {
        BWR_TRY(spmm(M, op2, pl.W, mp, (const uint32_t*)b.Y, b.dc2, (uint32_t*)nxt, st));
    }
    if (nb > 0) {
        e = launch_project(pl.W, smallp, nb, b.Ut, nxt, pl.esize, slot, pl.NB, mp, st);
        if (e != hipSuccess) return Error::device(e, "project launch");
    }
    return {};
}

// Times `iters` launches of fn with HIP events (after one untimed launch).
// back-to-back launches per autotuner timing (one untimed launch first)
constexpr int TUNE_ITERS = 4;

template <class Fn>
Error time_launches(int iters, hipStream_t st, Fn fn, double* us) {
    hipEvent_t ev[2];
    BWR_HIP(hipEventCreate(&ev[0]));
    BWR_HIP(hipEventCreate(&ev[1]));
    Error err = fn();
    if (err.ok()) (void)hipEventRecord(ev[0], st);
    for (int it = 0; it < iters && err.ok(); ++it) err = fn();
    if (err.ok()) {
        (void)hipEventRecord(ev[1], st);
        hipError_t e = hipEventSynchronize(ev[1]);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e != hipSuccess) err = Error::device(e, "event timing");
        *us = 1000.0 * ms / iters;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return err;
}

// Index of the fastest candidate: TUNE_ROUNDS rounds, each timing every candidate in turn; a candidate's
// time is its best round, so work that another stream runs meanwhile inflates the candidates alike
// instead of deciding the choice.
constexpr int TUNE_ROUNDS = 3;

Error pick_fastest(const std::vector<std::function<Error()>>& cands, hipStream_t st, int* best,
                   std::vector<double>* times = nullptr) {
    std::vector<double> t(cands.size(), 1e30);
    for (int r = 0; r < TUNE_ROUNDS; ++r)
        for (size_t i = 0; i < cands.size(); ++i) {
            double us = 0;
            BWR_TRY(time_launches(TUNE_ITERS, st, cands[i], &us));
            t[i] = std::min(t[i], us);
        }
    *best = (int)(std::min_element(t.begin(), t.end()) - t.begin());
    if (times) *times = t;
    return {};
}

// BWR_TUNE_LOG=1: the autotuner prints every candidate's time to stderr
bool tune_log() { return getenv("BWR_TUNE_LOG") != nullptr; }

}  // namespace

// Persistent blocks of the fused second product: at most `want`, and at most 2^19 partial words per step.
constexpr int64_t FUSED_PARTIAL_WORDS = 524288;
int64_t fused_nb_cap(int W, int64_t want) {
    return std::max<int64_t>(1, std::min<int64_t>(want, FUSED_PARTIAL_WORDS / ((int64_t)W * W)));
}

size_t sequence_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int32_t s, bool transpose) {
    const int W = padded_width(s);
    if (!W || m < 0 || n < 0 || nnz < 0) return 0;
    const int64_t nb = transpose ? m : n, outer = transpose ? n : m;
    // encode_matrix with the length-sorted relabelling: the first encoding, the relabelled CSR copy, the second
    // encoding and its counters (wide residues included): at most 40 nnz + 20 m + 24 n bytes and a few KB
    const int64_t enc = 40 * nnz + 24 * (m + n) + (64 << 10);
    // run_sequence: gathered U, V, D_c, D_r; U~, X_0, X_1 (nb x W) and Y (outer x W) of at most 4-byte residues;
    // the reduced diagonals; ARENA_CHUNK steps of projection partials (at most max(2^19, 512 W^2) words a step)
    const int64_t blocks = 8 * nb * s + 8 * nb + 8 * outer + 4 * (int64_t)W * (3 * nb + outer);
    const int64_t part = 4 * std::max<int64_t>(524288, 512LL * W * W) * ARENA_CHUNK;
    return (size_t)(enc + blocks + part + 64 * 256);
}

StepPlan plan_step(const DeviceMatrix& M, bool transpose, int32_t s, uint32_t p, bool allow_tiled) {
    StepPlan pl;
    pl.W = padded_width(s);
    Operand op1, op2;
    operands(M, transpose, &op1, &op2);
    const int64_t nb = op2.rows;
    if (M.packed && pl.W >= 4) {
        pl.G1 = env_int("BWR_G1", heuristic_g(op1, M.nnz, pl.W, false));
        int g2 = env_int("BWR_G2", heuristic_g(op2, M.nnz, pl.W, true));
        if (!split_supported(pl.W, pl.G1, false)) pl.G1 = heuristic_g(op1, M.nnz, pl.W, false);
        pl.fused = split_supported(pl.W, g2, true);
        pl.G2 = pl.fused ? g2 : (split_supported(pl.W, g2, false) ? g2 : heuristic_g(op2, M.nnz, pl.W, false));
    }
    // 16-bit storage of the iterated blocks when every kernel of the step can read it
    pl.esize = (p <= 65536u && pl.G1 > 0 && pl.G2 > 0 && env_int("BWR_E32", 0) == 0) ? 2 : 4;
    // column passes (32-bit residues): BWR_PARTS=2 forces two passes for both products
    if (pl.esize == 4 && M.packed && env_int("BWR_PARTS", 1) == 2) {
        pl.parts1 = pl.G1 > 0 && nb >= 2 ? 2 : 1;
        pl.parts2 = pl.G2 > 0 && op1.rows >= 2 ? 2 : 1;
    }
    if (pl.fused) {
        const int rpb = split_rows_per_block(pl.W, pl.G2);
        int64_t tiles = (nb + rpb - 1) / rpb;
        pl.NB = (int)std::max<int64_t>(1, std::min<int64_t>(tiles, fused_nb_cap(pl.W, 1024)));
    } else {
        pl.NB = proj_blocks(nb, pl.W);
    }
    // BWR_TILED=1: both products tiled (first geometry of tile_candidates) wherever the encoding allows it
    if (allow_tiled && env_int("BWR_TILED", -1) == 1 && pl.G1 > 0 && pl.G2 > 0) {
        const bool split = p > 65536u;
        if (tiled_acc_ok(M, op1.max_len, p)) {
            auto c = tile_candidates(op1.rows, nb, pl.W, pl.esize, split, false, M.max_abs);
            if (!c.empty()) pl.t1 = c[0];
        }
        if (tiled_acc_ok(M, op2.max_len, p)) {
            auto c = tile_candidates(op2.rows, op1.rows, pl.W, pl.esize, split, true, M.max_abs);
            if (!c.empty()) {
                pl.t2 = c[0];
                pl.fused = true;
                pl.NB = pl.t2.grid;
            }
        }
        pl.parts1 = pl.parts2 = 1;
    }
    return pl;
}

Error autotune_step(const DeviceMatrix& M, bool transpose, ModP mp, StepPlan* pl, hipStream_t st) {
    if (pl->G1 <= 0 && pl->G2 <= 0) return {};
    Operand op1, op2;
    operands(M, transpose, &op1, &op2);
    const int W = pl->W;
    const int64_t nb = op2.rows, outer = op1.rows;
    const bool smallp = mp.p <= 65536u;
    const size_t es = (size_t)pl->esize;
    DevBuf X, Y, Z, U, part;
    BWR_TRY(X.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Z.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(U.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Y.alloc(es * (size_t)std::max<int64_t>(outer * W, 1), st));
    const int cus = device_attr(hipDeviceAttributeMultiprocessorCount, 256);
    const int64_t part_words = std::max<int64_t>(std::max<int64_t>(FUSED_PARTIAL_WORDS, 2LL * cus * W * W),
                                                 (int64_t)proj_blocks(nb, W) * W * W);
    BWR_TRY(part.alloc(sizeof(uint32_t) * (size_t)part_words, st));
    // timing inputs: contents do not change the memory traffic
    BWR_HIP(launch_fill_zero(X.as<void>(), X.bytes(), st));
    BWR_HIP(launch_fill_zero(U.as<void>(), U.bytes(), st));
    BWR_HIP(launch_fill_zero(Y.as<void>(), Y.bytes(), st));
    // two-dimensional tiled candidates for matrices of at least 2^20 non-zeros (BWR_TILED=0: none)
    const bool split = !smallp;
    const bool tiles_on = M.packed && M.nnz >= (1 << 20) && env_int("BWR_TILED", -1) != 0;
    std::vector<StepPlan::Tile> tc1, tc2;
    std::vector<TiledOp> to1, to2;  // one encoding per distinct geometry; b1[i], b2[i]: candidate i's
    if (tiles_on && pl->G1 > 0 && tiled_acc_ok(M, op1.max_len, mp.p))
        tc1 = tile_candidates(op1.rows, nb, W, pl->esize, split, false, M.max_abs);
    if (tiles_on && pl->G2 > 0 && tiled_acc_ok(M, op2.max_len, mp.p))
        tc2 = tile_candidates(op2.rows, outer, W, pl->esize, split, true, M.max_abs);
    // candidates that differ only in their launch (entries per pass) share one encoding
    auto encodings = [&](const Operand& op, int64_t cols, const std::vector<StepPlan::Tile>& tc,
                         std::vector<TiledOp>* to, std::vector<size_t>* b) -> Error {
        std::vector<const StepPlan::Tile*> geo;
        for (const StepPlan::Tile& t : tc) {
            size_t j = 0;
            while (j < geo.size() && !(geo[j]->R == t.R && geo[j]->cb == t.cb && geo[j]->nrb == t.nrb)) ++j;
            if (j == geo.size()) geo.push_back(&t);
            b->push_back(j);
        }
        to->resize(geo.size());
        for (size_t j = 0; j < geo.size(); ++j) BWR_TRY(build_tiled(op, cols, M.nnz, M.max_abs, *geo[j], st, &(*to)[j]));
        return {};
    };
    std::vector<size_t> b1, b2;
    BWR_TRY(encodings(op1, nb, tc1, &to1, &b1));
    BWR_TRY(encodings(op2, outer, tc2, &to2, &b2));
    pl->t1 = StepPlan::Tile{};
    pl->t2 = StepPlan::Tile{};
    if (pl->G1 > 0) {
        std::vector<int> gs;  // row split G, or -(1 + index) of a tiled candidate
        std::vector<std::function<Error()>> runs;
        for (int g = 1; g <= 16; g <<= 1) {
            if (!split_supported(W, g, false)) continue;
            gs.push_back(g);
            runs.push_back([&, g]() -> Error {
                hipError_t e = launch_spmm_split(W, g, false, acc_mode(M, op1.max_len, mp.p, g), smallp, pl->esize,
                                                 op1.rows, op1.rp, op1.ent, X.as<void>(), nullptr, Y.as<void>(),
                                                 nullptr, nullptr, 0, mp, st);
                return e == hipSuccess ? Error{} : Error::device(e, "autotune");
            });
        }
        for (size_t i = 0; i < tc1.size(); ++i) {
            gs.push_back(-1 - (int)i);
            runs.push_back([&, i]() -> Error {
                hipError_t e = launch_spmm_tiled(to1[b1[i]].v, W, 0, split, pl->esize, X.as<void>(), nullptr,
                                                 Y.as<void>(), nullptr, nullptr, nullptr,
                                                 tiled_launch(to1[b1[i]], tc1[i]), mp, st);
                return e == hipSuccess ? Error{} : Error::device(e, "autotune (tiled)");
            });
        }
        int bi = 0;
        std::vector<double> tt;
        BWR_TRY(pick_fastest(runs, st, &bi, &tt));
        if (tune_log())
            for (size_t i = 0; i < gs.size(); ++i) {
                if (gs[i] > 0)
                    fprintf(stderr, "[bwr tune] first product  row split G=%d: %.2f us\n", gs[i], tt[i]);
                else {
                    const auto& c = tc1[-1 - gs[i]];
                    fprintf(stderr, "[bwr tune] first product  tiled R=%d cb=%d grid=%d un=%d: %.2f us\n", c.R,
                            c.cb, c.grid, c.un, tt[i]);
                }
            }
        if (gs[bi] > 0)
            pl->G1 = gs[bi];
        else
            pl->t1 = tc1[-1 - gs[bi]];
    }
    if (pl->G2 > 0) {
        // second product and projection: fused, with 1024 or 2048 persistent blocks or with the row tiles
        // split evenly over ceil(tiles / k) blocks (k = 1 .. 4, so no block runs one tile more than the
        // others), or the plain product followed by the projection kernel; the fastest pair wins
        struct Cand {
            int g, nbk;
            bool fused;
        };
        std::vector<Cand> cs;
        std::vector<std::function<Error()>> runs;
        const int pnb = proj_blocks(nb, W);
        for (int g = 1; g <= 16; g <<= 1) {
            const int rpb = split_rows_per_block(W, g);
            const int64_t tiles = (nb + rpb - 1) / rpb;
            std::vector<int> nbs;  // fused block counts; 0 = plain product + projection kernel
            if (split_supported(W, g, true)) {
                for (int64_t want : {(int64_t)1024, (int64_t)2048, tiles, (tiles + 1) / 2, (tiles + 2) / 3,
                                     (tiles + 3) / 4}) {
                    const int c = (int)std::min<int64_t>(std::max<int64_t>(1, tiles), fused_nb_cap(W, want));
                    if (std::find(nbs.begin(), nbs.end(), c) == nbs.end()) nbs.push_back(c);
                }
            }
            if (split_supported(W, g, false)) nbs.push_back(0);
            for (int c : nbs) {
                const bool fused = c > 0;
                const int nbk = fused ? c : pnb;
                cs.push_back({g, nbk, fused});
                runs.push_back([&, g, nbk, fused]() -> Error {
                    hipError_t e = launch_spmm_split(W, g, fused, acc_mode(M, op2.max_len, mp.p, g), smallp, pl->esize,
                                                     op2.rows, op2.rp, op2.ent, Y.as<void>(), nullptr, Z.as<void>(),
                                                     U.as<void>(), part.as<uint32_t>(), fused ? nbk : 0, mp, st);
                    if (e == hipSuccess && !fused && nb > 0)
                        e = launch_project(W, smallp, nb, U.as<void>(), Z.as<void>(), pl->esize, part.as<uint32_t>(),
                                           nbk, mp, st);
                    return e == hipSuccess ? Error{} : Error::device(e, "autotune");
                });
            }
        }
        for (size_t i = 0; i < tc2.size(); ++i) {
            cs.push_back({-1 - (int)i, tc2[i].grid, true});
            runs.push_back([&, i]() -> Error {
                hipError_t e = launch_spmm_tiled(to2[b2[i]].v, W, 1, split, pl->esize, Y.as<void>(), nullptr,
                                                 Z.as<void>(), U.as<void>(), nullptr, part.as<uint32_t>(),
                                                 tiled_launch(to2[b2[i]], tc2[i]), mp, st);
                return e == hipSuccess ? Error{} : Error::device(e, "autotune (tiled)");
            });
        }
        int bi = 0;
        std::vector<double> tt;
        BWR_TRY(pick_fastest(runs, st, &bi, &tt));
        if (tune_log())
            for (size_t i = 0; i < cs.size(); ++i) {
                if (cs[i].g > 0)
                    fprintf(stderr, "[bwr tune] second product row split G=%d fused=%d blocks=%d: %.2f us\n", cs[i].g,
                            (int)cs[i].fused, cs[i].nbk, tt[i]);
                else {
                    const auto& c = tc2[-1 - cs[i].g];
                    fprintf(stderr, "[bwr tune] second product tiled R=%d cb=%d grid=%d un=%d: %.2f us\n", c.R,
                            c.cb, c.grid, c.un, tt[i]);
                }
            }
        if (cs[bi].g > 0) {
            pl->G2 = cs[bi].g;
        } else {
            pl->t2 = tc2[-1 - cs[bi].g];
        }
        pl->NB = cs[bi].nbk;
        pl->fused = cs[bi].fused;
    }
    to1.clear();
    to2.clear();
    // 32-bit residues: does running each product in two column passes (each gathering from half of the
    // block, which then fits an XCD's L2) beat one pass?  (Not for a tiled product: its slabs already fit.)
    if (pl->esize == 4 && M.packed && env_int("BWR_NO_PARTS", 0) == 0 && getenv("BWR_PARTS") == nullptr) {
        SplitOp so1, so2;
        if (pl->G1 > 0 && nb >= 2 && pl->t1.R == 0) {
            BWR_TRY(build_split(op1, nb, M.nnz, W, st, &so1));
            auto run = [&](const SplitOp* so) -> Error {
                hipError_t e = first_product(M, op1, so, pl->G1, *pl, mp, X.as<void>(), nullptr, Y.as<void>(), st);
                return e == hipSuccess ? Error{} : Error::device(e, "autotune");
            };
            int bi = 0;
            BWR_TRY(pick_fastest({[&]() { return run(nullptr); }, [&]() { return run(&so1); }}, st, &bi));
            pl->parts1 = bi == 1 ? 2 : 1;
        }
        if (pl->G2 > 0 && outer >= 2 && pl->t2.R == 0) {
            BWR_TRY(build_split(op2, outer, M.nnz, W, st, &so2));
            auto run = [&](const SplitOp* so) -> Error {
                hipError_t e = second_product(M, op2, so, pl->G2, pl->fused, pl->NB, *pl, mp, Y.as<void>(), nullptr,
                                              Z.as<void>(), U.as<void>(), part.as<uint32_t>(), st);
                if (e == hipSuccess && !pl->fused && nb > 0)
                    e = launch_project(W, smallp, nb, U.as<void>(), Z.as<void>(), pl->esize, part.as<uint32_t>(),
                                       pl->NB, mp, st);
                return e == hipSuccess ? Error{} : Error::device(e, "autotune");
            };
            int bi = 0;
            BWR_TRY(pick_fastest({[&]() { return run(nullptr); }, [&]() { return run(&so2); }}, st, &bi));
            pl->parts2 = bi == 1 ? 2 : 1;
        }
    }
    return {};
}

namespace {

// Launch plans tuned in this process, by matrix shape, orientation, block width and prime: a plan only
// changes speed, so a matrix of the same shape reuses it (the second and later solves do not retune,
// and every solve of a shape runs the same kernels).  BWR_NO_PLAN_CACHE=1 retunes every call.
struct PlanKey {
    int dev;
    int64_t m, n, nnz;
    int32_t la, lt;
    bool transpose, sorted;
    int W, esize;
    uint32_t p;
    bool operator<(const PlanKey& o) const {
        return std::tie(dev, m, n, nnz, la, lt, transpose, sorted, W, esize, p) <
               std::tie(o.dev, o.m, o.n, o.nnz, o.la, o.lt, o.transpose, o.sorted, o.W, o.esize, o.p);
    }
};
std::mutex g_plan_mu;
std::map<PlanKey, StepPlan> g_plans;

Error tuned_plan(const DeviceMatrix& M, bool transpose, ModP mp, StepPlan* pl, hipStream_t st) {
    int dev = 0;
    BWR_HIP(hipGetDevice(&dev));
    const PlanKey key{dev, M.m, M.n, M.nnz, M.max_len_a, M.max_len_t, transpose, M.sorted, pl->W, pl->esize, mp.p};
    const bool cache = env_int("BWR_NO_PLAN_CACHE", 0) == 0 && getenv("BWR_PARTS") == nullptr;
    if (cache) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) {
            *pl = it->second;
            return {};
        }
    }
    BWR_TRY(autotune_step(M, transpose, mp, pl, st));
    if (cache) {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        g_plans[key] = *pl;
    }
    return {};
}

}  // namespace

namespace {

// Keeps the enqueueing thread at most two chunks ahead of the device (SequenceArgs::stop): before chunk n
// waits for the event recorded after chunk n - 2.  Recorded outside graph capture only.
struct Pacer {
    bool on = false;
    int64_t n = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    ~Pacer() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    Error before_chunk() {
        if (!on || n < 2) return {};
        const hipError_t e = hipEventSynchronize(ev[n & 1]);
        return e == hipSuccess ? Error{} : Error::device(e, "hipEventSynchronize");
    }
    Error after_chunk(hipStream_t st) {
        if (!on) return {};
        hipEvent_t& e = ev[n & 1];
        hipError_t r = e ? hipSuccess : hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r == hipSuccess) r = hipEventRecord(e, st);
        if (r != hipSuccess) return Error::device(r, "hipEventRecord");
        ++n;
        return {};
    }
};

// The symmetric sequence in Gram form (symmetric.hip): S_0 = X_0^T D_c^-2 X_0, then per application of B the
// terms S_2k+1 = Y_k^T D_r^-1 Y_k (from the first product's output) and S_2k+2 = X_k+1^T D_c^-2 X_k+1 (from the
// second's); the products run without a fused projection.  Chunks of CH applications are captured as one HIP
// graph and replayed, like the plain sequence.
Error gram_sequence(const SequenceArgs& a, const DeviceMatrix& M, const Operand& op1, const Operand& op2,
                    const StepPlan& pl, const SplitOp* so1, const SplitOp* so2, const TiledOp* to1, const TiledOp* to2,
                    void* X0, void* X1, void* Y, const uint32_t* drp, const uint32_t* dc2p, const uint32_t* aDr,
                    const uint32_t* aDc, int32_t* flag, hipStream_t st) {
    const int W = pl.W;
    const int64_t nb = op2.rows, outer = op1.rows;
    const ModP mp = a.mp;
    const bool smallp = mp.p <= 65536u;
    const int64_t E = (int64_t)W * W;
    DevBuf w1, w2, part, part0;
    BWR_TRY(w1.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer, 1), st));
    BWR_TRY(w2.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb, 1), st));
    BWR_HIP(launch_inv_diag(outer, aDr, mp, 1, w1.as<uint32_t>(), st));
    BWR_HIP(launch_inv_diag(nb, aDc, mp, 2, w2.as<uint32_t>(), st));
    // partial blocks of each product's Gram term: the tiled kernels form it in their epilogue (one partial per
    // workgroup), the others through k_gram
    const bool t1 = to1 && to1->on, t2 = to2 && to2->on;
    const int NBg = std::max(proj_blocks(std::max<int64_t>(nb, 1), W), proj_blocks(std::max<int64_t>(outer, 1), W));
    const int nb1 = t1 ? pl.t1.grid : NBg, nb2 = t2 ? pl.t2.grid : NBg;
    const int64_t P = (int64_t)(nb1 + nb2) * E;  // partial words per application
    int64_t CH = current_arena() ? ARENA_CHUNK : 128;  // applications per chunk (2 CH terms)
    CH = std::max<int64_t>(2, std::min<int64_t>(CH, (int64_t)((256u << 20) / (P * 4))) & ~(int64_t)1);
    BWR_TRY(part.alloc(sizeof(uint32_t) * (size_t)(P * CH), st));
    BWR_TRY(part0.alloc(sizeof(uint32_t) * (size_t)(NBg * E), st));
    uint32_t* slots = part.as<uint32_t>();
    // S_0 = X_0^T D_c^-2 X_0
    if (nb > 0) {
        BWR_HIP(launch_gram(W, smallp, nb, X0, pl.esize, w2.as<uint32_t>(), part0.as<uint32_t>(), NBg, mp, st));
    } else {
        BWR_HIP(launch_fill_zero(part0.as<void>(), sizeof(uint32_t) * (size_t)(NBg * E), st));
    }
    BWR_HIP(launch_reduce_partials(W, a.s, NBg, 1, part0.as<uint32_t>(), a.S_out, mp, st));
    BWR_HIP(launch_mirror(1, a.s, a.S_out, st));
    if (a.progress) BWR_TRY(a.progress(1));
    // one application: S_2k+1 from the first product's output, S_2k+2 from the second's
    auto app = [&](const void* cur, void* nxt, uint32_t* slot) -> Error {
        hipError_t e;
        if (t1) {
            e = launch_spmm_tiled(to1->v, W, 2, !smallp, pl.esize, cur, drp, Y, nullptr, w1.as<uint32_t>(), slot,
                                  tiled_launch(*to1, pl.t1), mp, st);
        } else {
            if (pl.G1 > 0)
                e = first_product(M, op1, so1, pl.G1, pl, mp, cur, drp, Y, st, nullptr);
            else
                e = spmm(M, op1, W, mp, (const uint32_t*)cur, drp, (uint32_t*)Y, st).ok() ? hipSuccess
                                                                                          : hipErrorUnknown;
            if (e == hipSuccess) e = launch_gram(W, smallp, outer, Y, pl.esize, w1.as<uint32_t>(), slot, NBg, mp, st);
        }
        if (e != hipSuccess) return Error::device(e, "gram step (first product)");
        uint32_t* slot2 = slot + (size_t)nb1 * E;
        if (t2) {
            e = launch_spmm_tiled(to2->v, W, 2, !smallp, pl.esize, Y, dc2p, nxt, nullptr, w2.as<uint32_t>(), slot2,
                                  tiled_launch(*to2, pl.t2), mp, st);
        } else {
            if (pl.G2 > 0)
                e = second_product(M, op2, so2, pl.G2, false, 0, pl, mp, Y, dc2p, nxt, nullptr, nullptr, st);
            else
                e = spmm(M, op2, W, mp, (const uint32_t*)Y, dc2p, (uint32_t*)nxt, st).ok() ? hipSuccess
                                                                                           : hipErrorUnknown;
            if (e == hipSuccess) e = launch_gram(W, smallp, nb, nxt, pl.esize, w2.as<uint32_t>(), slot2, NBg, mp, st);
        }
        if (e != hipSuccess) return Error::device(e, "gram step (second product)");
        return {};
    };
    void* cur = X0;
    void* nxt = X1;
    const bool use_graph = !current_arena() && env_int("BWR_NO_GRAPH", 0) == 0 && nb > 0 && (a.len - 1) >= 4 * CH;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Error err;
    Pacer pace;
    pace.on = (bool)a.stop;
    int64_t t = 1;
    while (t < a.len && err.ok()) {
        if (!(err = pace.before_chunk()).ok()) break;
        const int64_t apps = std::min<int64_t>(CH, (a.len - t + 1) / 2);
        if (use_graph && apps == CH) {
            if (!exec) {
                hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) {
                    err = Error::device(e, "hipStreamBeginCapture");
                    break;
                }
                for (int64_t i = 0; i < CH && err.ok(); ++i) {
                    err = app(cur, nxt, slots + P * i);
                    std::swap(cur, nxt);
                }
                e = hipStreamEndCapture(st, &graph);
                if (err.ok() && e != hipSuccess) err = Error::device(e, "hipStreamEndCapture");
                if (err.ok()) {
                    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                    if (e != hipSuccess) err = Error::device(e, "hipGraphInstantiate");
                }
                if (!err.ok()) break;
            }
            const hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) {
                err = Error::device(e, "hipGraphLaunch");
                break;
            }
        } else {
            for (int64_t i = 0; i < apps && err.ok(); ++i) {
                err = app(cur, nxt, slots + P * i);
                std::swap(cur, nxt);
            }
            if (!err.ok()) break;
        }
        // terms t, t + 2, ... from the first products; t + 1, t + 3, ... from the second
        const int64_t nterms = std::min<int64_t>(2 * apps, a.len - t);
        uint32_t* out = a.S_out + (size_t)t * a.s * a.s;
        hipError_t e = launch_reduce_partials(W, a.s, nb1, (nterms + 1) / 2, slots, out, mp, st, P, 2);
        if (e == hipSuccess)
            e = launch_reduce_partials(W, a.s, nb2, nterms / 2, slots + (size_t)nb1 * E, out + (size_t)a.s * a.s, mp,
                                       st, P, 2);
        if (e == hipSuccess) e = launch_mirror(nterms, a.s, out, st);
        if (e != hipSuccess) err = Error::device(e, "gram reduce");
        t += nterms;
        if (err.ok() && a.progress) err = a.progress(t);
        if (err.ok()) err = pace.after_chunk(st);
        if (err.ok() && a.stop && t < a.len && a.stop(t)) break;
    }
    if (a.len_out) *a.len_out = std::min(t, a.len);
    int32_t bad = 0;
    hipError_t he = hipSuccess;
    if (err.ok()) he = hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, st);
    const hipError_t hs = hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (!err.ok()) return err;
    if (he != hipSuccess) return Error::device(he, "hipMemcpyAsync");
    if (hs != hipSuccess) return Error::device(hs, "hipStreamSynchronize");
    if (bad) return Error::inval("d_col has an entry divisible by p");
    return {};
}

}  // namespace

Error run_sequence(const SequenceArgs& a, hipStream_t st) {
    const DeviceMatrix& M = *a.M;
    if (!M.packed && M.wide_p != a.mp.p) return Error::inval("matrix was encoded for another prime");
    const int W = padded_width(a.s);
    if (!W) return Error::inval("block size must be in 1..64");
    if (a.len <= 0) return {};
    Operand op1, op2;
    operands(M, a.transpose, &op1, &op2);
    const int64_t nb = op2.rows;     // iterated dimension
    const int64_t outer = op1.rows;  // intermediate dimension
    const ModP mp = a.mp;
    const bool smallp = mp.p <= 65536u;

    // inside an arena (caller workspace, or the entry point that allocates nothing): the heuristic row-split
    // plan, no tuning trials and no tiled encodings, whose buffers sequence_workspace_bytes bounds
    const bool in_arena = current_arena() != nullptr;
    StepPlan pl = plan_step(M, a.transpose, a.s, mp.p, !in_arena);
    if (!in_arena && a.len >= 64 && M.nnz >= 100000 && env_int("BWR_NO_TUNE", 0) == 0 && getenv("BWR_G1") == nullptr &&
        getenv("BWR_G2") == nullptr && env_int("BWR_TILED", -1) != 1)
        BWR_TRY(tuned_plan(M, a.transpose, mp, &pl, st));
    if (in_arena) pl.parts1 = pl.parts2 = 1;
    if (a.plan_out) *a.plan_out = pl;

    const size_t es = (size_t)pl.esize;
    SplitOp so1, so2;
    if (pl.parts1 == 2) BWR_TRY(build_split(op1, nb, M.nnz, W, st, &so1));
    if (pl.parts2 == 2) BWR_TRY(build_split(op2, outer, M.nnz, W, st, &so2));
    TiledOp own1, own2;
    const TiledOp* to1 = nullptr;
    const TiledOp* to2 = nullptr;
    if (pl.t1.R > 0) {
        BWR_TRY(get_tiled(M, op1, nb, pl.t1, st, &own1, &to1));
        BWR_HIP(prepare_spmm_tiled(to1->v, W, 0, !smallp, pl.esize));
        BWR_HIP(prepare_spmm_tiled(to1->v, W, 2, !smallp, pl.esize));
    }
    if (pl.t2.R > 0) {
        BWR_TRY(get_tiled(M, op2, outer, pl.t2, st, &own2, &to2));
        BWR_HIP(prepare_spmm_tiled(to2->v, W, 1, !smallp, pl.esize));
        BWR_HIP(prepare_spmm_tiled(to2->v, W, 2, !smallp, pl.esize));
    }
    // a length-sorted encoding works in relabelled coordinates: U, V, D_c (iterated side) and D_r (other
    // side) are gathered into that order, which leaves every S_k unchanged
    const uint32_t* aU = a.symmetric ? a.V : a.U;
    const uint32_t* aV = a.V;
    const uint32_t* aDr = a.d_row;
    const uint32_t* aDc = a.d_col;
    DevBuf gU, gV, gDr, gDc;
    if (M.sorted) {
        const int32_t* pn = (a.transpose ? M.perm_r : M.perm_c).as<int32_t>();  // iterated side
        const int32_t* po = (a.transpose ? M.perm_c : M.perm_r).as<int32_t>();  // other side
        if (nb > 0) {
            BWR_TRY(gU.alloc(sizeof(uint32_t) * (size_t)(nb * a.s), st));
            BWR_TRY(gV.alloc(sizeof(uint32_t) * (size_t)(nb * a.s), st));
            BWR_HIP(launch_gather_rows(nb, a.s, pn, aU, gU.as<uint32_t>(), st));
            BWR_HIP(launch_gather_rows(nb, a.s, pn, a.V, gV.as<uint32_t>(), st));
            aU = gU.as<uint32_t>();
            aV = gV.as<uint32_t>();
            if (a.d_col) {
                BWR_TRY(gDc.alloc(sizeof(uint32_t) * (size_t)nb, st));
                BWR_HIP(launch_gather_rows(nb, 1, pn, a.d_col, gDc.as<uint32_t>(), st));
                aDc = gDc.as<uint32_t>();
            }
        }
        if (a.d_row && outer > 0) {
            BWR_TRY(gDr.alloc(sizeof(uint32_t) * (size_t)outer, st));
            BWR_HIP(launch_gather_rows(outer, 1, po, a.d_row, gDr.as<uint32_t>(), st));
            aDr = gDr.as<uint32_t>();
        }
    }
    DevBuf Ut, X0, X1, Y, dr, dc2, part, flag;
    BWR_TRY(Ut.alloc(es * (size_t)(nb * W), st));
    BWR_TRY(X0.alloc(es * (size_t)(nb * W), st));
    BWR_TRY(X1.alloc(es * (size_t)(nb * W), st));
    BWR_TRY(Y.alloc(es * (size_t)std::max<int64_t>(outer * W, 1), st));
    BWR_TRY(flag.alloc(sizeof(int32_t), st));
    BWR_HIP(launch_fill_zero(flag.as<int32_t>(), sizeof(int32_t), st));
    const uint32_t* drp = nullptr;
    const uint32_t* dc2p = nullptr;
    if (aDr && outer > 0) {
        BWR_TRY(dr.alloc(sizeof(uint32_t) * (size_t)outer, st));
        BWR_HIP(launch_reduce_vec(outer, aDr, mp, dr.as<uint32_t>(), st));
        drp = dr.as<uint32_t>();
    }
    if (aDc && nb > 0) {
        BWR_TRY(dc2.alloc(sizeof(uint32_t) * (size_t)nb, st));
        BWR_HIP(launch_square_diag(nb, aDc, mp, dc2.as<uint32_t>(), flag.as<int32_t>(), st));
        dc2p = dc2.as<uint32_t>();
    }
    // X_0 = D_c V and U~ = D_c^{-1} U, so that S_k = U~^T X_k with X_{k+1} = D_c^2 A^T D_r A X_k
    BWR_HIP(launch_pad_scale(nb, a.s, W, aU, aDc, aDc ? 2 : 0, mp, Ut.as<void>(), pl.esize, st));
    BWR_HIP(launch_pad_scale(nb, a.s, W, aV, aDc, aDc ? 1 : 0, mp, X0.as<void>(), pl.esize, st));

    const size_t per_step = (size_t)pl.NB * W * W;
    int64_t CH = in_arena ? ARENA_CHUNK : 256;
    CH = std::max<int64_t>(2, std::min<int64_t>(CH, (int64_t)((256u << 20) / (per_step * 4))) & ~(int64_t)1);
    BWR_TRY(part.alloc(sizeof(uint32_t) * per_step * (size_t)CH, st));
    uint32_t* slots = part.as<uint32_t>();
    Bufs bufs{drp, dc2p, Ut.as<void>(), Y.as<void>()};

    if (a.symmetric && a.gram) return gram_sequence(a, M, op1, op2, pl, &so1, &so2, to1, to2, X0.as<void>(),
                                                    X1.as<void>(), Y.as<void>(), drp, dc2p, aDr, aDc, flag.as<int32_t>(),
                                                    st);
    // S_0
    if (nb > 0) {
        hipError_t e = launch_project(W, smallp, nb, Ut.as<void>(), X0.as<void>(), pl.esize, slots, pl.NB, mp, st);
        if (e != hipSuccess) return Error::device(e, "project launch");
    } else {
        BWR_HIP(launch_fill_zero(slots, sizeof(uint32_t) * per_step, st));
    }
    BWR_HIP(launch_reduce_partials(W, a.s, pl.NB, 1, slots, a.S_out, mp, st));
    if (a.progress) BWR_TRY(a.progress(1));

    void* cur = X0.as<void>();
    void* nxt = X1.as<void>();
    // no graphs inside an arena: instantiating one is work (and memory) of the runtime's own
    const bool use_graph = !in_arena && env_int("BWR_NO_GRAPH", 0) == 0 && a.len - 1 >= 2 * CH && nb > 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Error err;
    Pacer pace;
    pace.on = (bool)a.stop;
    int64_t k = 1;
    while (k < a.len && err.ok()) {
        if (!(err = pace.before_chunk()).ok()) break;
        const int64_t cnt = std::min<int64_t>(CH, a.len - k);
        if (use_graph && cnt == CH) {
            if (!exec) {
                hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess) {
                    err = Error::device(e, "hipStreamBeginCapture");
                    break;
                }
                for (int64_t i = 0; i < CH && err.ok(); ++i) {
                    err = launch_step(M, op1, op2, &so1, &so2, pl, mp, bufs, cur, nxt, slots + per_step * (size_t)i, st,
                                      to1, to2);
                    std::swap(cur, nxt);
                }
                e = hipStreamEndCapture(st, &graph);
                if (err.ok() && e != hipSuccess) err = Error::device(e, "hipStreamEndCapture");
                if (err.ok()) {
                    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                    if (e != hipSuccess) err = Error::device(e, "hipGraphInstantiate");
                }
                if (!err.ok()) break;
            }
            hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) {
                err = Error::device(e, "hipGraphLaunch");
                break;
            }
        } else {
            for (int64_t i = 0; i < cnt && err.ok(); ++i) {
                err = launch_step(M, op1, op2, &so1, &so2, pl, mp, bufs, cur, nxt, slots + per_step * (size_t)i, st,
                                  to1, to2);
                std::swap(cur, nxt);
            }
            if (!err.ok()) break;
        }
        hipError_t e = launch_reduce_partials(W, a.s, pl.NB, cnt, slots, a.S_out + (size_t)k * a.s * a.s, mp, st);
        if (e != hipSuccess) err = Error::device(e, "reduce launch");
        k += cnt;
        if (err.ok() && a.progress) err = a.progress(k);
        if (err.ok()) err = pace.after_chunk(st);
        if (err.ok() && a.stop && k < a.len && a.stop(k)) break;
    }
    const int64_t done_len = std::min(k, a.len);
    if (a.len_out) *a.len_out = done_len;
    // the graph is destroyed only once its launches have run: a launch in flight (and a tracer that inspects
    // its dispatches when they complete) must not outlive the executable graph
    // the symmetric projection's check: every term V^T B^k V must be symmetric (bit 2 of the flag)
    DevBuf symflag;
    if (err.ok() && a.symmetric) {
        hipError_t e = symflag.alloc(sizeof(int32_t), st).ok() ? launch_fill_zero(symflag.as<void>(), 4, st)
                                                                : hipErrorOutOfMemory;
        if (e == hipSuccess) e = launch_sym_check(done_len, a.s, a.S_out, symflag.as<int32_t>(), st);
        if (e != hipSuccess) err = Error::device(e, "symmetry check");
    }
    int32_t bad = 0, asym = 0;
    hipError_t he = hipSuccess;
    if (err.ok()) he = hipMemcpyAsync(&bad, flag.as<int32_t>(), sizeof(bad), hipMemcpyDeviceToHost, st);
    if (err.ok() && he == hipSuccess && a.symmetric)
        he = hipMemcpyAsync(&asym, symflag.as<int32_t>(), sizeof(asym), hipMemcpyDeviceToHost, st);
    const hipError_t hs = hipStreamSynchronize(st);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (!err.ok()) return err;
    if (he != hipSuccess) return Error::device(he, "hipMemcpyAsync");
    if (hs != hipSuccess) return Error::device(hs, "hipStreamSynchronize");
    if (bad) return Error::inval("d_col has an entry divisible by p");
    if (asym) return Error::device(hipErrorUnknown, "symmetric projection check: a term V^T B^k V is not symmetric");
    return {};
}

Error apply_once(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, const uint32_t* d_row,
                 const uint32_t* d_col, const uint32_t* X, uint32_t* Z, hipStream_t st) {
    if (M.sorted) return Error::inval("one application of B needs the plain (unsorted) encoding");
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
    // Z = D_c A^T D_r A D_c X; BWR_TILED=1 runs each product through the tiled kernel where it applies
    BWR_HIP(launch_pad_scale(nb, s, W, X, dcp, dcp ? 1 : 0, mp, Xp.as<void>(), 4, st));
    const bool split = mp.p > 65536u;
    const bool tiled = env_int("BWR_TILED", -1) == 1 && M.packed;
    TiledOp to1, to2;
    if (tiled && tiled_acc_ok(M, op1.max_len, mp.p)) {
        auto c = tile_candidates(op1.rows, nb, W, 4, split, false, M.max_abs);
        if (!c.empty()) BWR_TRY(build_tiled(op1, nb, M.nnz, M.max_abs, c[0], st, &to1));
        if (to1.on) BWR_HIP(launch_spmm_tiled(to1.v, W, 0, split, 4, Xp.as<void>(), drp, Y.as<void>(), nullptr,
                                              nullptr, nullptr, tiled_launch(to1, c[0]), mp, st));
    }
    if (!to1.on) BWR_TRY(spmm(M, op1, W, mp, Xp.as<uint32_t>(), drp, Y.as<uint32_t>(), st));
    if (tiled && tiled_acc_ok(M, op2.max_len, mp.p)) {
        auto c = tile_candidates(op2.rows, outer, W, 4, split, false, M.max_abs);
        if (!c.empty()) BWR_TRY(build_tiled(op2, outer, M.nnz, M.max_abs, c[0], st, &to2));
        if (to2.on) BWR_HIP(launch_spmm_tiled(to2.v, W, 0, split, 4, Y.as<void>(), dcp, Zp.as<void>(), nullptr,
                                              nullptr, nullptr, tiled_launch(to2, c[0]), mp, st));
    }
    if (!to2.on) BWR_TRY(spmm(M, op2, W, mp, Y.as<uint32_t>(), dcp, Zp.as<uint32_t>(), st));
    BWR_HIP(launch_unpad(nb, s, W, Zp.as<void>(), 4, Z, st));
    BWR_HIP(hipStreamSynchronize(st));
    return {};
}

Error time_step_kernels(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, int iters, hipStream_t st,
                        double us[3], StepPlan* plan_out) {
    const int W = padded_width(s);
    if (!W || iters < 1) return Error::inval("bad block size or iteration count");
    Operand op1, op2;
    operands(M, transpose, &op1, &op2);
    const int64_t nb = op2.rows, outer = op1.rows;
    StepPlan pl = plan_step(M, transpose, s, mp.p);
    if (M.nnz >= 100000 && env_int("BWR_NO_TUNE", 0) == 0 && getenv("BWR_G1") == nullptr && getenv("BWR_G2") == nullptr &&
        env_int("BWR_TILED", -1) != 1)
        BWR_TRY(tuned_plan(M, transpose, mp, &pl, st));
    if (plan_out) *plan_out = pl;
    const size_t es = (size_t)pl.esize;
    DevBuf X, Y, Z, U, d1, d2, part;
    BWR_TRY(X.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Z.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(U.alloc(es * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_TRY(Y.alloc(es * (size_t)std::max<int64_t>(outer * W, 1), st));
    BWR_TRY(d1.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(outer, 1), st));
    BWR_TRY(d2.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb, 1), st));
    BWR_TRY(part.alloc(sizeof(uint32_t) * (size_t)std::max(pl.NB, 1) * W * W, st));
    // random residues (in [0, p), so valid for either storage width)
    DevBuf tmp;
    BWR_TRY(tmp.alloc(sizeof(uint32_t) * (size_t)std::max<int64_t>(nb * W, 1), st));
    BWR_HIP(launch_rng_block(12345, 0, nb, W, W, mp, 0, tmp.as<uint32_t>(), st));
    BWR_HIP(launch_pad_scale(nb, W, W, tmp.as<uint32_t>(), nullptr, 0, mp, X.as<void>(), pl.esize, st));
    BWR_HIP(launch_rng_block(12345, 1, nb, W, W, mp, 0, tmp.as<uint32_t>(), st));
    BWR_HIP(launch_pad_scale(nb, W, W, tmp.as<uint32_t>(), nullptr, 0, mp, U.as<void>(), pl.esize, st));
    BWR_HIP(launch_rng_block(12345, 2, outer, 1, 1, mp, 1, d1.as<uint32_t>(), st));
    BWR_HIP(launch_rng_block(12345, 3, nb, 1, 1, mp, 1, d2.as<uint32_t>(), st));
    const bool smallp = mp.p <= 65536u;
    SplitOp so1, so2;
    if (pl.parts1 == 2) BWR_TRY(build_split(op1, nb, M.nnz, W, st, &so1));
    if (pl.parts2 == 2) BWR_TRY(build_split(op2, outer, M.nnz, W, st, &so2));
    TiledOp own1, own2;
    const TiledOp* to1 = nullptr;
    const TiledOp* to2 = nullptr;
    if (pl.t1.R > 0) BWR_TRY(get_tiled(M, op1, nb, pl.t1, st, &own1, &to1));
    if (pl.t2.R > 0) BWR_TRY(get_tiled(M, op2, outer, pl.t2, st, &own2, &to2));
    // [0] first product, [1] second product (+ projection when fused), [2] separate projection (0 when fused);
    // a product in two column passes counts both
    BWR_TRY(time_launches(iters, st, [&]() -> Error {
        if (pl.G1 > 0 || to1) {
            hipError_t e = first_product(M, op1, &so1, pl.G1, pl, mp, X.as<void>(), d1.as<uint32_t>(), Y.as<void>(), st,
                                         to1);
            return e == hipSuccess ? Error{} : Error::device(e, "sparse product (first)");
        }
        return spmm(M, op1, W, mp, X.as<uint32_t>(), d1.as<uint32_t>(), Y.as<uint32_t>(), st);
    }, &us[0]));
    BWR_TRY(time_launches(iters, st, [&]() -> Error {
        if (pl.G2 > 0 || to2) {
            hipError_t e = second_product(M, op2, &so2, pl.G2, pl.fused, pl.NB, pl, mp, Y.as<void>(),
                                          d2.as<uint32_t>(), Z.as<void>(), U.as<void>(), part.as<uint32_t>(), st, to2);
            return e == hipSuccess ? Error{} : Error::device(e, "spmm_split");
        }
        return spmm(M, op2, W, mp, Y.as<uint32_t>(), d2.as<uint32_t>(), Z.as<uint32_t>(), st);
    }, &us[1]));
    us[2] = 0;
    if (!pl.fused && nb > 0)
        BWR_TRY(time_launches(iters, st, [&]() -> Error {
            hipError_t e = launch_project(W, smallp, nb, U.as<void>(), Z.as<void>(), pl.esize, part.as<uint32_t>(),
                                          pl.NB, mp, st);
            return e == hipSuccess ? Error{} : Error::device(e, "project");
        }, &us[2]));
    return {};
}

}  // namespace bwr
