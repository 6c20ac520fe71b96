// Device runtime of the block Wiedemann path: the encoded matrix store and the
// sequence driver.  Internal C++; the public surface is the C-ABI in bwrank.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "modp.h"

namespace bwr {

// Error codes of the C-ABI (mirrored in bwrank.h).
enum : int { OK = 0, EINVAL_ = -1, EPRIME_ = -2, ENOMEM_ = -3, EDEVICE_ = -4, EBUSY_ = -5, ESHORT_ = -6 };

struct Error {
    int code = OK;
    std::string msg;
    bool ok() const { return code == OK; }
    static Error inval(const std::string& m) { return {EINVAL_, m}; }
    static Error device(hipError_t e, const char* where);
};

// A device region that DevBuf::alloc carves from, instead of allocating, while it is installed on the calling
// thread (ArenaScope): the caller-workspace entry points and the entry point that allocates nothing.  Carving
// is a bump of `used` (256-byte aligned); a buffer released while it is the topmost one gives its bytes back.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0, peak = 0;
};
class ArenaScope {
   public:
    explicit ArenaScope(Arena* a);
    ~ArenaScope();
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;

   private:
    Arena* prev_;
};
Arena* current_arena();
// device allocations the library has made so far (every DevBuf that did not come from an arena)
int64_t device_allocations();

// The static device scratch of the entry point that allocates nothing (noalloc.hip): its size, and on the
// current device its address (resolved once per device) with the lock its users take turns under.
size_t noalloc_scratch_bytes();
Error noalloc_scratch(void** ptr, std::mutex** use);

// Device buffer owned by the library (freed on destruction, stream-ordered), or carved from the installed
// arena.
class DevBuf {
   public:
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept;
    ~DevBuf() { release(); }
    Error alloc(size_t bytes, hipStream_t st);
    void release();
    // the stream a later release is ordered on (a buffer kept beyond the stream it was made on)
    void set_stream(hipStream_t st) { st_ = st; }
    template <class T>
    T* as() const { return reinterpret_cast<T*>(ptr_); }
    size_t bytes() const { return bytes_; }

   private:
    void* ptr_ = nullptr;
    size_t bytes_ = 0;
    hipStream_t st_ = nullptr;
    Arena* arena_ = nullptr;  // set when carved from an arena
};

struct TiledStore;  // tiled encodings kept with a matrix (engine.cpp)

// A sparse integer matrix on the device, encoded for the two products of a
// step: CSR of A and CSR of A^T.  Packed form (prime independent): column
// index in the low 24 bits and the int8 value in the high 8 bits of one
// uint32.  Wide form (one prime): int32 columns and uint32 residues.
struct DeviceMatrix {
    int64_t m = 0, n = 0, nnz = 0;
    int32_t max_len_a = 0, max_len_t = 0, max_abs = 0;
    bool packed = true;
    uint32_t wide_p = 0;  // prime the wide values are reduced for
    DevBuf rp_a, ent_a, rp_t, ent_t;     // packed (ent) or wide columns (ent as int32)
    DevBuf val_a, val_t;                 // wide residues
    // Length-sorted encoding: row i of the encoded A is row perm_r[i] of the input and column j is input
    // column perm_c[j] (int32, device), so that rows of A and of A^T come in order of decreasing length
    bool sorted = false;
    DevBuf perm_r, perm_c;
    // Optional store of the tiled encodings the sequences of this matrix use (engine.cpp), for matrices kept
    // across calls: each geometry is built once and reused.  Null: built per call.
    std::shared_ptr<TiledStore> tiled;
};

// A store for DeviceMatrix::tiled whose buffers are released on stream `home`.
std::shared_ptr<TiledStore> make_tiled_store(hipStream_t home);
// Orders the later release of every buffer of M on stream `home`.
void rehome(DeviceMatrix& M, hipStream_t home);

struct CsrView {  // caller-owned CSR (host or device pointers)
    int64_t m, n, nnz;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* val;
};

// Validate and encode a device-resident CSR.  p is used only by the wide form
// (values beyond int8 or dimensions beyond 2^24).  With sort, the rows and the
// columns are relabelled in order of decreasing length (a wave of the row-split
// kernels then holds rows of similar length, so its dependent load chains are
// about as long as its rows need, not as long as the longest row of a random
// mix); run_sequence permutes the draws to match, so every S_k is unchanged
// (S_k = U^T B^k V is invariant under a simultaneous relabelling).
// BWR_NO_SORT=1 turns the relabelling off.
Error encode_matrix(const CsrView& A_dev, uint32_t p, hipStream_t st, DeviceMatrix* out, bool sort = false);

// Host CSR checks (row pointers, column range) before any upload.
Error check_host_csr(const CsrView& A);

struct Operand {  // one product of a step: out[r] = scale[r] * sum a_rt in[col_t]
    int64_t rows;
    int32_t max_len;
    const int32_t* rp;
    const uint32_t* ent;  // packed entries, or wide columns
    const uint32_t* val;  // wide residues (null when packed)
};

// One sequence run: S_k = U^T B^k V for k < len, B = D_c A^T D_r A D_c, or with
// the roles of A and A^T swapped (transpose = true: B acts on GF(p)^m).
// Kernel choice for one step: padded width W, lanes per row slice of each
// product (0 = one lane group per row, the legacy kernels), whether the
// projection is fused into the second product, and the number of projection
// partials per step.
struct StepPlan {
    int W = 0;
    int G1 = 0, G2 = 0;
    bool fused = false;
    int NB = 0;
    int esize = 4;  // bytes per stored residue of the iterated blocks (2 when p <= 2^16)
    // column parts of each product (1 or 2): with 2, the entries gathering from each half of the block
    // run as separate passes (32-bit residues only), so that each pass gathers from a half that fits L2
    int parts1 = 1, parts2 = 1;
    // two-dimensional tiled form of a product (spmm_tiled.hip), R = 0: not tiled.  nrb interleaved row
    // blocks of at most R output rows, 2^cb gathered rows per slab, grid persistent workgroups.  A tiled
    // second product always has the projection fused, with one partial per workgroup (NB = t2.grid).
    struct Tile {
        int R = 0, cb = 0, grid = 0;
        int64_t nrb = 0;
        int un = 1;  // entries each lane takes per pass (see TiledLaunch)
    };
    Tile t1, t2;
};

struct SequenceArgs {
    const DeviceMatrix* M;
    bool transpose = false;
    ModP mp;
    int32_t s;
    const uint32_t* d_row = nullptr;  // device, rows of the first product, or null
    const uint32_t* d_col = nullptr;  // device, length of the iterated dimension, or null
    const uint32_t* U = nullptr;      // device, nb x s
    const uint32_t* V = nullptr;      // device, nb x s
    int64_t len = 0;
    uint32_t* S_out = nullptr;  // device, len x s x s
    StepPlan* plan_out = nullptr;  // optional: the plan used
    // optional: called from the enqueueing thread each time the reductions of the terms
    // S_0 .. S_{t-1} have been enqueued on the sequence stream (t increasing, last t = len)
    std::function<Error(int64_t t)> progress;
    // optional: asked after each progress(t); true ends the sequence there, with S_0 .. S_{t-1} complete.
    // While it is set the enqueueing thread stays at most two chunks of steps ahead of the device, so that
    // a stop is taken close to the device's position rather than after every chunk has been queued.
    std::function<bool(int64_t t)> stop;
    int64_t* len_out = nullptr;  // optional: the number of terms computed (len unless stopped)
    // Symmetric projection U = V (U is ignored): S_k = V^T B^k V (Section 2.3), every term checked to be
    // symmetric after the run (an error otherwise).  With gram, two terms per application of B through the
    // weighted Gram identities of symmetric.hip (terms exact, symmetric by construction; not in the paper).
    bool symmetric = false;
    bool gram = false;
};

Error run_sequence(const SequenceArgs& a, hipStream_t st);

// Z = B X for one block (no projection): parity hook for a single step.
Error apply_once(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, const uint32_t* d_row,
                 const uint32_t* d_col, const uint32_t* X, uint32_t* Z, hipStream_t st);

int padded_width(int32_t s);  // 0 if unsupported

// Average device time (microseconds, HIP events on stream st) of each kernel
// of one step, launched `iters` times back to back on the encoded matrix with
// random blocks: [0] first sparse product + row scale, [1] second sparse
// product + column scale (+ the projection when fused), [2] the separate
// projection (0 when fused).
Error time_step_kernels(const DeviceMatrix& M, bool transpose, ModP mp, int32_t s, int iters, hipStream_t st,
                        double us[3], StepPlan* plan_out = nullptr);

// Heuristic plan, and its refinement by timing every valid split factor on M.
// allow_tiled = false: only the row-split kernels (the plan used inside an arena, whose memory need has a
// closed form: sequence_workspace_bytes).
StepPlan plan_step(const DeviceMatrix& M, bool transpose, int32_t s, uint32_t p, bool allow_tiled = true);

// Device bytes an arena must hold for encode_matrix (sorted) plus run_sequence on an m x n matrix with nnz
// entries, block s, B on the n side (transpose = false) or the m side: an upper bound, counted from the
// buffers those functions carve (see engine.cpp).
size_t sequence_workspace_bytes(int64_t m, int64_t n, int64_t nnz, int32_t s, bool transpose);
// Steps per chunk of partial sums inside an arena.
constexpr int64_t ARENA_CHUNK = 16;
Error autotune_step(const DeviceMatrix& M, bool transpose, ModP mp, StepPlan* pl, hipStream_t st);

}  // namespace bwr
