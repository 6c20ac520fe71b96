// C-ABI of libbwrank (declared and documented in include/bwrank.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/bwrank.h"
#include "engine.h"
#include "kernels.h"
#include "sigma.h"
#include "sigma_gpu.h"
#include "batch_runner.h"
#include "readout.h"
#include "server.h"
#include "splitmix.h"

using namespace bwr;

namespace {

thread_local std::string g_err;

// independent draws per rank computation (bwr_set_trials)
std::atomic<int32_t> g_trials{1};
// early termination of single-matrix ranks (bwr_set_early_termination)
std::atomic<int32_t> g_early{0};
// further draws where the primes of a batched matrix disagree (bwr_set_batch_retry)
std::atomic<int32_t> g_batch_retry{0};
// early termination's cut lengths: at least these many orders, else L / 32 and an eighth of that
constexpr int64_t EARLY_MIN_STEP = 512;
constexpr int64_t EARLY_MIN_VERIFY = 128;

int fail(const Error& e) {
    g_err = e.msg;
    return e.code;
}
int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool is_prime_u32(uint32_t p) {
    if (p < 2) return false;
    for (uint32_t d : {2u, 3u, 5u, 7u, 11u, 13u, 17u, 19u, 23u, 29u, 31u, 37u})
        if (p % d == 0) return p == d;
    uint32_t dd = p - 1;
    int r = 0;
    while (!(dd & 1)) {
        dd >>= 1;
        ++r;
    }
    ModP mp = ModP::make(p);
    for (uint32_t a : {2u, 7u, 61u}) {
        if (a % p == 0) continue;
        uint32_t x = powmod(mp, a % p, dd);
        if (x == 1 || x == p - 1) continue;
        bool comp = true;
        for (int i = 1; i < r; ++i) {
            x = mulmod(mp, x, x);
            if (x == p - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

Error check_prime(uint32_t p) {
    if (p < 3 || p >= (1u << 31) || !is_prime_u32(p)) return {EPRIME_, "p must be a prime in [3, 2^31)"};
    return {};
}

// Library streams of the calling host thread on the current device: stream 0 runs an entry point's work,
// stream 1 the sigma-basis that runs beside a rank computation's sequence.  They are non-blocking and per
// (host thread, device), so calls made from different host threads run concurrently on the device (e.g.
// one prime's sigma-basis beside another prime's sequence).
// The thread that loaded the library (normally the process's main thread): its streams are left to the
// runtime at process exit, when destroying them could outlive the runtime itself.
const std::thread::id g_load_thread = std::this_thread::get_id();

// A host thread's library streams, destroyed when the thread ends (pending work finishes first).
struct ThreadStreams {
    std::vector<hipStream_t> v;
    ~ThreadStreams() {
        if (std::this_thread::get_id() == g_load_thread) return;
        for (hipStream_t s : v)
            if (s) (void)hipStreamDestroy(s);
    }
};

hipStream_t lib_stream(Error* err, int which = 0) {
    thread_local ThreadStreams tls;
    std::vector<hipStream_t>& streams = tls.v;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *err = Error::device(e, "hipGetDevice");
        return nullptr;
    }
    const size_t slot = (size_t)dev * 2 + (which ? 1 : 0);
    if (streams.size() <= slot) streams.resize(slot + 1, nullptr);
    if (!streams[slot]) {
        e = hipStreamCreateWithFlags(&streams[slot], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[slot] = nullptr;
            *err = Error::device(e, "hipStreamCreate");
            return nullptr;
        }
        // keep freed device memory cached by the pool between calls
        static std::mutex mu;
        std::lock_guard<std::mutex> lk(mu);
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    }
    return streams[slot];
}

// Smallest chunk of the sigma-basis that runs beside the sequence (OnlineGenerator) for a sequence of
// L terms; 0 runs it after the sequence.  BWR_SIGMA_MIN_CHUNK overrides (0 = after the sequence).
int64_t online_min_chunk(int64_t L) {
    if (const char* v = getenv("BWR_SIGMA_MIN_CHUNK")) return std::max<int64_t>(0, atoll(v));
    return L >= 4096 ? std::max<int64_t>(1024, L / 8) : 0;
}

// Device entry points run on the library stream (which sequence capture needs:
// the legacy null stream cannot be captured), after the caller's stream has
// drained; they return once their own work has completed.
hipStream_t work_stream(void* user, Error* err) {
    hipError_t e = hipStreamSynchronize((hipStream_t)user);
    if (e != hipSuccess) {
        *err = Error::device(e, "hipStreamSynchronize (caller stream)");
        return nullptr;
    }
    return lib_stream(err);
}

CsrView view(const bwr_csr* A) { return CsrView{A->m, A->n, A->nnz, A->row_ptr, A->col_idx, A->val}; }

// Host CSR -> device copies (owned by the returned buffers).
struct HostUpload {
    DevBuf rp, col, val;
    CsrView dev{};
};

Error upload(const bwr_csr* A, hipStream_t st, HostUpload* u) {
    Error e = check_host_csr(view(A));
    if (!e.ok()) return e;
    const size_t nnz = (size_t)A->nnz;
    if (!(e = u->rp.alloc(sizeof(int64_t) * (size_t)(A->m + 1), st)).ok()) return e;
    if (!(e = u->col.alloc(sizeof(int32_t) * std::max<size_t>(nnz, 1), st)).ok()) return e;
    if (!(e = u->val.alloc(sizeof(int32_t) * std::max<size_t>(nnz, 1), st)).ok()) return e;
    hipError_t he = hipMemcpyAsync(u->rp.as<void>(), A->row_ptr, sizeof(int64_t) * (size_t)(A->m + 1),
                                   hipMemcpyHostToDevice, st);
    if (he == hipSuccess && nnz)
        he = hipMemcpyAsync(u->col.as<void>(), A->col_idx, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st);
    if (he == hipSuccess && nnz)
        he = hipMemcpyAsync(u->val.as<void>(), A->val, sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st);
    if (he != hipSuccess) return Error::device(he, "upload");
    u->dev = CsrView{A->m, A->n, A->nnz, u->rp.as<int64_t>(), u->col.as<int32_t>(), u->val.as<int32_t>()};
    return {};
}

Error copy_to_dev(const uint32_t* h, size_t count, hipStream_t st, DevBuf* d) {
    Error e = d->alloc(sizeof(uint32_t) * std::max<size_t>(count, 1), st);
    if (!e.ok()) return e;
    if (count) {
        hipError_t he = hipMemcpyAsync(d->as<void>(), h, sizeof(uint32_t) * count, hipMemcpyHostToDevice, st);
        if (he != hipSuccess) return Error::device(he, "hipMemcpyAsync");
    }
    return {};
}

Error sequence_dev_impl(const CsrView& A, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                        const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, hipStream_t st) {
    Error e = check_prime(p);
    if (!e.ok()) return e;
    if (s < 1 || s > 64) return Error::inval("block size must be in 1..64");
    if (len < 0) return Error::inval("len must be >= 0");
    if (len > 0 && (!S_out || (A.n > 0 && (!U || !V)))) return Error::inval("NULL output or block");
    if (len == 0) return {};
    DeviceMatrix M;
    if (!(e = encode_matrix(A, p, st, &M, true)).ok()) return e;
    SequenceArgs a;
    a.M = &M;
    a.transpose = false;
    a.mp = ModP::make(p);
    a.s = s;
    a.d_row = d_row;
    a.d_col = d_col;
    a.U = U;
    a.V = V;
    a.len = len;
    a.S_out = S_out;
    return run_sequence(a, st);
}

struct RankOut {
    int64_t rank = 0;
    bwr_rank_info info{};
    bool stopped_early = false;  // the sequence of the draw stopped before its full length
};

constexpr int64_t CHECK_TERMS = 4;

// Largest block (all of a job's primes side by side) a matrix may gather from in the batched launches,
// and the host threads of the single-matrix solves beside them.  Measured on the batched configuration
// (16 matrices x 3 16-bit primes and 2^31 - 1): 2 MB with the 16-bit primes batched in 16-bit residues
// and the large prime as single-matrix solves gave 1.15x the one-at-a-time rate; 8 MB gave 0.89x (the
// batched kernel loses to the single-matrix kernels once the block outgrows an XCD's L2); batching all four
// primes in 32-bit residues with 8 MB gave 1.08-1.11x.
constexpr int64_t BATCH_BLOCK_BYTES = 2 << 20;
constexpr int BATCH_SOLO_THREADS = 2;  // all 64 matrices x 4 primes: 2 threads 1.06x, 3 threads 1.02x

int64_t env_i64(const char* name, int64_t dflt) {
    const char* v = getenv(name);
    return (v && *v) ? atoll(v) : dflt;
}

// Waits for a stream's work at scope exit (so that buffers it reads outlive it on every return path).
struct StreamDrain {
    hipStream_t st = nullptr;
    ~StreamDrain() {
        if (st) (void)hipStreamSynchronize(st);
    }
};

// One draw of the rank algorithm on an encoded matrix (Section 2.5, steps 1-4): U, V, D_r, D_c from `seed`,
// the sequence with the sigma-basis beside it, the generator check and the read-out.
// proj: 0 = independent U and V; 1 = symmetric projection U = V (Section 2.3); 2 = symmetric, in Gram form.
Error rank_one_draw(const DeviceMatrix& M, const CsrView& A, uint32_t p, int32_t block, uint64_t seed, hipStream_t st,
                    RankOut* out, int proj, bool allow_early = true) {
    Error e;
    bwr_rank_info& info = out->info;
    const bool transpose = A.m < A.n;
    const int64_t nb = std::min(A.m, A.n);
    const int64_t outer = std::max(A.m, A.n);
    const int32_t s = (int32_t)std::min<int64_t>(block, nb);
    const int64_t L = 2 + (2 * nb + s - 1) / s;
    const int64_t total = L + CHECK_TERMS;
    // inside an arena the generator is computed on the host (the device sigma-basis allocates as it recurses)
    const bool on_device = gpu_leaf_order(s) > 0 && !getenv("BWR_HOST_SIGMA") && !current_arena();
    const int64_t min_chunk = on_device ? online_min_chunk(L) : 0;
    // early termination needs the basis beside the sequence
    const bool early = allow_early && min_chunk > 0 && g_early.load() != 0;
    info.s = s;
    info.len = L;
    info.check_terms = CHECK_TERMS;
    info.terms = total;
    const ModP mp = ModP::make(p);
    DevBuf U, V, dr, dc, S;
    if (!(e = U.alloc(sizeof(uint32_t) * (size_t)(nb * s), st)).ok()) return e;
    if (!(e = V.alloc(sizeof(uint32_t) * (size_t)(nb * s), st)).ok()) return e;
    if (!(e = dr.alloc(sizeof(uint32_t) * (size_t)outer, st)).ok()) return e;
    if (!(e = dc.alloc(sizeof(uint32_t) * (size_t)nb, st)).ok()) return e;
    if (!(e = S.alloc(sizeof(uint32_t) * (size_t)(total * s * s), st)).ok()) return e;
    hipError_t he = launch_rng_block(seed, STREAM_V, nb, s, s, mp, 0, V.as<uint32_t>(), st);
    if (he == hipSuccess) he = launch_rng_block(seed, STREAM_U, nb, s, s, mp, 0, U.as<uint32_t>(), st);
    if (he == hipSuccess) he = launch_rng_block(seed, STREAM_DROW, outer, 1, 1, mp, 1, dr.as<uint32_t>(), st);
    if (he == hipSuccess) he = launch_rng_block(seed, STREAM_DCOL, nb, 1, 1, mp, 1, dc.as<uint32_t>(), st);
    if (he != hipSuccess) return Error::device(he, "rng launch");
    SequenceArgs a;
    a.M = &M;
    a.transpose = transpose;
    a.mp = mp;
    a.s = s;
    a.d_row = dr.as<uint32_t>();
    a.d_col = dc.as<uint32_t>();
    a.U = U.as<uint32_t>();
    a.V = V.as<uint32_t>();
    a.len = total;
    a.S_out = S.as<uint32_t>();
    a.symmetric = proj != 0;
    a.gram = proj == 2;
    // device sigma-basis: its chunks run on stream 1 as the terms they need are reduced
    StreamDrain drain;  // declared first so that it runs after og's destructor has joined og's thread
    OnlineGenerator og;
    if (min_chunk > 0) {
        hipStream_t sst = lib_stream(&e, 1);
        if (!e.ok()) return e;
        drain.st = sst;
        if (early) {
            // BWR_EARLY_STEP and BWR_EARLY_VERIFY override the cut lengths (tests use tiny ones)
            const int64_t step = env_i64("BWR_EARLY_STEP", std::max<int64_t>(EARLY_MIN_STEP, L / 32));
            const int64_t verify = env_i64("BWR_EARLY_VERIFY", std::max<int64_t>(EARLY_MIN_VERIFY, step / 8));
            e = og.begin_early(S.as<uint32_t>(), L, s, p, step, verify, sst);
            if (e.ok()) og.force_converge_at(env_i64("BWR_EARLY_FORCE_AT", 0));
        } else {
            e = og.begin(S.as<uint32_t>(), L, s, p, min_chunk, sst);
        }
        if (!e.ok()) return e;
        // The generator's thread waits on the host for an event of st.  st captures a graph only for the
        // sequence's first chunk of steps (at least 32; graphs need two chunks' worth of terms, so L >= 61),
        // progress is called with t = 1 before that chunk and with t > 32 after it, and the first boundary
        // (a quarter of L, >= 15 when a graph is used) exceeds 1: st is never capturing during such a wait.
        // In early-termination mode every chunk of terms after the first is fed (t = 1 comes before the
        // captured chunk, so it is skipped there too), and the sequence stops once the basis has converged
        // and the terms it will be checked on are complete.
        a.progress = [&](int64_t t) -> Error {
            if (early) {
                if (t <= 1) return {};
            } else {
                const int64_t next = og.next_boundary();
                if (next < 0 || t < next) return {};
            }
            hipEvent_t ev = nullptr;
            hipError_t r = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (r == hipSuccess) r = hipEventRecord(ev, st);
            if (r != hipSuccess) {
                if (ev) (void)hipEventDestroy(ev);
                return Error::device(r, "hipEventRecord");
            }
            og.feed_async(t, ev);
            return {};
        };
        if (early)
            a.stop = [&](int64_t t) -> bool {
                const int64_t c = og.converged();
                return c > 0 && t >= c + CHECK_TERMS;
            };
    }
    int64_t have = total;  // terms computed
    a.len_out = &have;
    const double t1 = now_s();
    if (!(e = run_sequence(a, st)).ok()) return e;
    he = hipStreamSynchronize(st);
    if (he != hipSuccess) return Error::device(he, "sequence");
    const double t2 = now_s();
    info.t_sequence = t2 - t1;
    Generator g;
    SigmaStats ss;
    int64_t Lg = L;  // order of the generator's basis
    std::vector<uint32_t> Sh((size_t)(have * s * s));
    if (on_device && min_chunk > 0) {
        if (have < total && og.converged() == 0) return Error::inval("sequence stopped before the basis converged");
        // after a stop the basis has converged and ignores further terms; otherwise feed them all
        if (have == total) og.feed_async(L, nullptr);
        if (!(e = og.finish(&g)).ok()) return e;
        Lg = og.order();
        if (Lg + CHECK_TERMS > have) return Error::inval("too few terms past the generator's order to check it");
        info.len = Lg;
        info.terms = have;
        out->stopped_early = Lg < L;
        he = hipMemcpyAsync(Sh.data(), S.as<void>(), sizeof(uint32_t) * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
    } else if (on_device) {
        if (!(e = gpu_min_generator(S.as<uint32_t>(), L, s, p, st, &g, &ss)).ok()) return e;
        he = hipMemcpyAsync(Sh.data(), S.as<void>(), sizeof(uint32_t) * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
    } else {
        he = hipMemcpyAsync(Sh.data(), S.as<void>(), sizeof(uint32_t) * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
        if (!(e = min_generator(Sh.data(), L, s, p, &g, &ss)).ok()) return e;
    }
    const double t3 = now_s();
    info.t_sigma = t3 - t2;
    info.sigma_threads = on_device ? 0 : ss.threads;
    // the same number of check terms as the full length has (after an early stop more terms may be there:
    // checking each costs about s^3 (L / s) operations on the host, 15 ms at 2M x 1M)
    if (!(e = check_generator(g, Sh.data(), Lg, Lg + CHECK_TERMS, p)).ok()) return e;
    int64_t r = 0;
    if (!(e = rank_from_generator(g, p, &r)).ok()) return e;
    info.t_readout = now_s() - t3;
    for (int64_t x : g.delta) info.sum_delta += x;
    info.rank = r;
    out->rank = r;
    return {};
}



// Rank of A with `trials` independent draws (seeds seed, seed + 1, ...): each draw's result is at most the
// true rank (the method's error is one-sided, Section 2.5), so the largest is kept; the draws stop early
// once a draw reaches min(m, n).  The matrix is encoded once for all draws.
Error rank_dev_impl(const CsrView& A, uint32_t p, int32_t block, uint64_t seed, hipStream_t st, RankOut* out,
                    int32_t trials, int proj = 0) {
    Error e = check_prime(p);
    if (!e.ok()) return e;
    if (block < 1 || block > 64) return Error::inval("block size must be in 1..64");
    if (trials < 1) return Error::inval("trials must be >= 1");
    std::memset(&out->info, 0, sizeof(out->info));
    const double t0 = now_s();
    const int64_t nb = std::min(A.m, A.n);
    DeviceMatrix M;
    if (!(e = encode_matrix(A, p, st, &M, true)).ok()) return e;
    const double t_enc = now_s() - t0;
    out->info.nb = nb;
    out->info.transposed = A.m < A.n ? 1 : 0;
    out->info.t_encode = t_enc;
    out->info.trials = 0;
    out->rank = 0;
    if (nb == 0 || A.nnz == 0) return {};
    double tseq = 0, tsig = 0, tro = 0;
    for (int32_t t = 0; t < trials; ++t) {
        RankOut one;
        std::memset(&one.info, 0, sizeof(one.info));
        one.info.nb = nb;
        one.info.transposed = A.m < A.n ? 1 : 0;
        e = rank_one_draw(M, A, p, block, seed + (uint64_t)t, st, &one, proj);
        if (e.code == ESHORT_ && one.stopped_early) {
            // the generator kept by early termination failed its check (a premature stall): the same draw
            // again at the full length
            std::memset(&one.info, 0, sizeof(one.info));
            one.info.nb = nb;
            one.info.transposed = A.m < A.n ? 1 : 0;
            one.stopped_early = false;
            e = rank_one_draw(M, A, p, block, seed + (uint64_t)t, st, &one, proj, false);
        }
        if (!e.ok()) return e;
        tseq += one.info.t_sequence;
        tsig += one.info.t_sigma;
        tro += one.info.t_readout;
        if (t == 0 || one.rank > out->rank) {
            const int64_t best_before = out->rank;
            out->info = one.info;
            out->rank = one.rank;
            (void)best_before;
        }
        out->info.trials = t + 1;
        if (out->rank >= nb) break;
    }
    out->info.t_encode = t_enc;
    out->info.t_sequence = tseq;
    out->info.t_sigma = tsig;
    out->info.t_readout = tro;
    return {};
}

int pow2_at_most(double x, int lo, int hi) {
    int g = lo;
    while (g * 2 <= hi && g * 2 <= x) g *= 2;
    return g;
}

struct BatchPlan {
    int W = 0, G1 = 0, G2 = 0, per_job = 0;
};

struct Shape {
    int64_t rows1, rows2, nnz;
};

BatchPlan plan_batch(const std::vector<Shape>& shapes, int nprimes, int s) {
    BatchPlan bp;
    const int spad = (s + 3) & ~3;
    if (spad > 32) return bp;
    bp.per_job = std::max(1, std::min(nprimes, 32 / spad));
    bp.W = BatchRunner::width_for(bp.per_job, s);
    double r1 = 0, r2 = 0, nz = 0;
    for (const Shape& sh : shapes) {
        r1 += (double)sh.rows1;
        r2 += (double)sh.rows2;
        nz += (double)sh.nnz;
    }
    const double a1 = r1 > 0 ? nz / r1 : 1, a2 = r2 > 0 ? nz / r2 : 1;
    const int cg = bp.W / 4;
    bp.G1 = pow2_at_most(a1 / 4.0 + 1.0, 1, std::max(1, 64 / cg));
    bp.G2 = pow2_at_most(a2 / 4.0 + 1.0, std::max(1, bp.W / 4), std::max(1, 64 / cg));
    if (const char* e = getenv("BWR_BATCH_G1")) bp.G1 = atoi(e);
    if (const char* e = getenv("BWR_BATCH_G2")) bp.G2 = atoi(e);
    if (!batch_supported(bp.W, bp.G1, false) || !batch_supported(bp.W, bp.G2, true)) bp.W = 0;
    return bp;
}

}  // namespace

// The single-matrix rank of a device CSR, as bwr_rank_modp_dev with `trials` draws (the server's lane for
// large requests).
Error bwr::rank_single(const CsrView& A_dev, uint32_t p, int32_t block, uint64_t seed, int32_t trials,
                       hipStream_t st, int64_t* rank) {
    RankOut ro;
    Error e = rank_dev_impl(A_dev, p, block, seed, st, &ro, trials);
    if (e.ok()) *rank = ro.rank;
    return e;
}

struct bwr_server {
    std::unique_ptr<bwr::Server> impl;
};

extern "C" {

int bwr_version(void) { return 100; }

const char* bwr_last_error(void) { return g_err.c_str(); }

int bwr_is_prime(uint32_t p) { return (p >= 3 && p < (1u << 31) && is_prime_u32(p)) ? 1 : 0; }

int64_t bwr_sequence_length(int64_t nb, int32_t s) {
    if (s < 1 || nb < 0) return -1;
    return 2 + (2 * nb + s - 1) / s;
}

int bwr_set_trials(int32_t n) {
    if (n < 1 || n > 64) return fail(BWR_EINVAL, "trials must be in 1..64");
    g_trials.store(n);
    g_err.clear();
    return BWR_OK;
}

int32_t bwr_get_trials(void) { return g_trials.load(); }

int bwr_set_early_termination(int32_t on) {
    if (on != 0 && on != 1) return fail(BWR_EINVAL, "early termination is 0 (off) or 1 (on)");
    g_early.store(on);
    g_err.clear();
    return BWR_OK;
}

int32_t bwr_get_early_termination(void) { return g_early.load(); }

int bwr_set_batch_retry(int32_t n) {
    if (n < 0 || n > 16) return fail(BWR_EINVAL, "batch retry must be in 0..16");
    g_batch_retry.store(n);
    g_err.clear();
    return BWR_OK;
}

int32_t bwr_get_batch_retry(void) { return g_batch_retry.load(); }

int bwr_set_threads(int32_t n) {
    if (n < 1) return fail(BWR_EINVAL, "thread count must be positive");
    set_sigma_threads(n);
    g_err.clear();
    return BWR_OK;
}

int bwr_random_block(uint64_t seed, int32_t stream, int64_t rows, int32_t s, uint32_t p, int32_t diag,
                     uint32_t* out) {
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (rows < 0 || s < 1 || stream < 0 || (rows > 0 && !out)) return fail(BWR_EINVAL, "bad arguments");
    ModP mp = ModP::make(p);
    uint64_t key = sm_key(seed, stream);
    for (int64_t i = 0; i < rows * (int64_t)s; ++i) out[i] = sm_residue(mp, key, (uint64_t)i, diag ? 1 : 0);
    g_err.clear();
    return BWR_OK;
}

int bwr_sequence(const bwr_csr* A, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                 const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out) {
    if (!A) return fail(BWR_EINVAL, "A is NULL");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64 || len < 0) return fail(BWR_EINVAL, "block size must be in 1..64 and len >= 0");
    if (len > 0 && (!S_out || (A->n > 0 && (!U || !V)))) return fail(BWR_EINVAL, "NULL output or block");
    if (!(e = check_host_csr(view(A))).ok()) return fail(e);
    if (len == 0) {
        g_err.clear();
        return BWR_OK;
    }
    hipStream_t st = lib_stream(&e);
    if (!e.ok()) return fail(e);
    HostUpload up;
    DevBuf dU, dV, ddr, ddc, dS;
    if (!(e = upload(A, st, &up)).ok()) return fail(e);
    const size_t ns = (size_t)A->n * s;
    if (!(e = copy_to_dev(U, ns, st, &dU)).ok()) return fail(e);
    if (!(e = copy_to_dev(V, ns, st, &dV)).ok()) return fail(e);
    if (d_row && !(e = copy_to_dev(d_row, (size_t)A->m, st, &ddr)).ok()) return fail(e);
    if (d_col && !(e = copy_to_dev(d_col, (size_t)A->n, st, &ddc)).ok()) return fail(e);
    const size_t nS = (size_t)len * s * s;
    if (!(e = dS.alloc(sizeof(uint32_t) * nS, st)).ok()) return fail(e);
    e = sequence_dev_impl(up.dev, d_row ? ddr.as<uint32_t>() : nullptr, d_col ? ddc.as<uint32_t>() : nullptr,
                          dU.as<uint32_t>(), dV.as<uint32_t>(), p, s, len, dS.as<uint32_t>(), st);
    if (!e.ok()) return fail(e);
    std::vector<uint32_t> tmp(nS);
    hipError_t he = hipMemcpyAsync(tmp.data(), dS.as<void>(), sizeof(uint32_t) * nS, hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) return fail(Error::device(he, "download"));
    std::memcpy(S_out, tmp.data(), sizeof(uint32_t) * nS);
    g_err.clear();
    return BWR_OK;
}

int bwr_sequence_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                     const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream) {
    if (!A_dev) return fail(BWR_EINVAL, "A is NULL");
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    e = sequence_dev_impl(view(A_dev), d_row, d_col, U, V, p, s, len, S_out, st);
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_apply_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* X,
                  uint32_t p, int32_t s, uint32_t* Z, void* stream) {
    if (!A_dev) return fail(BWR_EINVAL, "A is NULL");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    if (A_dev->n > 0 && (!X || !Z)) return fail(BWR_EINVAL, "NULL block");
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    DeviceMatrix M;
    if (!(e = encode_matrix(view(A_dev), p, st, &M)).ok()) return fail(e);
    if (!(e = apply_once(M, false, ModP::make(p), s, d_row, d_col, X, Z, st)).ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

// ---- the sequence without any device allocation ----

int bwr_sequence_dev_noalloc(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                             const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream) {
    if (!A_dev) return fail(BWR_EINVAL, "NULL matrix");
    if (s < 1 || s > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    const size_t need = sequence_workspace_bytes(A_dev->m, A_dev->n, A_dev->nnz, s, false);
    if (need == 0 || need > noalloc_scratch_bytes())
        return fail(BWR_EINVAL, "matrix too large for bwr_sequence_dev_noalloc: it needs " + std::to_string(need) +
                                    " bytes of device scratch, the library holds " +
                                    std::to_string(noalloc_scratch_bytes()));
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    void* base = nullptr;
    std::mutex* use = nullptr;
    if (!(e = noalloc_scratch(&base, &use)).ok()) return fail(e);
    std::lock_guard<std::mutex> lk(*use);  // calls on one device take turns with the array
    Arena ar;
    ar.base = (char*)base;
    ar.size = noalloc_scratch_bytes();
    {
        ArenaScope scope(&ar);
        e = sequence_dev_impl(view(A_dev), d_row, d_col, U, V, p, s, len, S_out, st);
    }
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "sequence");
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

// ---- symmetric projection ----

int bwr_sequence_sym_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* V,
                         uint32_t p, int32_t s, int64_t len, int32_t gram, uint32_t* S_out, void* stream) {
    if (!A_dev) return fail(BWR_EINVAL, "NULL matrix");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    if (len < 0) return fail(BWR_EINVAL, "len must be >= 0");
    if (len > 0 && (!S_out || (A_dev->n > 0 && !V))) return fail(BWR_EINVAL, "NULL output or block");
    if (len == 0) return BWR_OK;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    DeviceMatrix M;
    e = encode_matrix(view(A_dev), p, st, &M, true);
    if (e.ok()) {
        SequenceArgs a;
        a.M = &M;
        a.mp = ModP::make(p);
        a.s = s;
        a.d_row = d_row;
        a.d_col = d_col;
        a.U = V;
        a.V = V;
        a.len = len;
        a.S_out = S_out;
        a.symmetric = true;
        a.gram = gram != 0;
        e = run_sequence(a, st);
    }
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "sequence");
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_modp_sym_dev(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, int32_t gram, void* stream,
                          int64_t* rank_out, bwr_rank_info* info) {
    if (!A_dev || !rank_out) return fail(BWR_EINVAL, "NULL argument");
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    RankOut ro;
    e = rank_dev_impl(view(A_dev), p, block, seed, st, &ro, g_trials.load(), gram ? 2 : 1);
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "rank");
    if (!e.ok()) return fail(e);
    *rank_out = ro.rank;
    if (info) *info = ro.info;
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_modp_sym(const bwr_csr* A, uint32_t p, int32_t block, uint64_t seed, int32_t gram, int64_t* rank_out,
                      bwr_rank_info* info) {
    if (!A || !rank_out) return fail(BWR_EINVAL, "NULL argument");
    Error e;
    hipStream_t st = lib_stream(&e);
    if (!e.ok()) return fail(e);
    HostUpload up;
    if (!(e = upload(A, st, &up)).ok()) return fail(e);
    RankOut ro;
    e = rank_dev_impl(up.dev, p, block, seed, st, &ro, g_trials.load(), gram ? 2 : 1);
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "rank");
    if (!e.ok()) return fail(e);
    *rank_out = ro.rank;
    if (info) *info = ro.info;
    g_err.clear();
    return BWR_OK;
}

// ---- caller-owned workspace ----

int64_t bwr_device_allocations(void) { return device_allocations(); }

size_t bwr_sequence_workspace(int64_t m, int64_t n, int64_t nnz, int32_t s) {
    if (m < 0 || n < 0 || nnz < 0 || s < 1 || s > 64) return 0;
    return sequence_workspace_bytes(m, n, nnz, s, false);
}

size_t bwr_rank_workspace(int64_t m, int64_t n, int64_t nnz, int32_t block) {
    if (m < 0 || n < 0 || nnz < 0 || block < 1 || block > 64) return 0;
    const int64_t nb = std::min(m, n), outer = std::max(m, n);
    const int64_t s = std::max<int64_t>(1, std::min<int64_t>(block, nb));
    const int64_t total = 2 + (2 * nb + s - 1) / s + CHECK_TERMS;
    // a draw's U, V, D_r, D_c and its sequence, beside what the sequence itself needs
    const int64_t draws = 8 * nb * s + 4 * outer + 4 * nb + 4 * total * s * s + 8 * 256;
    return (size_t)draws + sequence_workspace_bytes(m, n, nnz, (int32_t)s, m < n);
}

int bwr_sequence_dev_ws(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                        const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* workspace,
                        size_t workspace_bytes, void* stream) {
    if (!A_dev) return fail(BWR_EINVAL, "NULL matrix");
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(BWR_EINVAL, "workspace must be 256-byte aligned");
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    Arena ar;
    ar.base = (char*)workspace;
    ar.size = workspace_bytes;
    {
        ArenaScope scope(&ar);
        e = sequence_dev_impl(view(A_dev), d_row, d_col, U, V, p, s, len, S_out, st);
    }
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "sequence");
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_modp_dev_ws(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, void* workspace,
                         size_t workspace_bytes, void* stream, int64_t* rank_out, bwr_rank_info* info) {
    if (!A_dev || !rank_out) return fail(BWR_EINVAL, "NULL argument");
    if (!workspace || ((uintptr_t)workspace & 255)) return fail(BWR_EINVAL, "workspace must be 256-byte aligned");
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    Arena ar;
    ar.base = (char*)workspace;
    ar.size = workspace_bytes;
    RankOut ro;
    {
        ArenaScope scope(&ar);
        e = rank_dev_impl(view(A_dev), p, block, seed, st, &ro, g_trials.load());
    }
    const hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "rank");
    if (!e.ok()) return fail(e);
    *rank_out = ro.rank;
    if (info) *info = ro.info;
    g_err.clear();
    return BWR_OK;
}

// ---- a matrix encoded once for several sequences ----

}  // extern "C"

struct bwr_matrix {
    DeviceMatrix M;
    int dev = 0;
    hipStream_t home = nullptr;  // where the matrix's buffers are released
};

extern "C" {

int bwr_matrix_create_dev(const bwr_csr* A_dev, uint32_t p, void* stream, bwr_matrix** out) {
    if (!A_dev || !out) return fail(BWR_EINVAL, "NULL argument");
    *out = nullptr;
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    auto h = std::make_unique<bwr_matrix>();
    hipError_t he = hipGetDevice(&h->dev);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&h->home, hipStreamNonBlocking);
    if (he != hipSuccess) return fail(Error::device(he, "bwr_matrix_create_dev"));
    e = encode_matrix(view(A_dev), p, st, &h->M, true);
    he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "encode");
    rehome(h->M, h->home);
    h->M.tiled = make_tiled_store(h->home);
    if (!e.ok()) {
        bwr_matrix_destroy(h.release());
        return fail(e);
    }
    *out = h.release();
    g_err.clear();
    return BWR_OK;
}

int bwr_matrix_sequence_dev(bwr_matrix* M, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                            const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream) {
    if (!M) return fail(BWR_EINVAL, "NULL matrix");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    if (len < 0) return fail(BWR_EINVAL, "len must be >= 0");
    if (len > 0 && (!S_out || (M->M.n > 0 && (!U || !V)))) return fail(BWR_EINVAL, "NULL output or block");
    if (!M->M.packed && M->M.wide_p != p) return fail(BWR_EINVAL, "matrix was encoded for another prime");
    if (len == 0) return BWR_OK;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    SequenceArgs a;
    a.M = &M->M;
    a.transpose = false;
    a.mp = ModP::make(p);
    a.s = s;
    a.d_row = d_row;
    a.d_col = d_col;
    a.U = U;
    a.V = V;
    a.len = len;
    a.S_out = S_out;
    e = run_sequence(a, st);
    hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "sequence");
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_matrix_sequence_sym_dev(bwr_matrix* M, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* V,
                                uint32_t p, int32_t s, int64_t len, int32_t gram, uint32_t* S_out, void* stream) {
    if (!M) return fail(BWR_EINVAL, "NULL matrix");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    if (len < 0) return fail(BWR_EINVAL, "len must be >= 0");
    if (len > 0 && (!S_out || (M->M.n > 0 && !V))) return fail(BWR_EINVAL, "NULL output or block");
    if (!M->M.packed && M->M.wide_p != p) return fail(BWR_EINVAL, "matrix was encoded for another prime");
    if (len == 0) return BWR_OK;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    SequenceArgs a;
    a.M = &M->M;
    a.mp = ModP::make(p);
    a.s = s;
    a.d_row = d_row;
    a.d_col = d_col;
    a.U = V;
    a.V = V;
    a.len = len;
    a.S_out = S_out;
    a.symmetric = true;
    a.gram = gram != 0;
    e = run_sequence(a, st);
    hipError_t he = hipStreamSynchronize(st);
    if (e.ok() && he != hipSuccess) e = Error::device(he, "sequence");
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

void bwr_matrix_destroy(bwr_matrix* M) {
    if (!M) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(M->dev);
    (void)hipDeviceSynchronize();  // no kernel of any stream still reads the matrix
    hipStream_t home = M->home;
    delete M;  // buffers released on home
    if (home) {
        (void)hipStreamSynchronize(home);
        (void)hipStreamDestroy(home);
    }
    (void)hipSetDevice(cur);
}

int bwr_rank_modp(const bwr_csr* A, uint32_t p, int32_t block, uint64_t seed, int64_t* rank_out,
                  bwr_rank_info* info) {
    if (!A || !rank_out) return fail(BWR_EINVAL, "NULL argument");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (block < 1 || block > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    if (!(e = check_host_csr(view(A))).ok()) return fail(e);
    if (A->nnz == 0 || A->m == 0 || A->n == 0) {
        *rank_out = 0;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            info->nb = std::min(A->m, A->n);
        }
        g_err.clear();
        return BWR_OK;
    }
    hipStream_t st = lib_stream(&e);
    if (!e.ok()) return fail(e);
    HostUpload up;
    if (!(e = upload(A, st, &up)).ok()) return fail(e);
    RankOut ro;
    if (!(e = rank_dev_impl(up.dev, p, block, seed, st, &ro, g_trials.load())).ok()) return fail(e);
    *rank_out = ro.rank;
    if (info) *info = ro.info;
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_modp_dev(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, void* stream,
                      int64_t* rank_out, bwr_rank_info* info) {
    if (!A_dev || !rank_out) return fail(BWR_EINVAL, "NULL argument");
    RankOut ro;
    Error e;
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    e = rank_dev_impl(view(A_dev), p, block, seed, st, &ro, g_trials.load());
    if (!e.ok()) return fail(e);
    *rank_out = ro.rank;
    if (info) *info = ro.info;
    g_err.clear();
    return BWR_OK;
}

int bwr_time_step_kernels_dev(const bwr_csr* A_dev, uint32_t p, int32_t s, int32_t transpose, int32_t iters,
                              void* stream, double* us_out, int32_t* plan_out) {
    if (!A_dev || !us_out) return fail(BWR_EINVAL, "NULL argument");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    DeviceMatrix M;
    if (!(e = encode_matrix(view(A_dev), p, st, &M, true)).ok()) return fail(e);
    StepPlan pl;
    if (!(e = time_step_kernels(M, transpose != 0, ModP::make(p), s, iters, st, us_out, &pl)).ok()) return fail(e);
    if (plan_out) {
        const int32_t v[16] = {pl.W,      pl.G1,      pl.G2,   pl.fused ? 1 : 0, pl.NB,      pl.esize,
                               pl.parts1, pl.parts2,  pl.t1.R, pl.t1.cb,         pl.t1.grid, pl.t2.R,
                               pl.t2.cb,  pl.t2.grid, pl.t1.un, pl.t2.un};
        std::memcpy(plan_out, v, sizeof(v));
    }
    g_err.clear();
    return BWR_OK;
}

int bwr_min_generator(const uint32_t* S, int64_t len, int32_t s, uint32_t p, int64_t* delta_out, uint32_t* P_out,
                      int64_t P_cap_terms, int64_t* max_deg_out) {
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64 || len < 0 || (len > 0 && !S) || !delta_out || !P_out || !max_deg_out)
        return fail(BWR_EINVAL, "bad arguments");
    Generator g;
    if (!(e = min_generator(S, len, s, p, &g)).ok()) return fail(e);
    int64_t maxd = 0;
    for (int64_t x : g.delta) maxd = std::max(maxd, x);
    if (maxd + 1 > P_cap_terms) return fail(BWR_EINVAL, "P_out capacity too small");
    std::memset(P_out, 0, sizeof(uint32_t) * (size_t)(maxd + 1) * s * s);
    for (int i = 0; i < s; ++i) {
        delta_out[i] = g.delta[i];
        for (int j = 0; j < s; ++j) {
            const uint32_t* src = g.P.at(i, j);
            for (int64_t k = 0; k < g.P.len && k <= maxd; ++k) P_out[((size_t)k * s + i) * s + j] = src[k];
        }
    }
    *max_deg_out = maxd;
    g_err.clear();
    return BWR_OK;
}

int bwr_sequence_batch(const bwr_csr* const* A, int32_t nmat, const uint32_t* primes, int32_t nprimes, int32_t s,
                       uint64_t seed, const int64_t* len, uint32_t* const* S_out) {
    if (nmat < 0 || nprimes < 1 || (nmat > 0 && (!A || !primes || !len || !S_out)))
        return fail(BWR_EINVAL, "bad arguments");
    Error e;
    for (int t = 0; t < nprimes; ++t)
        if (!(e = check_prime(primes[t])).ok()) return fail(e);
    for (int j = 0; j < nmat; ++j) {
        if (!A[j] || !S_out[j] || len[j] < 1) return fail(BWR_EINVAL, "bad matrix, output or length");
        if (!(e = check_host_csr(view(A[j]))).ok()) return fail(e);
    }
    hipStream_t st = lib_stream(&e);
    if (!e.ok()) return fail(e);
    std::vector<HostUpload> ups(nmat);
    std::vector<DeviceMatrix> Ms(nmat);
    std::vector<bool> tr(nmat);
    for (int j = 0; j < nmat; ++j) {
        if (!(e = upload(A[j], st, &ups[j])).ok()) return fail(e);
        if (!(e = encode_matrix(ups[j].dev, primes[0], st, &Ms[j], true)).ok()) return fail(e);
        if (!Ms[j].packed) return fail(BWR_EINVAL, "batched sequences need entries in [-127, 127] and sizes <= 2^24");
        tr[j] = A[j]->m < A[j]->n;
    }
    std::vector<Shape> shapes;
    for (int j = 0; j < nmat; ++j)
        shapes.push_back({tr[j] ? Ms[j].n : Ms[j].m, tr[j] ? Ms[j].m : Ms[j].n, Ms[j].nnz});
    BatchPlan bp = plan_batch(shapes, nprimes, s);
    if (!bp.W) return fail(BWR_EINVAL, "block size too large for batched sequences");
    bool all_small = true;
    for (int t = 0; t < nprimes; ++t) all_small = all_small && primes[t] <= 65536u;
    BatchRunner R(bp.W, bp.G1, bp.G2, st, all_small ? 2 : 4);
    std::vector<std::pair<int, int>> owner;  // job -> (matrix, first prime index)
    for (int j = 0; j < nmat; ++j)
        for (int t0 = 0; t0 < nprimes; t0 += bp.per_job) {
            BatchSpec sp;
            sp.M = &Ms[j];
            sp.transpose = tr[j];
            sp.primes.assign(primes + t0, primes + std::min(nprimes, t0 + bp.per_job));
            sp.s = s;
            sp.seed = seed;
            sp.len = len[j];
            int id = 0;
            if (!(e = R.add(sp, &id)).ok()) return fail(e);
            owner.emplace_back(j, t0);
        }
    std::vector<int> done;
    while (true) {
        size_t before = done.size();
        if (!(e = R.advance(INT64_MAX, &done)).ok()) return fail(e);
        if (R.active() == 0 && done.size() == before) break;
        if (R.active() == 0 && done.size() == owner.size()) break;
    }
    for (size_t id = 0; id < owner.size(); ++id) {
        const int j = owner[id].first, t0 = owner[id].second;
        const int np = (int)R.spec((int)id).primes.size();
        for (int t = 0; t < np; ++t) {
            const size_t n = (size_t)len[j] * s * s;
            hipError_t he = hipMemcpyAsync(S_out[j] + (size_t)(t0 + t) * n, R.sequence((int)id, t), 4 * n,
                                           hipMemcpyDeviceToHost, st);
            if (he != hipSuccess) return fail(Error::device(he, "download"));
        }
    }
    hipError_t he = hipStreamSynchronize(st);
    if (he != hipSuccess) return fail(Error::device(he, "batch"));
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_modp_batch(const bwr_csr* const* A, int32_t nmat, const uint32_t* primes, int32_t nprimes,
                        int32_t block, uint64_t seed, int64_t* ranks_out, bwr_batch_info* info) {
    if (nmat < 0 || nprimes < 1 || (nmat > 0 && (!A || !primes || !ranks_out)))
        return fail(BWR_EINVAL, "bad arguments");
    if (block < 1 || block > 64) return fail(BWR_EINVAL, "block size must be in 1..64");
    Error e;
    for (int t = 0; t < nprimes; ++t)
        if (!(e = check_prime(primes[t])).ok()) return fail(e);
    for (int j = 0; j < nmat; ++j) {
        if (!A[j]) return fail(BWR_EINVAL, "NULL matrix");
        if (!(e = check_host_csr(view(A[j]))).ok()) return fail(e);
    }
    const double t0 = now_s();
    const int32_t trials = g_trials.load();
    bwr_batch_info bi;
    std::memset(&bi, 0, sizeof(bi));
    hipStream_t st = lib_stream(&e);
    if (!e.ok()) return fail(e);
    std::vector<HostUpload> ups(nmat);
    std::vector<DeviceMatrix> Ms(nmat);
    std::vector<bool> tr(nmat), batched(nmat, false);
    std::vector<int64_t> ranks((size_t)nmat * nprimes, 0);
    for (int j = 0; j < nmat; ++j) {
        tr[j] = A[j]->m < A[j]->n;
        if (A[j]->nnz == 0 || A[j]->m == 0 || A[j]->n == 0) continue;
        if (!(e = upload(A[j], st, &ups[j])).ok()) return fail(e);
        if (!(e = encode_matrix(ups[j].dev, primes[0], st, &Ms[j], true)).ok()) return fail(e);
        batched[j] = Ms[j].packed;
    }
    bi.t_encode = now_s() - t0;
    // Matrices whose block of all primes side by side (outer x W residues of 4 bytes) would exceed
    // BATCH_BLOCK_BYTES run as single-matrix solves instead: their gathers would miss the L2 of every XCD,
    // while the single-matrix path keeps one prime per block (16-bit residues for 16-bit primes).  Those
    // solves, and the matrices the batch kernels cannot take (wide entries), run on host threads of their
    // own beside the batched launches.  Every rank is the same either way.
    // When the primes mix 16-bit and larger ones, the 16-bit primes are batched with their blocks in
    // 16-bit residues (one gathered row of 64 bytes serves three of them) and the larger primes run as
    // single-matrix solves; otherwise every prime is batched (16-bit residues if all are 16-bit).
    std::vector<int> bt_small, bt_large;
    for (int t = 0; t < nprimes; ++t) (primes[t] <= 65536u ? bt_small : bt_large).push_back(t);
    const bool split_classes = !bt_small.empty() && !bt_large.empty() && env_i64("BWR_BATCH_SPLIT", 1) != 0;
    std::vector<int> bt = split_classes ? bt_small : (bt_small.empty() ? bt_large : bt_small);
    std::vector<bool> batched_prime(nprimes, false);
    for (int t : bt) batched_prime[t] = true;
    const int besize = bt_large.empty() || split_classes ? 2 : 4;
    const int nbp = (int)bt.size();
    const int64_t block_bytes_max = env_i64("BWR_BATCH_BLOCK_BYTES", BATCH_BLOCK_BYTES);
    for (int j = 0; j < nmat; ++j) {
        if (!batched[j]) continue;
        const int64_t nb = std::min(A[j]->m, A[j]->n), outer = std::max(A[j]->m, A[j]->n);
        const int spad = ((int)std::min<int64_t>(block, nb) + 3) & ~3;
        const int per_job = std::max(1, std::min(nbp, 32 / std::max(spad, 1)));
        if (outer * (int64_t)per_job * spad * besize > block_bytes_max) batched[j] = false;
    }
    // With early termination on, a matrix whose single-matrix solve can stop early (a sequence of at least
    // 4096 terms, whose sigma-basis then runs beside it on the device) goes to the single-matrix lanes: the
    // batched sequences always run their full length.
    if (g_early.load() != 0)
        for (int j = 0; j < nmat; ++j) {
            if (!batched[j]) continue;
            const int64_t nb = std::min(A[j]->m, A[j]->n);
            const int32_t s = (int32_t)std::min<int64_t>(block, nb);
            if (gpu_leaf_order(s) > 0 && online_min_chunk(2 + (2 * nb + s - 1) / s) > 0) batched[j] = false;
        }
    std::vector<std::pair<int, int>> solo;  // (matrix, prime) pairs for the single-matrix path
    for (int j = 0; j < nmat; ++j) {
        if (A[j]->nnz == 0 || A[j]->m == 0 || A[j]->n == 0) continue;
        for (int t = 0; t < nprimes; ++t)
            if (!batched[j] || !batched_prime[t]) solo.emplace_back(j, t);
    }
    std::vector<std::thread> solo_threads;
    std::mutex solo_mu;
    std::atomic<size_t> solo_next{0};
    Error solo_err;
    if (!solo.empty()) {
        hipError_t he = hipStreamSynchronize(st);  // uploads and encodings are complete
        if (he != hipSuccess) return fail(Error::device(he, "upload"));
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        // with early termination the large matrices are solo and fill the GPU one at a time (16 of the batched
        // configuration's matrices x 4 primes: 2.07 solves/s with one lane against 1.86 with two)
        const int64_t dflt = g_early.load() != 0 ? 1 : BATCH_SOLO_THREADS;
        const int nthr = (int)std::min<int64_t>((int64_t)solo.size(),
                                                std::max<int64_t>(1, env_i64("BWR_BATCH_SOLO_THREADS", dflt)));
        for (int w = 0; w < nthr; ++w)
            solo_threads.emplace_back([&, dev] {
                (void)hipSetDevice(dev);
                Error le;
                hipStream_t wst = lib_stream(&le);
                for (size_t i; le.ok() && (i = solo_next.fetch_add(1)) < solo.size();) {
                    const int j = solo[i].first, t = solo[i].second;
                    RankOut ro;
                    le = rank_dev_impl(ups[j].dev, primes[t], block, seed, wst, &ro, trials);
                    if (!le.ok()) {
                        // nothing this thread queued may still read the uploads once the call returns
                        (void)hipStreamSynchronize(wst);
                        break;
                    }
                    std::lock_guard<std::mutex> lk(solo_mu);
                    ranks[(size_t)j * nprimes + t] = ro.rank;
                    bi.t_sequence += ro.info.t_sequence;
                    bi.t_sigma += ro.info.t_sigma;
                }
                if (!le.ok()) {
                    std::lock_guard<std::mutex> lk(solo_mu);
                    if (solo_err.ok()) solo_err = le;
                    solo_next.store(solo.size());  // the other threads stop too
                }
            });
    }
    // on every return path below: stop handing out single-matrix solves and join their threads
    struct Joiner {
        std::vector<std::thread>* th;
        std::atomic<size_t>* next;
        size_t n;
        ~Joiner() {
            next->store(n);
            for (auto& t : *th)
                if (t.joinable()) t.join();
        }
    } joiner{&solo_threads, &solo_next, solo.size()};
    std::vector<int> live_of;
    for (int j = 0; j < nmat; ++j)
        if (batched[j]) live_of.push_back(j);
    if (!live_of.empty()) {
        // plan with the largest block any batched matrix uses
        int smax = 1;
        std::vector<Shape> shapes;
        for (int j : live_of) {
            smax = std::max<int>(smax, (int)std::min<int64_t>(block, std::min(A[j]->m, A[j]->n)));
            shapes.push_back({tr[j] ? Ms[j].n : Ms[j].m, tr[j] ? Ms[j].m : Ms[j].n, Ms[j].nnz});
        }
        const BatchPlan bp = plan_batch(shapes, nbp, smax);
        if (!bp.W) return fail(BWR_EINVAL, "block size too large for batched ranks");
        bi.width = bp.W;
        bi.g1 = bp.G1;
        bi.g2 = bp.G2;
        BatchRunner R(bp.W, bp.G1, bp.G2, st, besize);
        struct Own {
            int j;
            int64_t L;
            int32_t s;
            int tix[BATCH_MAX_PRIMES];  // the job's primes as indices into primes[]
        };
        std::vector<Own> owner;
        for (int j : live_of) {
            const int64_t nb = std::min(A[j]->m, A[j]->n);
            const int32_t s = (int32_t)std::min<int64_t>(block, nb);
            const int64_t L = 2 + (2 * nb + s - 1) / s;
            // one job per group of primes and per draw (seeds seed, seed + 1, ...): the ranks of a matrix's draws
            // meet in their maximum below
            for (int32_t trial = 0; trial < trials; ++trial)
                for (int k0 = 0; k0 < nbp; k0 += bp.per_job) {
                    BatchSpec sp;
                    sp.M = &Ms[j];
                    sp.transpose = tr[j];
                    Own o{j, L, s, {0, 0, 0, 0}};
                    for (int k = k0; k < std::min(nbp, k0 + bp.per_job); ++k) {
                        o.tix[k - k0] = bt[k];
                        sp.primes.push_back(primes[bt[k]]);
                    }
                    sp.s = s;
                    sp.seed = seed + (uint64_t)trial;
                    sp.len = L + CHECK_TERMS;
                    int id = 0;
                    if (!(e = R.add(sp, &id)).ok()) return fail(e);
                    owner.push_back(o);
                    ++bi.jobs;
                }
        }
        const double t1 = now_s();
        double t_sig = 0;
        // read-outs of finished jobs run on a pool of host threads (one stream each), beside the sequences
        // of the jobs still running; a job's buffers are released once all its primes are read out
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        const size_t ntasks = owner.size() * (size_t)bp.per_job;
        ReadoutPool pool((int)std::min<size_t>(READOUT_THREADS, std::max<size_t>(1, ntasks)), dev);
        std::vector<int> left(owner.size(), 0);
        size_t finished = 0;
        Error first;
        while (finished < owner.size()) {
            if (R.active() > 0 && first.ok()) {
                std::vector<int> done;
                if (!(e = R.advance(INT64_MAX, &done)).ok()) {
                    first = e;
                    break;
                }
                for (int id : done) {
                    const Own& o = owner[id];
                    const BatchSpec& sp = R.spec(id);
                    left[id] = (int)sp.primes.size();
                    // the job's primes share L and s: one read-out (one batched sigma-basis) for its 16-bit
                    // primes and one for the larger ones; BWR_SIGMA_BATCH=0 reads each prime out alone
                    for (int cls = 0; cls < 2; ++cls) {
                        uint64_t tags[BATCH_MAX_PRIMES];
                        const uint32_t* seqs[BATCH_MAX_PRIMES];
                        uint32_t ps[BATCH_MAX_PRIMES];
                        int n = 0;
                        for (size_t t = 0; t < sp.primes.size(); ++t) {
                            if ((sp.primes[t] <= 65536u) != (cls == 0)) continue;
                            tags[n] = (uint64_t)id * BATCH_MAX_PRIMES + t;
                            seqs[n] = R.sequence(id, (int)t);
                            ps[n] = sp.primes[t];
                            ++n;
                        }
                        const char* sb = getenv("BWR_SIGMA_BATCH");
                        const int group = (sb && atoi(sb) == 0) ? 1 : BATCH_MAX_PRIMES;
                        for (int g0 = 0; g0 < n; g0 += group) {
                            hipEvent_t ev = nullptr;
                            hipError_t he = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
                            if (he == hipSuccess) he = hipEventRecord(ev, st);
                            if (he != hipSuccess) return fail(Error::device(he, "read-out event"));
                            pool.submit_group(tags + g0, seqs + g0, ps + g0, std::min(group, n - g0), o.L,
                                              R.length(id), o.s, ev);
                        }
                    }
                }
            } else if (pool.outstanding() == 0) {
                break;
            }
            for (const ReadoutPool::Result& r : pool.collect(R.active() == 0 || !first.ok())) {
                const int id = (int)(r.tag / BATCH_MAX_PRIMES), t = (int)(r.tag % BATCH_MAX_PRIMES);
                if (!r.err.ok() && first.ok()) first = r.err;
                int64_t& dst = ranks[(size_t)owner[id].j * nprimes + owner[id].tix[t]];
                dst = std::max(dst, r.rank);
                t_sig += r.seconds;
                if (--left[id] == 0) {
                    R.release(id);
                    ++finished;
                }
            }
        }
        if (!first.ok()) return fail(first);
        bi.steps = R.global_step();
        std::lock_guard<std::mutex> lk(solo_mu);
        bi.t_sigma += t_sig;
        bi.t_sequence += now_s() - t1;
    }
    for (auto& t : solo_threads) t.join();
    if (!solo_err.ok()) return fail(solo_err);
    // agreement retry: further draws for a prime whose rank is below the matrix's largest rank at the others
    // (each draw is at most the rank mod p, so the largest is kept)
    if (const int32_t retry = g_batch_retry.load(); retry > 0 && nprimes > 1) {
        for (int j = 0; j < nmat; ++j) {
            if (A[j]->nnz == 0 || A[j]->m == 0 || A[j]->n == 0) continue;
            int64_t best = 0;
            for (int t = 0; t < nprimes; ++t) best = std::max(best, ranks[(size_t)j * nprimes + t]);
            for (int t = 0; t < nprimes; ++t) {
                int64_t& r = ranks[(size_t)j * nprimes + t];
                for (int32_t k = 0; k < retry && r < best; ++k) {
                    RankOut ro;
                    if (!(e = rank_dev_impl(ups[j].dev, primes[t], block, seed + (uint64_t)(trials + k), st, &ro, 1))
                             .ok())
                        return fail(e);
                    r = std::max(r, ro.rank);
                    ++bi.retries;
                }
            }
        }
    }
    std::memcpy(ranks_out, ranks.data(), sizeof(int64_t) * ranks.size());
    bi.t_total = now_s() - t0;
    if (info) *info = bi;
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_integer(const bwr_csr* A, const uint32_t* primes, int32_t nprimes, int32_t block, uint64_t seed,
                     int64_t* rank_out, int64_t* ranks_out) {
    if (!A || !primes || nprimes < 1 || !rank_out) return fail(BWR_EINVAL, "bad arguments");
    std::vector<int64_t> r((size_t)nprimes, 0);
    const bwr_csr* one[1] = {A};
    const int rc = bwr_rank_modp_batch(one, 1, primes, nprimes, block, seed, r.data(), nullptr);
    if (rc != BWR_OK) return rc;
    *rank_out = *std::max_element(r.begin(), r.end());
    if (ranks_out) std::memcpy(ranks_out, r.data(), sizeof(int64_t) * r.size());
    g_err.clear();
    return BWR_OK;
}

int bwr_min_generator_dev(const uint32_t* S_dev, int64_t len, int32_t s, uint32_t p, void* stream,
                          int64_t* delta_out, uint32_t* P_out, int64_t P_cap_terms, int64_t* max_deg_out) {
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64 || len < 0 || (len > 0 && !S_dev) || !delta_out || !P_out || !max_deg_out)
        return fail(BWR_EINVAL, "bad arguments");
    if (gpu_leaf_order(s) == 0) return fail(BWR_EINVAL, "block size too large for the device sigma-basis");
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    Generator g;
    // the whole sequence is there, so the basis is one PM-Basis call unless BWR_SIGMA_MIN_CHUNK asks for
    // the chunked order of the online generator (same result)
    int64_t mc = 0;
    if (const char* v = getenv("BWR_SIGMA_MIN_CHUNK")) mc = std::max<int64_t>(0, atoll(v));
    if (!(e = gpu_min_generator(S_dev, len, s, p, st, &g, nullptr, mc)).ok()) return fail(e);
    int64_t maxd = 0;
    for (int64_t x : g.delta) maxd = std::max(maxd, x);
    if (maxd + 1 > P_cap_terms) return fail(BWR_EINVAL, "P_out capacity too small");
    std::memset(P_out, 0, sizeof(uint32_t) * (size_t)(maxd + 1) * s * s);
    for (int i = 0; i < s; ++i) {
        delta_out[i] = g.delta[i];
        for (int j = 0; j < s; ++j) {
            const uint32_t* src = g.P.at(i, j);
            for (int64_t k = 0; k < g.P.len && k <= maxd; ++k) P_out[((size_t)k * s + i) * s + j] = src[k];
        }
    }
    *max_deg_out = maxd;
    g_err.clear();
    return BWR_OK;
}

int bwr_min_generators_dev(const uint32_t* const* S_dev, int32_t n, int64_t len, int32_t s, const uint32_t* p,
                           void* stream, int64_t* delta_out, uint32_t* P_out, int64_t P_cap_terms,
                           int64_t* max_deg_out) {
    if (n < 1 || n > SIGMA_BATCH_MAX || !S_dev || !p) return fail(BWR_EINVAL, "bad arguments");
    Error e;
    for (int b = 0; b < n; ++b)
        if (!(e = check_prime(p[b])).ok()) return fail(e);
    if (s < 1 || s > 64 || len < 0 || !delta_out || !P_out || !max_deg_out) return fail(BWR_EINVAL, "bad arguments");
    for (int b = 0; b < n; ++b)
        if (len > 0 && !S_dev[b]) return fail(BWR_EINVAL, "bad arguments");
    if (gpu_leaf_order(s) == 0) return fail(BWR_EINVAL, "block size too large for the device sigma-basis");
    hipStream_t st = work_stream(stream, &e);
    if (!e.ok()) return fail(e);
    std::vector<Generator> g(n);
    if (!(e = gpu_min_generators(S_dev, n, len, s, p, st, g.data())).ok()) return fail(e);
    for (int b = 0; b < n; ++b) {
        int64_t maxd = 0;
        for (int64_t x : g[b].delta) maxd = std::max(maxd, x);
        if (maxd + 1 > P_cap_terms) return fail(BWR_EINVAL, "P_out capacity too small");
    }
    for (int b = 0; b < n; ++b) {
        int64_t maxd = 0;
        for (int64_t x : g[b].delta) maxd = std::max(maxd, x);
        uint32_t* Pb = P_out + (size_t)b * P_cap_terms * s * s;
        std::memset(Pb, 0, sizeof(uint32_t) * (size_t)(maxd + 1) * s * s);
        for (int i = 0; i < s; ++i) {
            delta_out[(size_t)b * s + i] = g[b].delta[i];
            for (int j = 0; j < s; ++j) {
                const uint32_t* src = g[b].P.at(i, j);
                for (int64_t k = 0; k < g[b].P.len && k <= maxd; ++k) Pb[((size_t)k * s + i) * s + j] = src[k];
            }
        }
        max_deg_out[b] = maxd;
    }
    g_err.clear();
    return BWR_OK;
}

int bwr_rank_from_sequence(const uint32_t* S, int64_t len, int64_t check, int32_t s, uint32_t p, int64_t* rank_out) {
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (s < 1 || s > 64 || len < 0 || check < 0 || (len + check > 0 && !S) || !rank_out)
        return fail(BWR_EINVAL, "bad arguments");
    Generator g;
    if (!(e = min_generator(S, len, s, p, &g)).ok()) return fail(e);
    if (!(e = check_generator(g, S, len, len + check, p)).ok()) return fail(e);
    int64_t r = 0;
    if (!(e = rank_from_generator(g, p, &r)).ok()) return fail(e);
    *rank_out = r;
    g_err.clear();
    return BWR_OK;
}

int bwr_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t block, bwr_server** out) {
    if (!out || max_slots < 1 || block < 1 || block > 32 || hbm_budget_bytes == 0)
        return fail(BWR_EINVAL, "bad arguments");
    auto srv = std::make_unique<bwr_server>();
    srv->impl = std::make_unique<Server>((int64_t)std::min<uint64_t>(hbm_budget_bytes, (uint64_t)INT64_MAX), max_slots,
                                         block);
    Error e = srv->impl->start();
    if (!e.ok()) return fail(e);
    *out = srv.release();
    g_err.clear();
    return BWR_OK;
}

int bwr_server_submit(bwr_server* srv, const bwr_csr* A, uint32_t p, uint64_t seed, uint64_t* ticket) {
    if (!srv || !A || !ticket) return fail(BWR_EINVAL, "NULL argument");
    Error e = check_prime(p);
    if (!e.ok()) return fail(e);
    if (!(e = check_host_csr(view(A))).ok()) return fail(e);
    if (!(e = srv->impl->submit(view(A), p, seed, g_trials.load(), ticket)).ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_server_poll(bwr_server* srv, uint64_t ticket, int32_t* done, int64_t* rank) {
    if (!srv || !done || !rank) return fail(BWR_EINVAL, "NULL argument");
    bool d = false;
    Error e = srv->impl->poll(ticket, &d, rank);
    *done = d ? 1 : 0;
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_server_wait(bwr_server* srv, uint64_t ticket, int64_t* rank) {
    if (!srv || !rank) return fail(BWR_EINVAL, "NULL argument");
    Error e = srv->impl->wait(ticket, rank);
    if (!e.ok()) return fail(e);
    g_err.clear();
    return BWR_OK;
}

int bwr_server_get_stats(bwr_server* srv, bwr_server_stats* out) {
    if (!srv || !out) return fail(BWR_EINVAL, "NULL argument");
    ServerStats st = srv->impl->stats();
    out->p50_ms = st.p50_ms;
    out->p99_ms = st.p99_ms;
    out->solves_per_s = st.solves_per_s;
    out->busy_s = st.busy_s;
    out->completed = st.completed;
    out->max_queue = st.max_queue;
    out->max_active = st.max_active;
    out->steps = st.steps;
    out->peak_bytes = st.peak_bytes;
    g_err.clear();
    return BWR_OK;
}

void bwr_server_destroy(bwr_server* srv) { delete srv; }

}  // extern "C"
