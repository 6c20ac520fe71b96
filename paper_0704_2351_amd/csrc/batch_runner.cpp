// Batched sequence driver: jobs (matrix x up to four primes) advance together,
// one launch per product per step over all active jobs (batch.hip).  The
// active set only changes at chunk boundaries: a chunk never runs past the
// step at which a job completes, and new jobs join between chunks.  Full
// chunks starting on an even step replay one captured HIP graph per active set.
#include "batch_runner.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "kernels.h"
#include "splitmix.h"

namespace bwr {

#define BWR_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return Error::device(e_, #call); \
    } while (0)

#define BWR_TRY(expr)              \
    do {                           \
        Error er_ = (expr);        \
        if (!er_.ok()) return er_; \
    } while (0)

struct BatchRunner::Job {
    BatchSpec spec;
    BatchJob d{};
    DevBuf X0, X1, Y, Ut, dr, dc2, S;
    int64_t nb = 0, outer = 0, bytes = 0;
    bool done = false, released = false;
};

namespace {

int round4(int s) { return (s + 3) & ~3; }

constexpr double SECOND_BLOCKS = 2048;
// BWR_BATCH_ACC=0 forces the int64 accumulators (tests use it to cover both kernels)
int env_acc(int mode) {
    const char* v = getenv("BWR_BATCH_ACC");
    return (v && atoi(v) == 0) ? 0 : mode;
}

double second_blocks() {
    static const double v = getenv("BWR_BATCH_BLOCKS") ? std::max(1, atoi(getenv("BWR_BATCH_BLOCKS"))) : SECOND_BLOCKS;
    return v;
}

}  // namespace

int BatchRunner::width_for(int nprimes, int s) {
    int need = nprimes * round4(s);
    int w = 4;
    while (w < need) w <<= 1;
    return w;
}

BatchRunner::BatchRunner(int W, int G1, int G2, hipStream_t st, int esize)
    : W_(W), G1_(G1), G2_(G2), st_(st), esize_(esize == 2 ? 2 : 4) {
    const char* c = getenv("BWR_BATCH_CHUNK");
    if (c && atoi(c) >= 2) chunk_ = atoi(c) & ~1;
}

BatchRunner::~BatchRunner() {
    // no launch of the graph may still be in flight when it is destroyed
    if (exec_ || graph_) (void)hipStreamSynchronize(st_);
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
}

int BatchRunner::active() const {
    int a = 0;
    for (auto& j : jobs_)
        if (!j->done) ++a;
    return a;
}

const uint32_t* BatchRunner::sequence(int id, int t) const {
    const Job& J = *jobs_[id];
    return J.S.as<uint32_t>() + (size_t)t * J.d.len * J.d.s * J.d.s;
}

int64_t BatchRunner::length(int id) const { return jobs_[id]->d.len; }
const BatchSpec& BatchRunner::spec(int id) const { return jobs_[id]->spec; }
int64_t BatchRunner::bytes_in_use() const { return bytes_; }

int64_t BatchRunner::footprint(const DeviceMatrix& M, bool transpose, int W, int nprimes, int s, int64_t len) {
    const int64_t nb = transpose ? M.m : M.n, outer = transpose ? M.n : M.m;
    return 4 * (3 * nb * W + outer * W + (int64_t)nprimes * (outer + nb) + (int64_t)nprimes * len * s * s) + 4096;
}

void BatchRunner::release(int id) {
    Job& J = *jobs_[id];
    if (J.released) return;
    if (!J.done) {
        // a job released before its last step (an error path) leaves the batch: the next advance rebuilds the
        // active set and its graph without it, so no launch reads the buffers freed below
        J.done = true;
        dirty_ = true;
    }
    J.X0.release();
    J.X1.release();
    J.Y.release();
    J.Ut.release();
    J.dr.release();
    J.dc2.release();
    J.S.release();
    bytes_ -= J.bytes;
    J.released = true;
}

Error BatchRunner::add(const BatchSpec& sp, int* id) {
    const DeviceMatrix& M = *sp.M;
    const int np = (int)sp.primes.size();
    if (!M.packed) return Error::inval("batched sequences need the packed encoding");
    if (np < 1 || np > BATCH_MAX_PRIMES) return Error::inval("a batch job takes 1 to 4 primes");
    if (sp.s < 1 || np * round4(sp.s) > W_) return Error::inval("job wider than the batch block");
    if (sp.len < 1) return Error::inval("a job needs at least one term");
    if (esize_ == 2)
        for (uint32_t p : sp.primes)
            if (p > 65536u) return Error::inval("16-bit batch storage needs primes <= 2^16");
    auto J = std::make_unique<Job>();
    J->spec = sp;
    const bool tr = sp.transpose;
    J->nb = tr ? M.m : M.n;
    J->outer = tr ? M.n : M.m;
    const int64_t nb = J->nb, outer = J->outer;
    const int spad = round4(sp.s);
    const size_t es = (size_t)esize_;
    BWR_TRY(J->X0.alloc(es * (size_t)std::max<int64_t>(nb * W_, 1), st_));
    BWR_TRY(J->X1.alloc(es * (size_t)std::max<int64_t>(nb * W_, 1), st_));
    BWR_TRY(J->Ut.alloc(es * (size_t)std::max<int64_t>(nb * W_, 1), st_));
    BWR_TRY(J->Y.alloc(es * (size_t)std::max<int64_t>(outer * W_, 1), st_));
    BWR_TRY(J->dr.alloc(4 * (size_t)std::max<int64_t>(np * outer, 1), st_));
    BWR_TRY(J->dc2.alloc(4 * (size_t)std::max<int64_t>(np * nb, 1), st_));
    BWR_TRY(J->S.alloc(4 * (size_t)np * sp.len * sp.s * sp.s, st_));
    J->bytes = footprint(M, tr, W_, np, sp.s, sp.len);
    BWR_HIP(hipMemsetAsync(J->X0.as<void>(), 0, J->X0.bytes(), st_));
    BWR_HIP(hipMemsetAsync(J->X1.as<void>(), 0, J->X1.bytes(), st_));
    BWR_HIP(hipMemsetAsync(J->Ut.as<void>(), 0, J->Ut.bytes(), st_));
    BWR_HIP(hipMemsetAsync(J->Y.as<void>(), 0, J->Y.bytes(), st_));
    DevBuf tu, tv, tdc, flag;
    BWR_TRY(tu.alloc(4 * (size_t)std::max<int64_t>(nb * sp.s, 1), st_));
    BWR_TRY(tv.alloc(4 * (size_t)std::max<int64_t>(nb * sp.s, 1), st_));
    BWR_TRY(tdc.alloc(4 * (size_t)std::max<int64_t>(nb, 1), st_));
    BWR_TRY(flag.alloc(4, st_));
    BatchJob& d = J->d;
    // the same draws as the single-matrix rank, prime by prime; a length-sorted encoding gets them in its
    // relabelled order (gathered from the draws in the input order), which leaves every S_k unchanged
    DevBuf gtmp;
    const int32_t* pn = nullptr;  // iterated side
    const int32_t* po = nullptr;  // other side
    if (M.sorted) {
        pn = (tr ? M.perm_r : M.perm_c).as<int32_t>();
        po = (tr ? M.perm_c : M.perm_r).as<int32_t>();
        BWR_TRY(gtmp.alloc(4 * (size_t)std::max<int64_t>(std::max(nb * sp.s, outer), 1), st_));
    }
    auto draw = [&](uint64_t stream, int64_t rows, int width, int diag, const ModP& mp, const int32_t* perm,
                    uint32_t* out) -> Error {
        if (!perm) {
            BWR_HIP(launch_rng_block(sp.seed, stream, rows, width, width, mp, diag, out, st_));
            return {};
        }
        BWR_HIP(launch_rng_block(sp.seed, stream, rows, width, width, mp, diag, gtmp.as<uint32_t>(), st_));
        BWR_HIP(launch_gather_rows(rows, width, perm, gtmp.as<uint32_t>(), out, st_));
        return {};
    };
    for (int t = 0; t < np; ++t) {
        const uint32_t p = sp.primes[t];
        const ModP mp = ModP::make(p);
        d.mp[t] = mp;
        BWR_TRY(draw(STREAM_V, nb, sp.s, 0, mp, pn, tv.as<uint32_t>()));
        BWR_TRY(draw(STREAM_U, nb, sp.s, 0, mp, pn, tu.as<uint32_t>()));
        BWR_TRY(draw(STREAM_DROW, outer, 1, 1, mp, po, J->dr.as<uint32_t>() + (size_t)t * outer));
        BWR_TRY(draw(STREAM_DCOL, nb, 1, 1, mp, pn, tdc.as<uint32_t>()));
        BWR_HIP(launch_place_block(nb, sp.s, W_, t * spad, tv.as<uint32_t>(), tdc.as<uint32_t>(), 1, mp,
                                   J->X0.as<void>(), esize_, st_));
        BWR_HIP(launch_place_block(nb, sp.s, W_, t * spad, tu.as<uint32_t>(), tdc.as<uint32_t>(), 2, mp,
                                   J->Ut.as<void>(), esize_, st_));
        BWR_HIP(launch_square_diag(nb, tdc.as<uint32_t>(), mp, J->dc2.as<uint32_t>() + (size_t)t * nb,
                                   flag.as<int32_t>(), st_));
    }
    for (int t = np; t < BATCH_MAX_PRIMES; ++t) d.mp[t] = d.mp[0];
    Operand op1, op2;
    {
        Operand a{M.m, M.max_len_a, M.rp_a.as<int32_t>(), M.ent_a.as<uint32_t>(), nullptr};
        Operand tt{M.n, M.max_len_t, M.rp_t.as<int32_t>(), M.ent_t.as<uint32_t>(), nullptr};
        op1 = tr ? tt : a;
        op2 = tr ? a : tt;
    }
    d.rows1 = op1.rows;
    d.rows2 = op2.rows;
    d.rp1 = op1.rp;
    d.ent1 = op1.ent;
    d.rp2 = op2.rp;
    d.ent2 = op2.ent;
    d.X[0] = J->X0.as<uint32_t>();
    d.X[1] = J->X1.as<uint32_t>();
    d.Y = J->Y.as<uint32_t>();
    d.Ut = J->Ut.as<uint32_t>();
    d.dr = J->dr.as<uint32_t>();
    d.dc2 = J->dc2.as<uint32_t>();
    d.S = J->S.as<uint32_t>();
    d.nprimes = np;
    d.spad = spad;
    d.s = sp.s;
    d.len = sp.len;
    d.g0 = g_;
    d.par = (int32_t)(g_ & 1);
    d.nblk2 = 1;  // persistent blocks of the second product: set for the active set in rebuild()
    // S_0
    const int nblk0 = (int)std::max<int64_t>(1, std::min<int64_t>(64, (nb + 255) / 256));
    DevBuf p0;
    BWR_TRY(p0.alloc(4 * (size_t)nblk0 * np * spad * spad, st_));
    BWR_HIP(launch_batch_s0(W_, esize_, d, p0.as<uint32_t>(), nblk0, st_));
    if (sp.len == 1) J->done = true;
    bytes_ += J->bytes;
    *id = (int)jobs_.size();
    jobs_.push_back(std::move(J));
    dirty_ = true;
    return {};
}

Error BatchRunner::rebuild() {
    active_.clear();
    for (size_t i = 0; i < jobs_.size(); ++i)
        if (!jobs_[i]->done) active_.push_back((int)i);
    std::vector<BatchJob> descs;
    std::vector<int32_t> s1(1, 0), s2(1, 0);
    int64_t off = 0;
    max_entries_ = 0;
    const int rpb1 = batch_rows_per_block(W_, G1_);
    const int rpb2 = batch_rows_per_block(W_, G2_);
    // the second product's persistent blocks (each writes one partial per prime and step) are shared out in
    // proportion to the jobs' rows, about SECOND_BLOCKS in all: enough waves to fill the device
    double rows_all = 0;
    for (int id : active_) rows_all += (double)jobs_[id]->d.rows2;
    for (int id : active_) {
        BatchJob& dj = jobs_[id]->d;
        const int64_t tiles2 = std::max<int64_t>(1, (dj.rows2 + rpb2 - 1) / rpb2);
        const int64_t want = (int64_t)(second_blocks() * (double)dj.rows2 / std::max(rows_all, 1.0) + 0.5);
        dj.nblk2 = (int32_t)std::max<int64_t>(1, std::min<int64_t>(tiles2, want));
    }
    for (int id : active_) {
        BatchJob d = jobs_[id]->d;
        d.part_off = off;
        off += (int64_t)d.nblk2 * d.nprimes * d.spad * d.spad;
        descs.push_back(d);
        const int64_t tiles1 = std::max<int64_t>(1, (d.rows1 + rpb1 - 1) / rpb1);
        s1.push_back(s1.back() + (int32_t)tiles1);
        s2.push_back(s2.back() + d.nblk2);
        max_entries_ = std::max(max_entries_, d.nprimes * d.s * d.s);
    }
    slot_words_ = std::max<int64_t>(off, 1);
    nblocks1_ = s1.back();
    nblocks2_ = s2.back();
    // accumulators: split 32-bit sums when every active job's rows allow them
    int64_t len1 = 0, len2 = 0;
    int32_t vabs = 1;
    for (int id : active_) {
        const Job& J = *jobs_[id];
        const DeviceMatrix& M = *J.spec.M;
        len1 = std::max<int64_t>(len1, J.spec.transpose ? M.max_len_t : M.max_len_a);
        len2 = std::max<int64_t>(len2, J.spec.transpose ? M.max_len_a : M.max_len_t);
        vabs = std::max(vabs, M.max_abs);
    }
    acc1_ = env_acc(batch_acc_mode(len1, vabs, G1_));
    acc2_ = env_acc(batch_acc_mode(len2, vabs, G2_));
    // the previous active set's graph is destroyed only after its launches have run (a launch in flight, and a
    // tracer that inspects its dispatches when they complete, must not outlive the executable graph)
    if (exec_ || graph_) BWR_HIP(hipStreamSynchronize(st_));
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    exec_ = nullptr;
    graph_ = nullptr;
    if (!descs.empty()) {
        BWR_TRY(djobs_.alloc(sizeof(BatchJob) * descs.size(), st_));
        BWR_TRY(dstart1_.alloc(sizeof(int32_t) * s1.size(), st_));
        BWR_TRY(dstart2_.alloc(sizeof(int32_t) * s2.size(), st_));
        BWR_HIP(hipMemcpyAsync(djobs_.as<void>(), descs.data(), sizeof(BatchJob) * descs.size(), hipMemcpyHostToDevice,
                               st_));
        BWR_HIP(hipMemcpyAsync(dstart1_.as<void>(), s1.data(), sizeof(int32_t) * s1.size(), hipMemcpyHostToDevice, st_));
        BWR_HIP(hipMemcpyAsync(dstart2_.as<void>(), s2.data(), sizeof(int32_t) * s2.size(), hipMemcpyHostToDevice, st_));
        const size_t need = 4 * (size_t)slot_words_ * (size_t)chunk_;
        if (part_.bytes() < need) BWR_TRY(part_.alloc(need, st_));
        // the host arrays above must outlive their (possibly staged) copies
        BWR_HIP(hipStreamSynchronize(st_));
    }
    dirty_ = false;
    return {};
}

Error BatchRunner::advance(int64_t max_steps, std::vector<int>* done) {
    for (size_t i = 0; i < jobs_.size(); ++i) {
        Job& J = *jobs_[i];
        if (!J.done && J.d.len <= 1) {
            J.done = true;
            dirty_ = true;
            done->push_back((int)i);
        }
    }
    if (dirty_) BWR_TRY(rebuild());
    if (active_.empty() || max_steps <= 0) return {};
    const int nact = (int)active_.size();
    const char* ng = getenv("BWR_NO_GRAPH");
    const bool graphs = !(ng && atoi(ng) != 0);
    while (max_steps > 0) {
        int64_t rem = INT64_MAX;
        for (int id : active_) {
            const BatchJob& d = jobs_[id]->d;
            rem = std::min(rem, d.g0 + d.len - 1 - g_);
        }
        if (rem <= 0) break;
        const int64_t cnt = std::min({chunk_, max_steps, rem});
        const BatchJob* dj = djobs_.as<BatchJob>();
        const int32_t* st1 = dstart1_.as<int32_t>();
        const int32_t* st2 = dstart2_.as<int32_t>();
        uint32_t* part = part_.as<uint32_t>();
        auto launch_chunk = [&](int64_t steps, int64_t g_start) -> Error {
            for (int64_t i = 0; i < steps; ++i) {
                const int par = (int)((g_start + i) & 1);
                BWR_HIP(launch_batch_first(W_, G1_, acc1_, esize_, dj, st1, nact, nblocks1_, par, st_));
                BWR_HIP(launch_batch_second(W_, G2_, acc2_, esize_, dj, st2, nact, nblocks2_, par, part,
                                            i * slot_words_, st_));
            }
            return {};
        };
        if (graphs && cnt == chunk_ && (g_ & 1) == 0) {
            if (!exec_) {
                BWR_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
                Error e = launch_chunk(chunk_, 0);
                hipError_t he = hipStreamEndCapture(st_, &graph_);
                if (!e.ok()) return e;
                if (he != hipSuccess) return Error::device(he, "hipStreamEndCapture");
                BWR_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
            }
            BWR_HIP(hipGraphLaunch(exec_, st_));
        } else {
            BWR_TRY(launch_chunk(cnt, g_));
        }
        BWR_HIP(launch_batch_reduce(dj, nact, g_, (int)cnt, part, slot_words_, max_entries_, st_));
        g_ += cnt;
        max_steps -= cnt;
        bool any = false;
        for (int id : active_) {
            Job& J = *jobs_[id];
            if (J.d.g0 + J.d.len - 1 - g_ <= 0) {
                J.done = true;
                done->push_back(id);
                any = true;
            }
        }
        if (any) {
            dirty_ = true;
            break;
        }
    }
    return {};
}

}  // namespace bwr
