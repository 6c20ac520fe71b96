// Rank server: requests (matrix, prime, seed) arrive at any time; a worker
// thread keeps two batches of sequences running on the device (requests at
// 16-bit primes in 16-bit residues, the others in 32-bit residues, each batch
// on a stream of its own) and admits queued requests at step boundaries
// whenever the HBM budget and the slot count allow (continuous batching).  A
// request whose sequence is complete gets its sigma-basis and read-out, frees
// its memory and is answered.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/bwrank.h"
#include "batch_runner.h"
#include "readout.h"
#include "server.h"
#include "sigma.h"
#include "sigma_gpu.h"

namespace bwr {

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int64_t CHECK_TERMS = 4;

#define BWR_TRY_S(expr)               \
    do {                              \
        Error er_ = (expr);           \
        if (!er_.ok()) return er_;    \
    } while (0)

}  // namespace

struct Server::Req {
    uint64_t ticket = 0;
    // host copy of the CSR until the request is admitted and encoded (queued requests hold no device memory)
    int64_t m = 0, n = 0, nnz = 0;
    std::vector<int64_t> hrp;
    std::vector<int32_t> hcol, hval;
    DeviceMatrix M;
    bool encoded = false;
    bool transpose = false;
    uint32_t p = 0;
    uint64_t seed = 0;
    int32_t trials = 1, draws = 0;  // independent draws asked for and made (draw t uses seed + t)
    int32_t s = 0;
    int64_t nb = 0, L = 0;
    int64_t footprint = 0;  // device bytes while admitted: encoded matrix + the runner's blocks and sequence
    int64_t transient = 0;  // extra device bytes while it is being uploaded and encoded
    bool counted = false;   // footprint counted in held_
    double arrival = 0, admitted = 0, finished = 0;
    bool solo = false;  // runs through the single-matrix path (solo lane)
    int cls = 1;  // runner: 0 for primes <= 2^16, 1 otherwise
    int job = -1;
    bool done = false;
    int64_t rank = 0;
    int code = 0;
    std::string msg;
};

Server::Server(int64_t budget, int max_slots, int32_t block) : budget_(budget), max_slots_(max_slots), block_(block) {}

Server::~Server() { stop(); }

Error Server::start() {
    hipError_t e = hipGetDevice(&device_);
    for (int c = 0; c < 2 && e == hipSuccess; ++c) e = hipStreamCreateWithFlags(&compute_[c], hipStreamNonBlocking);
    if (const char* a = getenv("BWR_SERVER_AHEAD")) ahead_ = std::max(0, std::min(MAX_AHEAD, atoi(a)));
    if (const char* f = getenv("BWR_SERVER_FAIL_ADVANCE")) fail_after_ = atoi(f);
    for (int c = 0; c < 2 && e == hipSuccess; ++c)
        for (int i = 0; i < ahead_ && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&ahead_ev_[c][i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&upload_, hipStreamNonBlocking);
    if (e != hipSuccess) return Error::device(e, "server streams");
    const int spad = (block_ + 3) & ~3;
    W_ = BatchRunner::width_for(1, block_);
    if (spad > 32 || !batch_supported(W_, std::max(1, W_ / 4), true)) return Error::inval("block size unsupported by the server");
    // matrices of the paper's kind have ~10-20 entries per row
    G1_ = std::max(1, std::min(4, 64 / (W_ / 4)));
    G2_ = std::max(W_ / 4, std::min(4, 64 / (W_ / 4)));
    if (!batch_supported(W_, G1_, false)) G1_ = 1;
    if (!batch_supported(W_, G2_, true)) G2_ = W_ / 4;
    runners_[0] = std::make_unique<BatchRunner>(W_, G1_, G2_, compute_[0], 2);
    runners_[1] = std::make_unique<BatchRunner>(W_, G1_, G2_, compute_[1], 4);
    solo_nnz_ = 1 << 20;
    if (const char* v = getenv("BWR_SERVER_SOLO_NNZ")) solo_nnz_ = std::max<int64_t>(0, atoll(v));
    worker_ = std::thread([this] { loop(); });
    if (solo_nnz_ > 0) solo_ = std::thread([this] { solo_loop(); });
    return {};
}

void Server::stop() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        quit_ = true;
    }
    cv_.notify_all();
    done_cv_.notify_all();
    solo_cv_.notify_all();
    if (worker_.joinable()) worker_.join();
    if (solo_.joinable()) solo_.join();
    solo_q_.clear();
    runners_[0].reset();
    runners_[1].reset();
    reqs_.clear();
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < MAX_AHEAD; ++i) {
            if (ahead_ev_[c][i]) (void)hipEventDestroy(ahead_ev_[c][i]);
            ahead_ev_[c][i] = nullptr;
            ahead_rec_[c][i] = false;
        }
    for (hipStream_t& c : compute_) {
        if (c) (void)hipStreamDestroy(c);
        c = nullptr;
    }
    if (upload_) (void)hipStreamDestroy(upload_);
    upload_ = nullptr;
}

Error Server::submit(const CsrView& A, uint32_t p, uint64_t seed, int32_t trials, uint64_t* ticket) {
    auto R = std::make_shared<Req>();
    R->arrival = now_s();
    R->p = p;
    R->seed = seed;
    R->trials = std::max(1, trials);
    R->transpose = A.m < A.n;
    R->m = A.m;
    R->n = A.n;
    R->nnz = A.nnz;
    const int64_t nb = std::min(A.m, A.n);
    R->nb = nb;
    // the batch kernels take the packed encoding: entries in [-127, 127], dimensions up to 2^24
    bool packed = A.m <= (1LL << 24) && A.n <= (1LL << 24);
    for (int64_t t = 0; packed && t < A.nnz; ++t) packed = A.val[t] >= -127 && A.val[t] <= 127;
    if (nb == 0 || A.nnz == 0 || !packed) {
        // nothing to iterate, or entries the batch kernels cannot take: answer at once
        R->done = true;
        R->finished = now_s();
        if (nb > 0 && A.nnz > 0) {
            R->code = BWR_EINVAL;
            R->msg = "server requests need entries in [-127, 127] and sizes <= 2^24";
        }
    } else {
        R->s = (int32_t)std::min<int64_t>(block_, nb);
        R->L = 2 + (2 * nb + R->s - 1) / R->s;
        DeviceMatrix shape;
        shape.m = A.m;
        shape.n = A.n;
        shape.nnz = A.nnz;
        // encoded CSR of A and A^T with their relabellings, and the runner's blocks and sequence
        R->footprint = BatchRunner::footprint(shape, R->transpose, W_, 1, R->s, R->L + CHECK_TERMS) +
                       8 * (A.m + A.n + 2) + 8 * A.nnz;
        // the uploaded CSR (int64 row pointers, int32 columns and values) and the relabelled copy the encoder
        // builds from it, with its counters
        R->transient = 2 * (8 * (A.m + 1) + 8 * A.nnz) + 16 * std::max(A.m, A.n) + 4096;
        if (solo_nnz_ > 0 && A.nnz >= solo_nnz_) {
            // the single-matrix path's device memory: encoded CSR of A and A^T with their relabellings, the
            // tiled encodings its autotuner builds (at most six geometries per product) and keeps, the blocks,
            // the sequence and the sigma-basis (about 2 (2s)^2 L words)
            R->solo = true;
            R->footprint = 64 * A.nnz + 64 * (A.m + A.n + 2) + 16 * std::max(A.m, A.n) * R->s +
                           8LL * (4 * R->s * R->s) * (R->L + CHECK_TERMS);
            R->transient = 2 * (8 * (A.m + 1) + 8 * A.nnz);
        }
        if (R->footprint + R->transient > budget_) return Error{ENOMEM_, "request larger than the server's HBM budget"};
        R->hrp.assign(A.row_ptr, A.row_ptr + A.m + 1);
        R->hcol.assign(A.col_idx, A.col_idx + A.nnz);
        R->hval.assign(A.val, A.val + A.nnz);
    }
    std::lock_guard<std::mutex> lk(mu_);
    R->ticket = ++next_ticket_;
    *ticket = R->ticket;
    reqs_[R->ticket] = R;
    if (R->done) {
        latencies_.push_back(R->finished - R->arrival);
        ++completed_;
        done_cv_.notify_all();
    } else if (R->solo) {
        solo_q_.push_back(R);
        solo_cv_.notify_all();
    } else {
        queue_.push_back(R->ticket);
        max_queue_ = std::max<int64_t>(max_queue_, (int64_t)queue_.size());
    }
    if (first_arrival_ == 0) first_arrival_ = R->arrival;
    cv_.notify_all();
    return {};
}

// Uploads and encodes an admitted request's matrix on the worker thread (upload stream), then drops the host
// copy.
Error Server::encode(Req& R) {
    DevBuf rp, col, val;
    const size_t nnz = (size_t)R.nnz;
    BWR_TRY_S(rp.alloc(sizeof(int64_t) * (size_t)(R.m + 1), upload_));
    BWR_TRY_S(col.alloc(4 * std::max<size_t>(nnz, 1), upload_));
    BWR_TRY_S(val.alloc(4 * std::max<size_t>(nnz, 1), upload_));
    hipError_t he = hipMemcpyAsync(rp.as<void>(), R.hrp.data(), 8 * R.hrp.size(), hipMemcpyHostToDevice, upload_);
    if (he == hipSuccess && nnz) he = hipMemcpyAsync(col.as<void>(), R.hcol.data(), 4 * nnz, hipMemcpyHostToDevice, upload_);
    if (he == hipSuccess && nnz) he = hipMemcpyAsync(val.as<void>(), R.hval.data(), 4 * nnz, hipMemcpyHostToDevice, upload_);
    if (he != hipSuccess) {
        (void)hipStreamSynchronize(upload_);
        return Error::device(he, "server upload");
    }
    const CsrView dv{R.m, R.n, R.nnz, rp.as<int64_t>(), col.as<int32_t>(), val.as<int32_t>()};
    Error e = encode_matrix(dv, R.p, upload_, &R.M, true);
    he = hipStreamSynchronize(upload_);  // the host copies and the uploaded CSR are no longer read
    if (e.ok() && he != hipSuccess) e = Error::device(he, "server upload");
    if (!e.ok()) return e;
    R.hrp = std::vector<int64_t>();
    R.hcol = std::vector<int32_t>();
    R.hval = std::vector<int32_t>();
    R.encoded = true;
    return {};
}

Error Server::poll(uint64_t ticket, bool* done, int64_t* rank) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return Error::inval("unknown ticket");
    *done = it->second->done;
    if (*done) {
        if (it->second->code) return Error{it->second->code, it->second->msg};
        *rank = it->second->rank;
    }
    return {};
}

Error Server::wait(uint64_t ticket, int64_t* rank) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return Error::inval("unknown ticket");
    std::shared_ptr<Req> R = it->second;
    done_cv_.wait(lk, [&] { return R->done || quit_; });
    if (!R->done) return Error::inval("server stopped");
    if (R->code) return Error{R->code, R->msg};
    *rank = R->rank;
    return {};
}

ServerStats Server::stats() {
    std::lock_guard<std::mutex> lk(mu_);
    ServerStats st{};
    std::vector<double> l = latencies_;
    std::sort(l.begin(), l.end());
    auto q = [&](double f) { return l.empty() ? 0.0 : l[std::min(l.size() - 1, (size_t)(f * (double)l.size()))]; };
    st.p50_ms = 1000.0 * q(0.50);
    st.p99_ms = 1000.0 * q(0.99);
    st.completed = completed_;
    st.max_queue = max_queue_;
    st.max_active = max_active_;
    st.steps = steps_;
    const double span = last_finish_ - first_arrival_;
    st.solves_per_s = (span > 0 && completed_ > 0) ? (double)completed_ / span : 0.0;
    st.busy_s = busy_s_;
    st.peak_bytes = peak_held_;
    return st;
}

// Answers R (under mu_): its memory leaves the budget, its latency is recorded.
void Server::answer_locked(Req& R, int code, const std::string& msg, int64_t rank) {
    R.done = true;
    R.code = code;
    R.msg = msg;
    R.rank = rank;
    R.finished = now_s();
    latencies_.push_back(R.finished - R.arrival);
    ++completed_;
    last_finish_ = R.finished;
    if (R.counted) held_ -= R.footprint;
    R.counted = false;
    R.M = DeviceMatrix();
    done_cv_.notify_all();
    solo_cv_.notify_all();  // memory left the budget
}

// The solo lane: one large request at a time, admitted against the same budget as the batches, uploaded on
// the lane's stream and ranked by the single-matrix path (trials draws, the largest rank kept).
void Server::solo_loop() {
    (void)hipSetDevice(device_);
    hipStream_t st = nullptr;
    const hipError_t se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (;;) {
        std::shared_ptr<Req> R;
        {
            std::unique_lock<std::mutex> lk(mu_);
            solo_cv_.wait(lk, [&] {
                if (quit_) return true;
                if (solo_q_.empty()) return false;
                const Req& F = *solo_q_.front();
                return held_ == 0 || held_ + F.footprint + F.transient <= budget_;
            });
            if (quit_) break;
            R = solo_q_.front();
            solo_q_.pop_front();
            held_ += R->footprint + R->transient;
            peak_held_ = std::max(peak_held_, held_);
            R->counted = true;
            R->admitted = now_s();
        }
        Error e;
        int64_t rank = 0;
        if (se != hipSuccess) {
            e = Error::device(se, "server solo stream");
        } else {
            DevBuf rp, col, val;
            const size_t nnz = (size_t)R->nnz;
            e = rp.alloc(sizeof(int64_t) * (size_t)(R->m + 1), st);
            if (e.ok()) e = col.alloc(4 * std::max<size_t>(nnz, 1), st);
            if (e.ok()) e = val.alloc(4 * std::max<size_t>(nnz, 1), st);
            hipError_t he = hipSuccess;
            if (e.ok()) he = hipMemcpyAsync(rp.as<void>(), R->hrp.data(), 8 * R->hrp.size(), hipMemcpyHostToDevice, st);
            if (e.ok() && he == hipSuccess && nnz)
                he = hipMemcpyAsync(col.as<void>(), R->hcol.data(), 4 * nnz, hipMemcpyHostToDevice, st);
            if (e.ok() && he == hipSuccess && nnz)
                he = hipMemcpyAsync(val.as<void>(), R->hval.data(), 4 * nnz, hipMemcpyHostToDevice, st);
            if (e.ok() && he != hipSuccess) e = Error::device(he, "server upload");
            if (e.ok()) {
                const CsrView dv{R->m, R->n, R->nnz, rp.as<int64_t>(), col.as<int32_t>(), val.as<int32_t>()};
                e = rank_single(dv, R->p, block_, R->seed, R->trials, st, &rank);
            }
            (void)hipStreamSynchronize(st);  // the uploads and everything reading them are done
        }
        std::lock_guard<std::mutex> lk(mu_);
        R->hrp = std::vector<int64_t>();
        R->hcol = std::vector<int32_t>();
        R->hval = std::vector<int32_t>();
        held_ -= R->transient;  // the upload; answer_locked releases the footprint
        answer_locked(*R, e.ok() ? 0 : e.code, e.msg, e.ok() ? rank : 0);
    }
    if (se == hipSuccess) (void)hipStreamDestroy(st);
}

void Server::loop() {
    (void)hipSetDevice(device_);
    // sigma-bases and read-outs of finished sequences run on a pool of host threads (one stream each),
    // beside the batch that keeps advancing
    ReadoutPool pool(READOUT_THREADS, device_);
    std::vector<std::shared_ptr<Req>> active;       // sequences in the batch
    std::map<uint64_t, std::shared_ptr<Req>> reading;  // (runner << 32 | job id) -> request being read out
    for (;;) {
        // admission at a step boundary: a request enters while the device bytes of every admitted request
        // (encoded matrix, blocks, sequence), its own included, stay within the budget
        {
            std::unique_lock<std::mutex> lk(mu_);
            if (active.empty() && reading.empty()) cv_.wait(lk, [&] { return quit_ || !queue_.empty(); });
            if (quit_) break;
            while (!queue_.empty() && (int)(active.size() + reading.size()) < max_slots_) {
                std::shared_ptr<Req> R = reqs_[queue_.front()];
                if (!R->counted) {
                    const int64_t need = R->footprint + R->transient;
                    if (held_ + need > budget_ && held_ > 0) break;
                    held_ += need;
                    peak_held_ = std::max(peak_held_, held_);
                    R->counted = true;
                }
                queue_.pop_front();
                lk.unlock();
                Error e;
                if (!R->encoded) {
                    e = encode(*R);
                    std::lock_guard<std::mutex> lk2(mu_);
                    held_ -= R->transient;  // the upload and the encoder's temporaries are released
                }
                if (e.ok()) {
                    BatchSpec sp;
                    sp.M = &R->M;
                    sp.transpose = R->transpose;
                    sp.primes = {R->p};
                    sp.s = R->s;
                    sp.seed = R->seed + (uint64_t)R->draws;
                    sp.len = R->L + CHECK_TERMS;
                    R->cls = R->p <= 65536u ? 0 : 1;
                    e = runners_[R->cls]->add(sp, &R->job);
                }
                lk.lock();
                if (R->draws == 0) R->admitted = now_s();
                if (!e.ok()) {
                    answer_locked(*R, e.code, e.msg, 0);
                    continue;
                }
                active.push_back(R);
            }
            max_active_ = std::max<int64_t>(max_active_, (int64_t)(active.size() + reading.size()));
        }
        const double t0 = now_s();
        Error e;
        for (int cls = 0; cls < 2 && e.ok(); ++cls) {
            if (std::none_of(active.begin(), active.end(), [&](const std::shared_ptr<Req>& r) { return r->cls == cls; }))
                continue;
            BatchRunner& run = *runners_[cls];
            std::vector<int> fin;
            // wait until the advance queued ahead_ advances ago has run (no capture is open on this thread)
            const int slot = ahead_pos_[cls];
            if (ahead_ > 0 && ahead_rec_[cls][slot]) {
                const hipError_t he = hipEventSynchronize(ahead_ev_[cls][slot]);
                if (he != hipSuccess) e = Error::device(he, "server advance wait");
            }
            if (e.ok() && fail_after_ >= 0 && advances_ >= fail_after_) {
                e = Error{EDEVICE_, "advance failed (BWR_SERVER_FAIL_ADVANCE)"};
                fail_after_ = -1;  // once
            }
            ++advances_;
            if (e.ok()) e = run.advance(64, &fin);
            if (e.ok() && ahead_ > 0) {
                const hipError_t he = hipEventRecord(ahead_ev_[cls][slot], compute_[cls]);
                if (he != hipSuccess) e = Error::device(he, "server advance event");
                ahead_rec_[cls][slot] = he == hipSuccess;
                ahead_pos_[cls] = (slot + 1) % ahead_;
            }
            steps_ = runners_[0]->global_step() + runners_[1]->global_step();
            for (int id : fin) {
                auto it = std::find_if(active.begin(), active.end(),
                                       [&](const std::shared_ptr<Req>& r) { return r->cls == cls && r->job == id; });
                if (it == active.end()) continue;
                std::shared_ptr<Req> R = *it;
                active.erase(it);
                hipEvent_t ev = nullptr;
                hipError_t he = e.ok() ? hipEventCreateWithFlags(&ev, hipEventDisableTiming) : hipSuccess;
                if (e.ok() && he == hipSuccess) he = hipEventRecord(ev, compute_[cls]);
                if (!e.ok() || he != hipSuccess) {
                    if (ev) (void)hipEventDestroy(ev);
                    (void)hipStreamSynchronize(compute_[cls]);
                    const Error er = e.ok() ? Error::device(he, "read-out event") : e;
                    run.release(id);
                    std::lock_guard<std::mutex> lk(mu_);
                    answer_locked(*R, er.code, er.msg, 0);
                    continue;
                }
                const uint64_t tag = ((uint64_t)cls << 32) | (uint32_t)id;
                reading[tag] = R;
                pool.submit(tag, run.sequence(id, 0), R->L, run.length(id), R->s, R->p, ev);
            }
        }
        if (!e.ok()) {
            // a failed advance: every request still in a batch is answered with the error and its job released
            for (hipStream_t c : compute_) (void)hipStreamSynchronize(c);
            for (auto& R : active) runners_[R->cls]->release(R->job);
            std::lock_guard<std::mutex> lk(mu_);
            for (auto& R : active) answer_locked(*R, e.code, e.msg, 0);
            active.clear();
        }
        // answer the requests whose read-out finished (wait for one when nothing else is running); a request
        // with draws left whose best rank is below min(m, n) goes back to the front of the queue with its
        // matrix kept
        for (const ReadoutPool::Result& r : pool.collect(active.empty() && !reading.empty())) {
            auto it = reading.find(r.tag);
            if (it == reading.end()) continue;
            std::shared_ptr<Req> R = it->second;
            reading.erase(it);
            runners_[r.tag >> 32]->release((int)(r.tag & 0xffffffffu));
            std::lock_guard<std::mutex> lk(mu_);
            if (!r.err.ok()) {
                answer_locked(*R, r.err.code, r.err.msg, 0);
                continue;
            }
            R->rank = R->draws == 0 ? r.rank : std::max(R->rank, r.rank);
            ++R->draws;
            if (R->draws < R->trials && R->rank < R->nb && !quit_) {
                queue_.push_front(R->ticket);
                cv_.notify_all();
                continue;
            }
            answer_locked(*R, 0, std::string(), R->rank);
        }
        busy_s_ += now_s() - t0;
    }
}

}  // namespace bwr
