// Read-out of finished sequences and the pool that runs read-outs concurrently.
#include "readout.h"

#include <chrono>
#include <cstdlib>

#include "sigma.h"
#include "sigma_gpu.h"

namespace bwr {

namespace {

#define BWR_TRY(expr)              \
    do {                           \
        Error er_ = (expr);        \
        if (!er_.ok()) return er_; \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

Error rank_of_sequence_dev(const uint32_t* S_dev, int64_t L, int64_t total, int32_t s, uint32_t p, hipStream_t st,
                           int64_t* rank, double* t_sigma) {
    const double t0 = now_s();
    Generator g;
    Error e;
    std::vector<uint32_t> Sh((size_t)(total * s * s));
    if (gpu_leaf_order(s) > 0 && !getenv("BWR_HOST_SIGMA")) {
        if (!(e = gpu_min_generator(S_dev, L, s, p, st, &g)).ok()) return e;
        hipError_t he = hipMemcpyAsync(Sh.data(), S_dev, 4 * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
    } else {
        hipError_t he = hipMemcpyAsync(Sh.data(), S_dev, 4 * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
        if (!(e = min_generator(Sh.data(), L, s, p, &g)).ok()) return e;
    }
    *t_sigma += now_s() - t0;
    if (!(e = check_generator(g, Sh.data(), L, total, p)).ok()) return e;
    return rank_from_generator(g, p, rank);
}

Error rank_of_sequences_dev(const uint32_t* const* S_dev, int n, int64_t L, int64_t total, int32_t s,
                            const uint32_t* p, hipStream_t st, int64_t* ranks, double* t_sigma) {
    if (n < 1 || n > SIGMA_BATCH_MAX) return Error::inval("read-out batch must hold 1 to 4 sequences");
    bool same_class = true;
    for (int b = 1; b < n; ++b) same_class = same_class && ((p[b] <= 65536u) == (p[0] <= 65536u));
    if (n == 1 || !same_class || gpu_leaf_order(s) == 0 || getenv("BWR_HOST_SIGMA")) {
        for (int b = 0; b < n; ++b) BWR_TRY(rank_of_sequence_dev(S_dev[b], L, total, s, p[b], st, &ranks[b], t_sigma));
        return {};
    }
    const double t0 = now_s();
    std::vector<Generator> g(n);
    BWR_TRY(gpu_min_generators(S_dev, n, L, s, p, st, g.data()));
    *t_sigma += now_s() - t0;
    std::vector<uint32_t> Sh((size_t)(total * s * s));
    for (int b = 0; b < n; ++b) {
        hipError_t he = hipMemcpyAsync(Sh.data(), S_dev[b], 4 * Sh.size(), hipMemcpyDeviceToHost, st);
        if (he == hipSuccess) he = hipStreamSynchronize(st);
        if (he != hipSuccess) return Error::device(he, "sequence download");
        BWR_TRY(check_generator(g[b], Sh.data(), L, total, p[b]));
        BWR_TRY(rank_from_generator(g[b], p[b], &ranks[b]));
    }
    return {};
}

ReadoutPool::ReadoutPool(int threads, int device) : device_(device) {
    if (const char* v = getenv("BWR_READOUT_THREADS")) threads = std::max(1, atoi(v));
    relay_init_ = hipStreamCreateWithFlags(&relay_, hipStreamNonBlocking);
    if (relay_init_ != hipSuccess) relay_ = nullptr;
    for (int i = 0; i < std::max(1, threads); ++i) workers_.emplace_back([this] { work(); });
}

ReadoutPool::~ReadoutPool() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        quit_ = true;
    }
    cv_.notify_all();
    for (auto& w : workers_) w.join();
    for (Task& t : queue_)
        if (t.ready) (void)hipEventDestroy(t.ready);
    if (relay_) (void)hipStreamDestroy(relay_);
}

void ReadoutPool::submit_group(const uint64_t* tags, const uint32_t* const* S_dev, const uint32_t* p, int n,
                               int64_t L, int64_t total, int32_t s, hipEvent_t ready) {
    Task t{};
    t.n = std::max(1, std::min(n, 4));
    for (int b = 0; b < t.n; ++b) {
        t.tag[b] = tags[b];
        t.S[b] = S_dev[b];
        t.p[b] = p[b];
    }
    t.L = L;
    t.total = total;
    t.s = s;
    t.ready = ready;
    t.relay_err = relay_init_;
    if (ready && t.relay_err == hipSuccess) {
        t.relay_err = hipStreamWaitEvent(relay_, ready, 0);
        if (t.relay_err == hipSuccess) t.relay_err = hipEventRecord(ready, relay_);
    }
    {
        std::lock_guard<std::mutex> lk(mu_);
        queue_.push_back(t);
        outstanding_ += (size_t)t.n;
    }
    cv_.notify_one();
}

std::vector<ReadoutPool::Result> ReadoutPool::collect(bool wait) {
    std::unique_lock<std::mutex> lk(mu_);
    if (wait) done_cv_.wait(lk, [&] { return !results_.empty() || outstanding_ == 0; });
    std::vector<Result> out;
    out.swap(results_);
    return out;
}

size_t ReadoutPool::outstanding() {
    std::lock_guard<std::mutex> lk(mu_);
    return outstanding_;
}

void ReadoutPool::work() {
    (void)hipSetDevice(device_);
    hipStream_t st = nullptr;
    hipError_t se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (;;) {
        Task t;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [&] { return quit_ || !queue_.empty(); });
            if (quit_ && queue_.empty()) break;
            t = queue_.front();
            queue_.pop_front();
        }
        int64_t ranks[4] = {0, 0, 0, 0};
        double seconds = 0;
        Error err;
        if (se != hipSuccess) {
            err = Error::device(se, "read-out stream");
        } else {
            // wait on the host for the event as re-recorded on the relay stream (never capturing); the
            // producer's own stream may be capturing its next graph by now
            hipError_t he = t.relay_err;
            if (he != hipSuccess) err = Error::device(he, "read-out relay");
            else if (t.ready && (he = hipEventSynchronize(t.ready)) != hipSuccess)
                err = Error::device(he, "hipEventSynchronize");
            if (err.ok()) err = rank_of_sequences_dev(t.S, t.n, t.L, t.total, t.s, t.p, st, ranks, &seconds);
            // the stream has been synchronized by the read-out (or nothing was queued after the wait)
            if (!err.ok()) (void)hipStreamSynchronize(st);
        }
        if (t.ready) (void)hipEventDestroy(t.ready);
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (int b = 0; b < t.n; ++b) {
                Result r;
                r.tag = t.tag[b];
                r.rank = ranks[b];
                r.seconds = b == 0 ? seconds : 0.0;  // the group's time, counted once
                r.err = err;
                results_.push_back(r);
            }
            outstanding_ -= (size_t)t.n;
        }
        done_cv_.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace bwr
