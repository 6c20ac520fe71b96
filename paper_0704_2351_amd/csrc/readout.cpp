// Read-out of finished sequences and the pool that runs read-outs concurrently.
#include "readout.h"

#include <chrono>
#include <cstdlib>

#include "sigma.h"
#include "sigma_gpu.h"

namespace bwr {

namespace {

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

ReadoutPool::ReadoutPool(int threads, int device) : device_(device) {
    if (const char* v = getenv("BWR_READOUT_THREADS")) threads = std::max(1, atoi(v));
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
}

void ReadoutPool::submit(uint64_t tag, const uint32_t* S_dev, int64_t L, int64_t total, int32_t s, uint32_t p,
                         hipEvent_t ready) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        queue_.push_back(Task{tag, S_dev, L, total, s, p, ready});
        ++outstanding_;
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
        Result r;
        r.tag = t.tag;
        if (se != hipSuccess) {
            r.err = Error::device(se, "read-out stream");
        } else {
            hipError_t he = t.ready ? hipStreamWaitEvent(st, t.ready, 0) : hipSuccess;
            if (he != hipSuccess) r.err = Error::device(he, "hipStreamWaitEvent");
            else r.err = rank_of_sequence_dev(t.S, t.L, t.total, t.s, t.p, st, &r.rank, &r.seconds);
            // the stream has been synchronized by the read-out (or nothing was queued after the wait)
            if (!r.err.ok()) (void)hipStreamSynchronize(st);
        }
        if (t.ready) (void)hipEventDestroy(t.ready);
        {
            std::lock_guard<std::mutex> lk(mu_);
            results_.push_back(r);
            --outstanding_;
        }
        done_cv_.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace bwr
