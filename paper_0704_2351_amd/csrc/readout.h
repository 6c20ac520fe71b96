// Read-out of finished sequences: sigma-basis, check on the extra terms and
// rank (Section 2.4 and steps 3-4 of the rank algorithm in Section 2.5).  A
// pool of host threads, each on its own device stream, runs read-outs
// concurrently with each other and with sequences still being computed.
// Internal C++.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "engine.h"

namespace bwr {

// Generator of S_dev[0 .. L) (device sigma-basis when its leaf fits in LDS, else host), checked on the
// terms L .. total - 1, and the rank it reads out.  Runs on st; adds its seconds to *t_sigma.
Error rank_of_sequence_dev(const uint32_t* S_dev, int64_t L, int64_t total, int32_t s, uint32_t p, hipStream_t st,
                           int64_t* rank, double* t_sigma);
// Same for n <= 4 sequences of one length and block size, one prime each: on the device the generators
// come from one batched sigma-basis when the primes are all <= 2^16 or all larger.
Error rank_of_sequences_dev(const uint32_t* const* S_dev, int n, int64_t L, int64_t total, int32_t s,
                            const uint32_t* p, hipStream_t st, int64_t* ranks, double* t_sigma);

// Host threads of a read-out pool: with the stream of the running batch this fills the four hardware
// queues a process gets by default; more concurrent sigma-bases only slow each other down.
constexpr int READOUT_THREADS = 3;

class ReadoutPool {
   public:
    struct Result {
        uint64_t tag = 0;
        int64_t rank = 0;
        double seconds = 0;
        Error err;
    };
    // threads >= 1; device = the HIP device the workers use
    ReadoutPool(int threads, int device);
    ~ReadoutPool();
    // Waits (on the worker's host thread) for `ready` before reading S_dev; the event is owned by the pool
    // afterwards.  S_dev must stay allocated until the task's result has been collected.  Called on the
    // producer's thread while no capture is open on the stream `ready` was recorded on: the event is
    // re-recorded on the pool's relay stream, which never captures, so that a worker's wait cannot meet a
    // capture the producer begins later on its own stream (HIP refuses a host wait on an event whose
    // stream is capturing, and invalidates that capture).
    void submit(uint64_t tag, const uint32_t* S_dev, int64_t L, int64_t total, int32_t s, uint32_t p,
                hipEvent_t ready) {
        submit_group(&tag, &S_dev, &p, 1, L, total, s, ready);
    }
    // n <= 4 sequences of one length and block size read out together (rank_of_sequences_dev); one
    // result per tag.
    void submit_group(const uint64_t* tags, const uint32_t* const* S_dev, const uint32_t* p, int n, int64_t L,
                      int64_t total, int32_t s, hipEvent_t ready);
    // Finished tasks; with wait = true blocks until at least one is available (if any is outstanding).
    std::vector<Result> collect(bool wait);
    size_t outstanding();

   private:
    struct Task {
        int n;
        uint64_t tag[4];
        const uint32_t* S[4];
        uint32_t p[4];
        int64_t L, total;
        int32_t s;
        hipEvent_t ready;
        hipError_t relay_err;  // failure to hand `ready` over to the relay stream
    };
    void work();
    int device_;
    hipStream_t relay_ = nullptr;
    hipError_t relay_init_ = hipSuccess;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Task> queue_;
    std::vector<Result> results_;
    size_t outstanding_ = 0;
    bool quit_ = false;
    std::vector<std::thread> workers_;
};

}  // namespace bwr
