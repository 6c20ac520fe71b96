// Continuous-batching rank server (server.cpp).  Internal C++; the public
// surface is bwr_server_* in bwrank.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "batch_runner.h"
#include "engine.h"

namespace bwr {

// The single-matrix rank of a device CSR with `trials` independent draws (defined with the C-ABI).
Error rank_single(const CsrView& A_dev, uint32_t p, int32_t block, uint64_t seed, int32_t trials, hipStream_t st,
                  int64_t* rank);

struct ServerStats {
    double p50_ms, p99_ms;  // latency = answer time - submit time
    double solves_per_s;    // completed / (last answer - first submit)
    double busy_s;          // worker time spent advancing and answering
    int64_t completed, max_queue, max_active, steps;
    int64_t peak_bytes;     // largest sum of admitted requests' device bytes (encoded matrices included)
};

class Server {
   public:
    Server(int64_t hbm_budget, int max_slots, int32_t block);
    ~Server();
    Error start();
    void stop();
    // Copies A into host memory and queues it (trials independent draws, the largest rank kept); the worker
    // uploads and encodes it when it is admitted.
    Error submit(const CsrView& A_host, uint32_t p, uint64_t seed, int32_t trials, uint64_t* ticket);
    Error poll(uint64_t ticket, bool* done, int64_t* rank);
    Error wait(uint64_t ticket, int64_t* rank);
    ServerStats stats();

   private:
    struct Req;
    void loop();
    void solo_loop();
    Error encode(Req& R);
    void answer_locked(Req& R, int code, const std::string& msg, int64_t rank);
    int64_t budget_;
    int max_slots_;
    int32_t block_;
    int device_ = 0;
    int W_ = 0, G1_ = 0, G2_ = 0;
    hipStream_t upload_ = nullptr;
    // batches of requests at primes <= 2^16 (16-bit residues) and at larger primes (32-bit residues), each
    // on a stream of its own so that the two batches' steps run side by side
    hipStream_t compute_[2] = {nullptr, nullptr};
    std::unique_ptr<BatchRunner> runners_[2];
    // advances a batch may have on the device (0: no bound): before queueing an advance the worker waits
    // for the event recorded after the advance queued ahead_ advances before, so that requests admitted
    // now start after at most ahead_ advances already queued
    static constexpr int MAX_AHEAD = 8;
    int ahead_ = 1;
    hipEvent_t ahead_ev_[2][MAX_AHEAD] = {};
    bool ahead_rec_[2][MAX_AHEAD] = {};
    int ahead_pos_[2] = {0, 0};
    std::thread worker_;
    // requests of at least solo_nnz_ non-zeros (BWR_SERVER_SOLO_NNZ, 0: none) run one at a time through the
    // single-matrix path (autotuned, tiled products) on a thread of their own, beside the batches: the batched
    // kernels lose to the tuned single-matrix ones once a job's block outgrows an XCD's L2
    int64_t solo_nnz_ = 0;
    std::thread solo_;
    std::deque<std::shared_ptr<Req>> solo_q_;
    std::condition_variable solo_cv_;
    std::mutex mu_, upload_mu_;
    std::condition_variable cv_, done_cv_;
    std::map<uint64_t, std::shared_ptr<Req>> reqs_;
    std::deque<uint64_t> queue_;
    uint64_t next_ticket_ = 0;
    bool quit_ = false;
    std::vector<double> latencies_;
    int64_t completed_ = 0, max_queue_ = 0, max_active_ = 0, steps_ = 0;
    // device bytes of the admitted requests (footprints, plus the transient of one being encoded)
    int64_t held_ = 0, peak_held_ = 0;
    // error handling test hook: BWR_SERVER_FAIL_ADVANCE=k makes the advance after k advances report an error
    // instead of launching (once); the requests in the batch are then answered with that error
    int64_t advances_ = 0, fail_after_ = -1;
    double first_arrival_ = 0, last_finish_ = 0, busy_s_ = 0;
};

}  // namespace bwr
