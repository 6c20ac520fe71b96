// Host driver of batched sequences (batch.hip): jobs join at step
// boundaries, every step advances all active jobs with one launch per product,
// and a job leaves when its terms are complete.  Used by the batched rank
// entry point and by the server (continuous batching).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <vector>

#include "batch.h"
#include "engine.h"

namespace bwr {

struct BatchSpec {
    const DeviceMatrix* M = nullptr;  // must outlive the job
    bool transpose = false;           // B on the rows of A (m < n)
    std::vector<uint32_t> primes;     // 1 .. BATCH_MAX_PRIMES
    int32_t s = 8;
    uint64_t seed = 1;
    int64_t len = 0;  // terms per prime
};

class BatchRunner {
   public:
    // W: block width of every job (nprimes * round4(s) <= W); G1, G2: row split of the two products.
    // esize: bytes per stored residue, 2 only if every job's primes are <= 2^16 (add() refuses others)
    BatchRunner(int W, int G1, int G2, hipStream_t st, int esize = 4);
    ~BatchRunner();
    static int width_for(int nprimes, int s);

    // Prepares the job's blocks from its seed exactly as the single-matrix rank
    // does (same U, V, D_r, D_c per prime) and computes S_0; the job makes its
    // first application of B at the next step.
    Error add(const BatchSpec& spec, int* id);
    // Advances all active jobs by up to max_steps steps, stopping early when a
    // job completes; ids of completed jobs are appended to `done`.
    Error advance(int64_t max_steps, std::vector<int>* done);
    int active() const;
    int64_t global_step() const { return g_; }
    // Device sequence of (job, prime index): len x s x s, valid once the job is done.
    const uint32_t* sequence(int id, int t) const;
    int64_t length(int id) const;
    const BatchSpec& spec(int id) const;
    // Frees the job's device memory (stream-ordered, after the work already queued on the runner's stream).
    // A job released before it is done leaves the batch: it is marked done and the next advance rebuilds
    // the active set and the step graph without it.
    void release(int id);
    int64_t bytes_in_use() const;
    static int64_t footprint(const DeviceMatrix& M, bool transpose, int W, int nprimes, int s, int64_t len);

   private:
    struct Job;
    Error rebuild();
    int W_, G1_, G2_;
    hipStream_t st_;
    int esize_ = 4;
    std::vector<std::unique_ptr<Job>> jobs_;
    std::vector<int> active_;
    int64_t g_ = 0;
    bool dirty_ = true;
    DevBuf djobs_, dstart1_, dstart2_, part_;
    int nblocks1_ = 0, nblocks2_ = 0, max_entries_ = 0;
    int acc1_ = 0, acc2_ = 0;  // accumulator modes of the active set (batch_acc_mode)
    int64_t slot_words_ = 0;
    int64_t chunk_ = 64;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    int64_t bytes_ = 0;
};

}  // namespace bwr
