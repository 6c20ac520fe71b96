// Device sigma-basis: launchers (sigma_gpu.hip) and the PM-Basis driver (sigma_gpu.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "early_cut.h"
#include "engine.h"
#include "modp.h"
#include "sigma.h"

namespace bwr {

// A batch of sigma-bases computed together: one target prime per batch element (same order and block size,
// so the PM-Basis recursion has the same shape for all).  The primes are all <= 2^16 or all larger.
constexpr int SIGMA_BATCH_MAX = 4;
struct PrimeBatch {
    int n = 0;
    ModP mp[SIGMA_BATCH_MAX];
    __host__ __device__ bool small() const {
        for (int i = 0; i < n; ++i)
            if (mp[i].p > 65536u) return false;
        return true;
    }
    __host__ __device__ bool large() const {
        for (int i = 0; i < n; ++i)
            if (mp[i].p <= 65536u) return false;
        return true;
    }
    __host__ __device__ uint32_t max_p() const {
        uint32_t m = 0;
        for (int i = 0; i < n; ++i) m = mp[i].p > m ? mp[i].p : m;
        return m;
    }
};

// Constants of one transform size N and the target primes of a batch over T <= 3 FFT primes.
struct NttConsts {
    uint32_t q[3];
    ModP mq[3];
    uint32_t r32[3];              // 2^32 mod q_t
    uint32_t ninv[3], ninvp[3];   // N^-1 mod q_t and its Shoup constant
    uint32_t inv01, inv012;       // q0^-1 mod q1, (q0 q1)^-1 mod q2
    uint32_t q0p[SIGMA_BATCH_MAX], q01p[SIGMA_BATCH_MAX];  // q0 mod p_b, q0 q1 mod p_b
    int64_t tw_stride;            // twiddle table length per prime
};

hipError_t gpu_load_polys(const uint32_t* src, int64_t ld, int64_t len, int64_t off, int nb, int64_t N, int T,
                          const NttConsts& c, uint32_t* dst, hipStream_t st);
hipError_t gpu_ntt(uint32_t* a, int lg, int nb, int T, const NttConsts& c, const uint32_t* tw, const uint32_t* itw,
                   bool forward, hipStream_t st);
// Transform-domain products of a batch: C_b = A_b B_b (r x k times k x c per batch element).
hipError_t gpu_pointwise(const uint32_t* A, const uint32_t* B, uint32_t* C, int r, int k, int c, int nbatch,
                         int64_t N, int T, const NttConsts& cs, hipStream_t st);
// npoly transformed polys (per_batch per batch element) back to residues mod the batch element's prime.
hipError_t gpu_crt(const uint32_t* C, int npoly, int per_batch, int64_t N, int64_t lo, int64_t W, int T,
                   const NttConsts& cs, const PrimeBatch& pb, uint32_t* out, hipStream_t st);
hipError_t gpu_schoolbook(const uint32_t* A, int64_t lenA, const uint32_t* B, int64_t lenB, int r, int k, int c,
                          int64_t lo, int64_t W, const PrimeBatch& pb, uint32_t* out, hipStream_t st);
// One workgroup per batch element b: the leaf of G + b gbs (degrees d + b m, output P + b pbs) mod p_b.
hipError_t gpu_mbasis_leaf(const uint32_t* G, int64_t ldG, int64_t gbs, int m, int n, int sigma, int64_t* d,
                           uint32_t* P, int64_t ldP, int64_t pbs, const PrimeBatch& pb, hipStream_t st);
size_t mbasis_leaf_lds(int m, int n, int sigma);
// LDS of the one-transform-per-order leaf (used for m = 2n, n <= LEAF2_MAX_S).
constexpr int LEAF2_MAX_S = 16;
size_t mbasis_leaf2_lds(int m, int n, int sigma);
// Coefficients k0 .. k1 - 1 of G = [S(x); -I_s], a 2s x s polynomial matrix with entries of length len
// (stride len); S holds L terms and coefficients k >= L of the S rows are zero.
hipError_t gpu_build_G(const uint32_t* S, int64_t L, int s, uint32_t p, uint32_t* G, int64_t len, int64_t k0,
                       int64_t k1, hipStream_t st);

// Rows chosen for the generator (at most 64): basis row indices and their shifted degrees.
struct GenRows {
    int32_t row[64];
    int64_t delta[64];
};
// dst[r * dld + x] = src[r * sld + x] for x < width, r < nrows (device memory)
hipError_t gpu_copy_rows(uint32_t* dst, int64_t dld, const uint32_t* src, int64_t sld, int64_t width, int64_t nrows,
                         hipStream_t st);
// out (s x s x olen) = the first s columns of the chosen rows of P (m x m, stride ld, len coefficients),
// coefficients above each row's shifted degree zeroed; *bad |= 1 if such a coefficient is non-zero.
hipError_t gpu_extract_rows(const uint32_t* P, int64_t ld, int64_t len, int m, int s, const GenRows& gr, int64_t olen,
                            uint32_t* out, int32_t* bad, hipStream_t st);

// A batch of device polynomial matrices: entry (r, c) of batch element b holds coefficients
// ptr[((b * rows + r) * cols + c) * ld + k], k < len.
struct DPoly {
    int rows = 0, cols = 0;
    int64_t len = 0;  // coefficients in use
    int64_t ld = 0;   // stride between entries (>= len)
    uint32_t* ptr = nullptr;
    int batch = 1;
};

// Largest leaf order (power of two <= 32) whose M-Basis fits the LDS budget; 0 if none.
int gpu_leaf_order(int s);

// Minimal generator of the device sequence S (L x s x s) on the device; the
// chosen rows come back to the host in `out`.  min_chunk > 0 takes the order
// range in the chunks of OnlineGenerator (same result; used by tests).
Error gpu_min_generator(const uint32_t* S_dev, int64_t L, int32_t s, uint32_t p, hipStream_t st, Generator* out,
                        SigmaStats* stats = nullptr, int64_t min_chunk = 0);
// The generators of nb <= SIGMA_BATCH_MAX sequences of the same length and block size, one prime each
// (all <= 2^16 or all larger), computed in one recursion: every leaf and product launch serves all of them.
Error gpu_min_generators(const uint32_t* const* S_dev, int nb, int64_t L, int32_t s, const uint32_t* p,
                         hipStream_t st, Generator* out);

// Sigma-basis of order L computed while the sequence is still being produced.
// The order range [0, L) is cut into chunks [c_{i-1}, c_i) (quarters of L while
// half of it is left, then halves of the rest down to min_chunk, then the
// rest); the basis of chunk i is the PM-Basis
// of the residual (Q_{i-1} G) mod x^{c_i} div x^{c_{i-1}}, with Q_{i-1} the
// product of the earlier chunks' bases, and Q_i = P_i Q_{i-1}.  Every order's
// M-Basis transform depends only on its residual coefficient and the shifted
// degrees, so the result equals the basis of one PM-Basis call over [0, L).
// Chunk i needs the terms S_0 .. S_{c_i - 1} only, so it can run on its own
// stream while the sequence computes later terms.
class OnlineGenerator {
   public:
    ~OnlineGenerator();
    // Work is enqueued on st; S_dev (L x s x s, device) must stay allocated until finish() returns.
    Error begin(const uint32_t* S_dev, int64_t L, int32_t s, uint32_t p, int64_t min_chunk, hipStream_t st) {
        return begin(&S_dev, 1, L, s, &p, min_chunk, st);
    }
    // A batch of nb sequences (same L and s), one prime each (all <= 2^16 or all larger).
    Error begin(const uint32_t* const* S_dev, int nb, int64_t L, int32_t s, const uint32_t* p, int64_t min_chunk,
                hipStream_t st);
    // The first `avail` terms of S_dev are complete once `ready` (an event recorded on the producer's
    // stream, or null when they are complete already) has fired: enqueue every chunk they cover.
    Error feed(int64_t avail, hipEvent_t ready);
    // Same, from a host thread of the generator's own (started on first use), so that the caller (which
    // enqueues the sequence) never waits on the basis stream's queue.  Takes ownership of `ready`.
    void feed_async(int64_t avail, hipEvent_t ready);
    // Call after feed(L, ...) or feed_async(L, ...): waits for the basis and returns the generator (one
    // per batch element).
    Error finish(Generator* out);
    // chunk end the next feed must reach to enqueue more work; -1 when every chunk is enqueued or queued
    // (not in early-termination mode, whose cuts are chosen by the worker: feed every chunk of terms there)
    int64_t next_boundary() const { return pending_ < (int64_t)cuts_.size() ? cuts_[pending_] : -1; }
    int chunks() const { return (int)cuts_.size(); }

    // Early termination (the outlook of the paper's conclusion; one sequence only).  The order range is cut
    // as the terms arrive: the first cut at max(step, L/8), then every `step` orders.  After each chunk the
    // sum of the s smallest shifted degrees (the generator rows' degrees) is compared with its value at the
    // previous cut.  While the sequence still looks generic the s pivots of every order include generator
    // rows, so that sum grows by about s/2 per order; when it has not changed over at least `verify` orders,
    // none of those rows was a pivot over them, i.e. every generator row annihilated the terms of those
    // orders.  The basis is then kept at that order (converged()), later feeds are ignored, and finish()
    // returns the generator of that order.  Once the other s rows' degrees sum to at least s * verify more
    // than the generator rows' (they have taken the pivots for that long), the next cut is only `verify`
    // orders on, to confirm the stall early (twice that after a confirming cut that did not confirm, and so
    // on up to `step`).
    Error begin_early(const uint32_t* S_dev, int64_t L, int32_t s, uint32_t p, int64_t step, int64_t verify,
                      hipStream_t st);
    int64_t converged() const { return conv_.load(); }  // order of the kept basis, 0 while not converged
    // (tests of the fallback) declare convergence at the first cut at or past order c, stalled or not
    void force_converge_at(int64_t c) { force_at_ = c; }
    int64_t order() const { return done_; }              // order of the basis computed so far

   private:
    Error join_worker();
    Error after_chunk_early();
    const uint32_t* S_[SIGMA_BATCH_MAX] = {};
    int64_t L_ = 0, built_ = 0, done_ = 0;
    int32_t s_ = 0;
    PrimeBatch pb_;
    int leaf_ = 0;
    hipStream_t st_ = nullptr;
    std::vector<int64_t> cuts_;  // chunk ends, increasing, last = L
    int next_ = 0;               // first chunk not enqueued on st_
    int pending_ = 0;            // first chunk not covered by a feed (caller's view)
    DevBuf gb_, db_, qb_;
    DPoly G_, Q_;
    // feed_async worker
    std::thread worker_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<std::pair<int64_t, hipEvent_t>> queue_;
    bool closing_ = false;
    Error werr_;
    // early termination
    bool early_ = false;
    int64_t step_ = 0, verify_ = 0, force_at_ = 0;
    EarlyCutState ecs_;
    std::atomic<int64_t> conv_{0};
};

// Window [lo, hi) of the products A_b B_b of two batches of device polynomial matrices, mod p_b.
Error gpu_polymat_mul(const DPoly& A, const DPoly& B, int64_t lo, int64_t hi, const PrimeBatch& pb, DPoly* C,
                      DevBuf* Cbuf, hipStream_t st);

}  // namespace bwr
