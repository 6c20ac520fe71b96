// Batched sequences: many (matrix, primes) jobs advanced together, one launch
// per product per step for all of them.  Internal C++; the public surface is
// bwr_rank_modp_batch and the server in bwrank.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modp.h"

namespace bwr {

constexpr int BATCH_MAX_PRIMES = 4;

// Device-resident descriptor of one job.  A job iterates one matrix with a
// W-wide block whose columns [t*spad, t*spad + s) belong to prime t (spad is
// s rounded up to a multiple of 4, so a lane's 4 columns share one prime).
struct BatchJob {
    int64_t rows1, rows2;  // rows of the first product (outer) and second (nb)
    const int32_t* rp1;
    const uint32_t* ent1;
    const int32_t* rp2;
    const uint32_t* ent2;
    uint32_t* X[2];        // ping-pong iterated block, nb x W (residues of the runner's storage size)
    uint32_t* Y;           // outer x W (same storage)
    const uint32_t* Ut;    // D_c^-1 U, nb x W (same storage)
    const uint32_t* dr;    // [nprimes][outer]
    const uint32_t* dc2;   // [nprimes][nb]
    uint32_t* S;           // [nprimes][len][s][s]
    ModP mp[BATCH_MAX_PRIMES];
    int32_t nprimes, spad, s, par;  // par: ping-pong parity offset
    int32_t nblk2;                  // blocks of the second product (partials per step)
    int32_t pad0;
    int64_t len;        // sequence terms of the job
    int64_t g0;         // global step at which the job makes its first application of B
    int64_t part_off;   // offset (uint32 words) of the job's partials inside one step slot
};

int batch_rows_per_block(int W, int G);
// Row split G valid for width W (second = the product carrying the projection).
bool batch_supported(int W, int G, bool second);

// Accumulator mode for a launch over jobs whose rows have at most max_len non-zeros of absolute value at
// most max_abs: 2 (16-bit halves in int32) when a lane's share of a row keeps those sums below 2^31, else
// 0 (int64).
int batch_acc_mode(int64_t max_len, int32_t max_abs, int G);
// First product for all jobs: block b belongs to the job j with start[j] <= b < start[j+1].
// esize: bytes per stored residue (2 when every prime of the jobs is <= 2^16, else 4).
hipError_t launch_batch_first(int W, int G, int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs,
                              int nblocks, int parity, hipStream_t st);
// Second product + per-prime projection partials into partial + slot_off.
hipError_t launch_batch_second(int W, int G, int acc, int esize, const BatchJob* jobs, const int32_t* start,
                               int njobs, int nblocks, int parity, uint32_t* partial, int64_t slot_off,
                               hipStream_t st);
// S terms of the chunk [g_first, g_first + nsteps) for every job (slot k of the chunk at k * slot_words).
hipError_t launch_batch_reduce(const BatchJob* jobs, int njobs, int64_t g_first, int nsteps, const uint32_t* partial,
                               int64_t slot_words, int max_entries, hipStream_t st);
// S_0 of one job (host descriptor copy): partials over nblk blocks, then the reduction.
hipError_t launch_batch_s0(int W, int esize, const BatchJob& job, uint32_t* partial, int nblk, hipStream_t st);
// out[r * W + off + c] = (in[r * s + c] mod p) * d[r]^(+1, -1 or 0) for c < s (mode 1, 2, 0); out holds
// esize-byte residues.
hipError_t launch_place_block(int64_t n, int32_t s, int W, int off, const uint32_t* in, const uint32_t* d, int mode,
                              ModP mp, void* out, int esize, hipStream_t st);

}  // namespace bwr
