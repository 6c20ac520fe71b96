// Batched sequence kernels: one launch advances one product of a step for
// every active job (matrix x set of primes).  The row mapping is that of the
// row-split kernel (W/4 column groups x G non-zero slices per row); each
// column group belongs to one prime of the job, so a single pass over a
// matrix serves all its primes and a gathered row of the block is W * 4 bytes
// (128 bytes for 4 primes x 8 columns: one cache line per non-zero).
// Accumulators: ACC 2 sums the 16-bit halves of the residues in two int32
// with full-rate 24-bit multiplies (when every active job's rows are short
// enough for the sums to stay below 2^31), ACC 0 sums in int64; primes of any
// size mix in one launch.  Projection sums are kept mod p in 32 bits.
// Residues are stored in 32 bits (E = uint32_t) or, when every prime of the
// launch is <= 2^16, in 16 bits (E = uint16_t: a gathered row of 3 primes x 8
// columns, padded to 32, is 64 bytes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "batch.h"
#include "kernels.h"

namespace bwr {

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, mask, 64);
    hi = __shfl_xor(hi, mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int find_job(const int32_t* __restrict__ start, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// 4 consecutive residues of storage type E
__device__ __forceinline__ uint4 load4e(const uint32_t* p) { return *reinterpret_cast<const uint4*>(p); }
__device__ __forceinline__ uint4 load4e(const uint16_t* p) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    return make_uint4(v.x & 0xffffu, v.x >> 16, v.y & 0xffffu, v.y >> 16);
}
__device__ __forceinline__ void store4e(uint32_t* p, const uint32_t (&y)[4]) {
    *reinterpret_cast<uint4*>(p) = make_uint4(y[0], y[1], y[2], y[3]);
}
__device__ __forceinline__ void store4e(uint16_t* p, const uint32_t (&y)[4]) {
    *reinterpret_cast<uint2*>(p) = make_uint2(y[0] | (y[1] << 16), y[2] | (y[3] << 16));
}

template <int W, int G, bool SECOND, int ACC, typename E>
__global__ __launch_bounds__(TPB) void k_batch(const BatchJob* __restrict__ jobs, const int32_t* __restrict__ start,
                                               int njobs, int parity, uint32_t* __restrict__ partial,
                                               int64_t slot_off) {
    constexpr int CG = W / 4;
    constexpr int LPR = CG * G;
    static_assert(LPR <= 64 && 64 % LPR == 0, "row group must divide a wave");
    constexpr int RPW = 64 / LPR;
    constexpr int RPB = (TPB / 64) * RPW;
    constexpr int IPL = SECOND ? W / G : 1;
    static_assert(!SECOND || (W % G == 0 && IPL <= 4), "projection needs W / G <= 4");

    const int jb = find_job(start, njobs, (int)blockIdx.x);
    const BatchJob& J = jobs[jb];
    const int lb = (int)blockIdx.x - start[jb];
    const int nblk = start[jb + 1] - start[jb];
    const int64_t rows = SECOND ? J.rows2 : J.rows1;
    const int32_t* __restrict__ rp = SECOND ? J.rp2 : J.rp1;
    const uint32_t* __restrict__ ent = SECOND ? J.ent2 : J.ent1;
    const int cur = (parity + J.par) & 1;
    const E* __restrict__ X = reinterpret_cast<const E*>(SECOND ? J.Y : J.X[cur]);
    E* __restrict__ Y = reinterpret_cast<E*>(SECOND ? J.X[cur ^ 1] : J.Y);
    const E* __restrict__ Ut = reinterpret_cast<const E*>(J.Ut);
    const uint32_t* __restrict__ scale = SECOND ? J.dc2 : J.dr;
    const int spad = J.spad, np = J.nprimes;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane % LPR;
    const int cg = sub % CG;
    const int j = sub / CG;
    const int slot = lane / LPR;
    const int tp = (cg * 4) / spad;  // prime of this lane's columns
    const bool live = tp < np;
    const ModP mp = J.mp[live ? tp : 0];

    uint32_t pacc[IPL][4];  // projection sums mod the lane's prime
#pragma unroll
    for (int u = 0; u < IPL; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) pacc[u][v] = 0;

    for (int64_t tile = lb; tile * RPB < rows; tile += nblk) {
        const int64_t row = tile * RPB + wave * RPW + slot;
        const bool active = row < rows;
        int64_t acc[4] = {0, 0, 0, 0};
        int32_t ah[4] = {0, 0, 0, 0}, al[4] = {0, 0, 0, 0};
        if (active && live) {
            const int32_t b = rp[row], e = rp[row + 1];
            const E* Xs = X + cg * 4;
            auto mac = [&](int32_t a, const uint4& x) {
                const uint32_t xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if constexpr (ACC == 2) {
                        ah[c] += __mul24(a, (int32_t)(xv[c] >> 16));
                        al[c] += __mul24(a, (int32_t)(xv[c] & 0xffffu));
                    } else {
                        acc[c] += (int64_t)a * (int64_t)xv[c];
                    }
                }
            };
            int32_t t = b + j;
            for (; t + 3 * G < e; t += 4 * G) {
                uint32_t en[4];
                uint4 x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) en[u] = ent[t + u * G];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = load4e(Xs + (size_t)(en[u] & 0xFFFFFFu) * W);
#pragma unroll
                for (int u = 0; u < 4; ++u) mac((int32_t)en[u] >> 24, x[u]);
            }
            for (; t < e; t += G) {
                const uint32_t en0 = ent[t];
                const uint4 x = load4e(Xs + (size_t)(en0 & 0xFFFFFFu) * W);
                mac((int32_t)en0 >> 24, x);
            }
        }
        if constexpr (ACC == 2) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = (int64_t)ah[c] * 65536 + al[c];
        }
#pragma unroll
        for (int off = CG; off < LPR; off <<= 1)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += (int64_t)shfl_xor_u64((uint64_t)acc[c], off);
        if (active) {
            uint32_t y[4] = {0, 0, 0, 0};
            if (live) {
                const uint32_t sc = scale[(size_t)tp * rows + row];
#pragma unroll
                for (int c = 0; c < 4; ++c) y[c] = mulmod(mp, reds64(mp, acc[c]), sc);
            }
            if (j == 0) store4e(Y + (size_t)row * W + cg * 4, y);
            if constexpr (SECOND) {
                if (live) {
#pragma unroll
                    for (int q = 0; q < IPL; ++q) {
                        const int i = j * IPL + q;
                        if (i / spad != tp) continue;  // only the diagonal blocks of one prime
                        const uint32_t u = Ut[(size_t)row * W + i];
#pragma unroll
                        for (int c = 0; c < 4; ++c) pacc[q][c] = addmod(mp, pacc[q][c], mulmod(mp, u, y[c]));
                    }
                }
            }
        }
    }
    if constexpr (SECOND) {
        // sums over the row slots of the wave: at most 64 terms below 2^31 each
        uint64_t ps[IPL][4];
#pragma unroll
        for (int q = 0; q < IPL; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) ps[q][c] = pacc[q][c];
#pragma unroll
        for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
            for (int q = 0; q < IPL; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) ps[q][c] += shfl_xor_u64(ps[q][c], off);
        __shared__ uint64_t sh[TPB / 64][W * W];
        if (lane < LPR) {
#pragma unroll
            for (int q = 0; q < IPL; ++q)
#pragma unroll
                for (int c = 0; c < 4; ++c) sh[wave][(j * IPL + q) * W + cg * 4 + c] = ps[q][c];
        }
        __syncthreads();
        const int per = spad * spad;
        uint32_t* out = partial + slot_off + J.part_off + (int64_t)lb * np * per;
        for (int e = threadIdx.x; e < np * per; e += TPB) {
            const int t = e / per, ii = (e % per) / spad, cc = e % spad;
            const int wi = (t * spad + ii) * W + t * spad + cc;
            uint64_t s = 0;
#pragma unroll
            for (int w = 0; w < TPB / 64; ++w) s += sh[w][wi];
            out[e] = red64(J.mp[t], s);
        }
    }
}

// grid: x over the steps of the chunk, y over jobs; 16 groups of 64 lanes split the job's partial
// blocks (each wave reads consecutive words), LDS adds the groups
constexpr int BRED_TPB = 1024;
__global__ __launch_bounds__(BRED_TPB) void k_batch_reduce(const BatchJob* __restrict__ jobs, int64_t g_first,
                                                           const uint32_t* __restrict__ partial, int64_t slot_words) {
    __shared__ uint64_t sh[BRED_TPB / 64][64];
    const BatchJob& J = jobs[blockIdx.y];
    const int s = J.s, spad = J.spad, np = J.nprimes;
    const int k = blockIdx.x;
    const int64_t kl = g_first + k - J.g0 + 1;  // the job's sequence index
    if (kl < 1 || kl >= J.len) return;          // uniform over the block
    const int per = spad * spad;
    const int per_step = np * s * s;
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const uint32_t* base = partial + (int64_t)k * slot_words + J.part_off;
    for (int e0 = 0; e0 < per_step; e0 += 64) {
        const int e = e0 + lane;
        int t = 0, i = 0, c = 0;
        uint64_t acc = 0;
        if (e < per_step) {
            t = e / (s * s);
            i = (e % (s * s)) / s;
            c = e % s;
            const uint32_t* src = base + (int64_t)t * per + i * spad + c;
            for (int b = g; b < J.nblk2; b += BRED_TPB / 64) acc += src[(int64_t)b * np * per];
        }
        sh[g][lane] = acc;
        __syncthreads();
        if (g == 0 && e < per_step) {
            uint64_t tot = 0;
#pragma unroll
            for (int q = 0; q < BRED_TPB / 64; ++q) tot += sh[q][lane];
            J.S[((int64_t)t * J.len + kl) * s * s + i * s + c] = red64(J.mp[t], tot);
        }
        __syncthreads();
    }
}

// S_0: thread t owns diagonal entries e = t, t + TPB, ... of the job; blocks split the rows
template <int W, typename E>
__global__ __launch_bounds__(TPB) void k_batch_s0(BatchJob J, uint32_t* __restrict__ partial) {
    const int spad = J.spad, np = J.nprimes, per = spad * spad;
    const int64_t nb = J.rows2;
    const int64_t rpb = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < nb ? r0 + rpb : nb;
    const E* X0 = reinterpret_cast<const E*>(J.X[0]);  // the initial block (the first step reads X[0])
    const E* Ut = reinterpret_cast<const E*>(J.Ut);
    for (int e = threadIdx.x; e < np * per; e += TPB) {
        const int t = e / per, ii = (e % per) / spad, cc = e % spad;
        const ModP mp = J.mp[t];
        uint64_t acc = 0;
        for (int64_t r = r0; r < r1; ++r) acc += mulmod(mp, Ut[r * W + t * spad + ii], X0[r * W + t * spad + cc]);
        partial[(int64_t)blockIdx.x * np * per + e] = red64(mp, acc);
    }
}

__global__ __launch_bounds__(TPB) void k_batch_s0_reduce(BatchJob J, const uint32_t* __restrict__ partial, int nblk) {
    const int s = J.s, spad = J.spad, np = J.nprimes, per = spad * spad;
    const int idx = blockIdx.x * TPB + threadIdx.x;
    if (idx >= np * s * s) return;
    const int t = idx / (s * s), i = (idx % (s * s)) / s, c = idx % s;
    uint64_t acc = 0;
    for (int b = 0; b < nblk; ++b) acc += partial[(int64_t)b * np * per + t * per + i * spad + c];
    J.S[((int64_t)t * J.len) * s * s + i * s + c] = red64(J.mp[t], acc);
}

template <typename E>
__global__ __launch_bounds__(TPB) void k_place_block(int64_t n, int32_t s, int W, int off, const uint32_t* __restrict__ in,
                                                     const uint32_t* __restrict__ d, int mode, ModP mp,
                                                     E* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= n * (int64_t)s) return;
    int64_t r = idx / s;
    int c = (int)(idx - r * s);
    uint32_t x = red32(mp, in[idx]);
    if (mode == 1) x = mulmod(mp, x, red32(mp, d[r]));
    else if (mode == 2) x = mulmod(mp, x, invmod(mp, red32(mp, d[r])));
    out[r * W + off + c] = (E)x;
}

template <int W, int G>
hipError_t first_wg(int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs, int nblocks,
                    int parity, hipStream_t st) {
    if constexpr ((W / 4) * G <= 64) {
        // 16-bit residues under acc 2: the high halves are 0, so one int32 sum carries the product
        if (esize == 2 && acc == 2)
            k_batch<W, G, false, 2, uint16_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, nullptr, 0);
        else if (esize == 2)
            k_batch<W, G, false, 0, uint16_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, nullptr, 0);
        else if (acc == 2)
            k_batch<W, G, false, 2, uint32_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, nullptr, 0);
        else
            k_batch<W, G, false, 0, uint32_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, nullptr, 0);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int W, int G>
hipError_t second_wg(int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs, int nblocks, int parity,
                     uint32_t* partial, int64_t slot_off, hipStream_t st) {
    if constexpr ((W / 4) * G <= 64 && W % G == 0 && W / G <= 4) {
        if (esize == 2 && acc == 2)
            k_batch<W, G, true, 2, uint16_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, partial, slot_off);
        else if (esize == 2)
            k_batch<W, G, true, 0, uint16_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, partial, slot_off);
        else if (acc == 2)
            k_batch<W, G, true, 2, uint32_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, partial, slot_off);
        else
            k_batch<W, G, true, 0, uint32_t><<<nblocks, TPB, 0, st>>>(jobs, start, njobs, parity, partial, slot_off);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int W>
hipError_t first_w(int G, int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs, int nblocks, int parity,
                   hipStream_t st) {
    switch (G) {
        case 1: return first_wg<W, 1>(acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 2: return first_wg<W, 2>(acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 4: return first_wg<W, 4>(acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 8: return first_wg<W, 8>(acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 16: return first_wg<W, 16>(acc, esize, jobs, start, njobs, nblocks, parity, st);
        default: return hipErrorInvalidValue;
    }
}

template <int W>
hipError_t second_w(int G, int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs, int nblocks, int parity,
                    uint32_t* partial, int64_t slot_off, hipStream_t st) {
    switch (G) {
        case 1: return second_wg<W, 1>(acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 2: return second_wg<W, 2>(acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 4: return second_wg<W, 4>(acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 8: return second_wg<W, 8>(acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 16: return second_wg<W, 16>(acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int batch_rows_per_block(int W, int G) { return (TPB / 64) * (64 / ((W / 4) * G)); }

int batch_acc_mode(int64_t max_len, int32_t max_abs, int G) {
    const int64_t share = (max_len + G - 1) / G;  // non-zeros of a row one lane sums
    return share * (int64_t)std::max(max_abs, 1) * 65535 < ((int64_t)1 << 31) ? 2 : 0;
}

bool batch_supported(int W, int G, bool second) {
    if (W != 4 && W != 8 && W != 16 && W != 32) return false;
    if (G < 1 || G > 16 || (G & (G - 1))) return false;
    if ((W / 4) * G > 64) return false;
    return !second || (W % G == 0 && W / G <= 4);
}

hipError_t launch_batch_first(int W, int G, int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs,
                              int nblocks, int parity, hipStream_t st) {
    if ((acc != 0 && acc != 2) || (esize != 2 && esize != 4)) return hipErrorInvalidValue;
    if (nblocks <= 0 || njobs <= 0) return hipSuccess;
    switch (W) {
        case 4: return first_w<4>(G, acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 8: return first_w<8>(G, acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 16: return first_w<16>(G, acc, esize, jobs, start, njobs, nblocks, parity, st);
        case 32: return first_w<32>(G, acc, esize, jobs, start, njobs, nblocks, parity, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_second(int W, int G, int acc, int esize, const BatchJob* jobs, const int32_t* start, int njobs,
                               int nblocks, int parity, uint32_t* partial, int64_t slot_off, hipStream_t st) {
    if ((acc != 0 && acc != 2) || (esize != 2 && esize != 4)) return hipErrorInvalidValue;
    if (nblocks <= 0 || njobs <= 0) return hipSuccess;
    switch (W) {
        case 4: return second_w<4>(G, acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 8: return second_w<8>(G, acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 16: return second_w<16>(G, acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        case 32: return second_w<32>(G, acc, esize, jobs, start, njobs, nblocks, parity, partial, slot_off, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_reduce(const BatchJob* jobs, int njobs, int64_t g_first, int nsteps, const uint32_t* partial,
                               int64_t slot_words, int max_entries, hipStream_t st) {
    (void)max_entries;
    if (njobs <= 0 || nsteps <= 0) return hipSuccess;
    dim3 grid((unsigned)nsteps, (unsigned)njobs);
    k_batch_reduce<<<grid, BRED_TPB, 0, st>>>(jobs, g_first, partial, slot_words);
    return hipGetLastError();
}

hipError_t launch_batch_s0(int W, int esize, const BatchJob& job, uint32_t* partial, int nblk, hipStream_t st) {
    if (esize == 2) {
        switch (W) {
            case 4: k_batch_s0<4, uint16_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 8: k_batch_s0<8, uint16_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 16: k_batch_s0<16, uint16_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 32: k_batch_s0<32, uint16_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (W) {
            case 4: k_batch_s0<4, uint32_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 8: k_batch_s0<8, uint32_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 16: k_batch_s0<16, uint32_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            case 32: k_batch_s0<32, uint32_t><<<nblk, TPB, 0, st>>>(job, partial); break;
            default: return hipErrorInvalidValue;
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_batch_s0_reduce<<<grid_for((int64_t)job.nprimes * job.s * job.s, TPB), TPB, 0, st>>>(job, partial, nblk);
    return hipGetLastError();
}

hipError_t launch_place_block(int64_t n, int32_t s, int W, int off, const uint32_t* in, const uint32_t* d, int mode,
                              ModP mp, void* out, int esize, hipStream_t st) {
    int64_t total = n * (int64_t)s;
    if (total == 0) return hipSuccess;
    if (esize == 2)
        k_place_block<uint16_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, off, in, d, mode, mp, (uint16_t*)out);
    else
        k_place_block<uint32_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, off, in, d, mode, mp, (uint32_t*)out);
    return hipGetLastError();
}

}  // namespace bwr
