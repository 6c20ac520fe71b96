// Sparse x block product mod p with the non-zeros of a row split over lanes,
// optionally fused with the U^T projection of its output (the "A^T A u" and
// "U^T v" operations of a sequence step, Table "tab:r-opp"; projections done
// by blocks as in Section 2.3).
//
// Mapping (wave64): a row of the W-wide output is owned by LPR = (W/4) * G
// lanes.  Lane (cg, j) of the row gathers the 4 columns cg*4 .. cg*4+3 of X
// for the non-zeros t = b + j, b + j + G, ... of the row (16 bytes per
// non-zero; 8 when p <= 2^16 and residues are stored in 16 bits), so G lanes walk a row in parallel and the dependent chain
// "load index -> gather" is about len / (4 G) deep instead of len / 4.  The G
// partial sums meet in a butterfly of cross-lane shuffles (every lane ends
// with the full sum), one Barrett reduction and the diagonal scale follow,
// and lane j = 0 stores.
//
// Projection (PROJ): the W x W partial U^T X of the rows a block visits is
// spread over the row's lanes: lane (cg, j) owns entries i = j*(W/G) .. +W/G-1
// times columns cg*4 .. +3 and keeps them across its rows (grid-stride
// loop).  Partials meet through shuffles (row slots of a wave) and LDS (the
// 4 waves), and one W x W partial per block goes to memory, reduced later by
// k_reduce_partials.  Sums are exact in 64 bits: products of residues below
// 2^16 are < 2^32 and summed as they are; for larger primes each product is
// reduced and a lane keeps its sums mod p in 32 bits (fewer registers).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"

namespace bwr {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, mask, 64);
    hi = __shfl_xor(hi, mask, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int32_t shfl_xor_acc(int32_t v, int mask) { return __shfl_xor(v, mask, 64); }
__device__ __forceinline__ int64_t shfl_xor_acc(int64_t v, int mask) {
    return (int64_t)shfl_xor_u64((uint64_t)v, mask);
}

// 4 consecutive residues: one 16-byte load (uint32 storage) or 8-byte load (uint16 storage)
__device__ __forceinline__ void load4(const uint32_t* p, uint32_t (&x)[4]) {
    uint4 v = *reinterpret_cast<const uint4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
}
__device__ __forceinline__ void load4(const uint16_t* p, uint32_t (&x)[4]) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    x[0] = v.x & 0xffffu;
    x[1] = v.x >> 16;
    x[2] = v.y & 0xffffu;
    x[3] = v.y >> 16;
}
__device__ __forceinline__ void store4(uint32_t* p, const uint32_t (&y)[4]) {
    *reinterpret_cast<uint4*>(p) = make_uint4(y[0], y[1], y[2], y[3]);
}
__device__ __forceinline__ void store4(uint16_t* p, const uint32_t (&y)[4]) {
    *reinterpret_cast<uint2*>(p) = make_uint2(y[0] | (y[1] << 16), y[2] | (y[3] << 16));
}

template <int N, typename E>
__device__ __forceinline__ void loadn(const E* p, uint32_t (&x)[N]) {
    if constexpr (N == 4) {
        load4(p, x);
    } else {
#pragma unroll
        for (int q = 0; q < N; ++q) x[q] = p[q];
    }
}

// acc += a * x for one residue x: int32 (ACC 1), two int32 over the 16-bit halves of x (ACC 2), or int64 (ACC 0)
template <int ACC, typename Acc>
__device__ __forceinline__ void mac(Acc& acc, int32_t& ah, int32_t& al, int32_t a, uint32_t x) {
    if constexpr (ACC == 1) {
        acc += __mul24(a, (int32_t)x);
    } else if constexpr (ACC == 2) {
        ah += __mul24(a, (int32_t)(x >> 16));
        al += __mul24(a, (int32_t)(x & 0xffffu));
    } else {
        acc += (int64_t)a * (int64_t)x;
    }
}

// PASS 0: one pass over the row.  PASS 1: first of two column parts: the reduced sum goes to carry (no scale,
// no store, no projection).  PASS 2: second part: carry is added before the scale, store and projection.
template <int W, int G, int ACC, bool SMALLP, bool PROJ, typename E, int PASS>
__device__ __forceinline__ void spmm_split_body(int64_t nrows, const int32_t* __restrict__ rp,
                                                const uint32_t* __restrict__ ent, const E* __restrict__ X,
                                                const uint32_t* __restrict__ scale, E* __restrict__ Y,
                                                const E* __restrict__ U, uint32_t* __restrict__ partial, ModP mp,
                                                uint32_t* __restrict__ carry) {
    constexpr int CG = W / 4;
    constexpr int LPR = CG * G;
    static_assert(LPR <= 64 && 64 % LPR == 0, "row group must divide a wave");
    constexpr int RPW = 64 / LPR;
    constexpr int RPB = (TPB / 64) * RPW;
    constexpr int IPL = PROJ ? W / G : 1;
    static_assert(!PROJ || (W % G == 0 && IPL <= 4), "projection needs W / G <= 4");
    // ACC 1: int32 sums (16-bit primes, bounded rows); 2: residues split into 16-bit halves summed in two
    // int32 with full-rate 24-bit multiplies (large primes, bounded share of a row per lane); 0: int64
    constexpr bool ACC32 = ACC == 1;
    using Acc = typename std::conditional<ACC32, int32_t, int64_t>::type;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane % LPR;
    const int cg = sub % CG;
    const int j = sub / CG;
    const int slot = lane / LPR;

    // projection sums: 64-bit sums of exact products below 2^32 (16-bit primes), else residues summed mod p
    // (32 bits, so the kernel keeps the occupancy of the unfused product)
    using PAcc = typename std::conditional<SMALLP, uint64_t, uint32_t>::type;
    PAcc pacc[IPL][4];
#pragma unroll
    for (int u = 0; u < IPL; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) pacc[u][v] = 0;

    for (int64_t tile = blockIdx.x; tile * RPB < nrows; tile += gridDim.x) {
        const int64_t row = tile * RPB + wave * RPW + slot;
        const bool active = row < nrows;
        Acc acc[4] = {0, 0, 0, 0};
        int32_t ah[4] = {0, 0, 0, 0}, al[4] = {0, 0, 0, 0};
        if (active) {
            const int32_t b = rp[row], e = rp[row + 1];
            const E* Xs = X + cg * 4;
            // 4 entries per lane in flight, then 2, then the rest of the lane's share one by one (measured
            // faster on the planted matrices than predicated rounds, which cost registers and occupancy)
            int32_t t = b + j;
            for (; t + 3 * G < e; t += 4 * G) {
                uint32_t en[4];
                uint32_t x[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) en[u] = ent[t + u * G];
#pragma unroll
                for (int u = 0; u < 4; ++u) load4(Xs + (size_t)(en[u] & 0xFFFFFFu) * W, x[u]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int32_t a = (int32_t)en[u] >> 24;
#pragma unroll
                    for (int c = 0; c < 4; ++c) mac<ACC>(acc[c], ah[c], al[c], a, x[u][c]);
                }
            }
            if (t + G < e) {  // two more entries in flight together
                const uint32_t en0 = ent[t], en1 = ent[t + G];
                uint32_t x0[4], x1[4];
                load4(Xs + (size_t)(en0 & 0xFFFFFFu) * W, x0);
                load4(Xs + (size_t)(en1 & 0xFFFFFFu) * W, x1);
                const int32_t a0 = (int32_t)en0 >> 24, a1 = (int32_t)en1 >> 24;
#pragma unroll
                for (int c = 0; c < 4; ++c) mac<ACC>(acc[c], ah[c], al[c], a0, x0[c]);
#pragma unroll
                for (int c = 0; c < 4; ++c) mac<ACC>(acc[c], ah[c], al[c], a1, x1[c]);
                t += 2 * G;
            }
            for (; t < e; t += G) {
                const uint32_t en0 = ent[t];
                uint32_t x[4];
                load4(Xs + (size_t)(en0 & 0xFFFFFFu) * W, x);
                const int32_t a = (int32_t)en0 >> 24;
#pragma unroll
                for (int c = 0; c < 4; ++c) mac<ACC>(acc[c], ah[c], al[c], a, x[c]);
            }
        }
        if constexpr (ACC == 2) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = (int64_t)ah[c] * 65536 + al[c];
        }
        // all G slices of the row end with the full sum
#pragma unroll
        for (int off = CG; off < LPR; off <<= 1)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] += shfl_xor_acc(acc[c], off);
        if (PASS == 1) {
            if (active && j == 0) {
                uint32_t r[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) r[c] = ACC32 ? reds32(mp, (int32_t)acc[c]) : reds64(mp, (int64_t)acc[c]);
                store4(carry + (size_t)row * W + cg * 4, r);
            }
            continue;
        }
        if (active) {
            const uint32_t sc = scale ? scale[row] : 1u;
            uint32_t y[4], cin[4] = {0, 0, 0, 0};
            if (PASS == 2) load4(carry + (size_t)row * W + cg * 4, cin);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                uint32_t r = ACC32 ? reds32(mp, (int32_t)acc[c]) : reds64(mp, (int64_t)acc[c]);
                if (PASS == 2) r = addmod(mp, r, cin[c]);
                y[c] = SMALLP ? mulmod16(mp, r, sc) : mulmod(mp, r, sc);
            }
            if (j == 0) store4(Y + (size_t)row * W + cg * 4, y);
            if constexpr (PROJ) {
                uint32_t u[IPL];
                loadn<IPL, E>(U + (size_t)row * W + j * IPL, u);
#pragma unroll
                for (int q = 0; q < IPL; ++q)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (SMALLP) {
                            pacc[q][c] += (uint64_t)(u[q] * y[c]);
                        } else {
                            pacc[q][c] = addmod(mp, pacc[q][c], mulmod(mp, u[q], y[c]));
                        }
                    }
            }
        }
    }
    if constexpr (PROJ) {
        // sum over the row slots of the wave (lanes with equal sub); at most 64 terms below 2^32 each
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
        for (int e = threadIdx.x; e < W * W; e += TPB) {
            uint64_t s = 0;
#pragma unroll
            for (int w = 0; w < TPB / 64; ++w) s += sh[w][e];
            partial[(size_t)blockIdx.x * W * W + e] = red64(mp, s);
        }
    }
}

template <int W, int G, int ACC, bool SMALLP, bool PROJ, typename E, int PASS>
__global__ __launch_bounds__(TPB) void k_spmm_split(int64_t nrows, const int32_t* __restrict__ rp,
                                                    const uint32_t* __restrict__ ent, const E* __restrict__ X,
                                                    const uint32_t* __restrict__ scale, E* __restrict__ Y,
                                                    const E* __restrict__ U, uint32_t* __restrict__ partial,
                                                    ModP mp, uint32_t* __restrict__ carry) {
    spmm_split_body<W, G, ACC, SMALLP, PROJ, E, PASS>(nrows, rp, ent, X, scale, Y, U, partial, mp, carry);
}

// The same kernel held to 72 registers (7 waves per SIMD instead of 6): used for the 8-wide fused
// projection with 32-bit residues and G >= 4, which fits 72 registers without spilling.
template <int W, int G, int ACC, bool SMALLP, bool PROJ, typename E, int PASS>
__global__ __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(7))) void k_spmm_split_o7(
    int64_t nrows, const int32_t* __restrict__ rp, const uint32_t* __restrict__ ent, const E* __restrict__ X,
    const uint32_t* __restrict__ scale, E* __restrict__ Y, const E* __restrict__ U, uint32_t* __restrict__ partial,
    ModP mp, uint32_t* __restrict__ carry) {
    spmm_split_body<W, G, ACC, SMALLP, PROJ, E, PASS>(nrows, rp, ent, X, scale, Y, U, partial, mp, carry);
}

bool use_o7() {
    static const bool on = getenv("BWR_NO_O7") == nullptr;
    return on;
}

struct Args {
    int64_t nrows;
    const int32_t* rp;
    const uint32_t* ent;
    const void* X;
    const uint32_t* scale;
    void* Y;
    const void* U;
    uint32_t* partial;
    ModP mp;
    uint32_t* carry;
};

template <int W, int G, bool PROJ, typename E, int PASS>
hipError_t launch_wgep(int acc, bool smallp, unsigned grid, const Args& a, hipStream_t st) {
    const E* X = (const E*)a.X;
    E* Y = (E*)a.Y;
    const E* U = (const E*)a.U;
#define BWR_SPLIT_ARGS a.nrows, a.rp, a.ent, X, a.scale, Y, U, a.partial, a.mp, a.carry
    if (acc == 1) {
        k_spmm_split<W, G, 1, true, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
    } else if (smallp) {
        k_spmm_split<W, G, 0, true, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
    } else {
        if constexpr (PROJ && W == 8 && G >= 4 && PASS == 0 && std::is_same<E, uint32_t>::value) {
            if (use_o7()) {
                if (acc == 2)
                    k_spmm_split_o7<W, G, 2, false, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
                else
                    k_spmm_split_o7<W, G, 0, false, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
                return hipGetLastError();
            }
        }
        if (acc == 2)
            k_spmm_split<W, G, 2, false, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
        else
            k_spmm_split<W, G, 0, false, PROJ, E, PASS><<<grid, TPB, 0, st>>>(BWR_SPLIT_ARGS);
    }
#undef BWR_SPLIT_ARGS
    return hipGetLastError();
}

template <int W, int G, bool PROJ>
hipError_t launch_wg(int acc, bool smallp, int esize, int pass, unsigned grid, const Args& a, hipStream_t st) {
    if (esize == 2) {
        if (pass != 0) return hipErrorInvalidValue;  // column parts are for 32-bit residues only
        return launch_wgep<W, G, PROJ, uint16_t, 0>(acc, true, grid, a, st);
    }
    if (pass == 1) {
        if constexpr (!PROJ) return launch_wgep<W, G, false, uint32_t, 1>(acc, smallp, grid, a, st);
        return hipErrorInvalidValue;
    }
    if (pass == 2) return launch_wgep<W, G, PROJ, uint32_t, 2>(acc, smallp, grid, a, st);
    return launch_wgep<W, G, PROJ, uint32_t, 0>(acc, smallp, grid, a, st);
}

template <int W, int G>
hipError_t launch_g(bool proj, int acc, bool smallp, int esize, int pass, unsigned grid, const Args& a,
                    hipStream_t st) {
    if constexpr ((W / 4) * G <= 64) {
        if (proj) {
            if constexpr (W % G == 0 && W / G <= 4)
                return launch_wg<W, G, true>(acc, smallp, esize, pass, grid, a, st);
            return hipErrorInvalidValue;
        }
        return launch_wg<W, G, false>(acc, smallp, esize, pass, grid, a, st);
    }
    return hipErrorInvalidValue;
}

template <int W>
hipError_t launch_w(int G, bool proj, int acc, bool smallp, int esize, int pass, unsigned grid, const Args& a,
                    hipStream_t st) {
    switch (G) {
        case 1: return launch_g<W, 1>(proj, acc, smallp, esize, pass, grid, a, st);
        case 2: return launch_g<W, 2>(proj, acc, smallp, esize, pass, grid, a, st);
        case 4: return launch_g<W, 4>(proj, acc, smallp, esize, pass, grid, a, st);
        case 8: return launch_g<W, 8>(proj, acc, smallp, esize, pass, grid, a, st);
        case 16: return launch_g<W, 16>(proj, acc, smallp, esize, pass, grid, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool split_supported(int W, int G, bool proj) {
    if (W < 4 || W > 64 || (G & (G - 1)) || G < 1 || G > 16) return false;
    if ((W / 4) * G > 64) return false;
    if (proj && (W % G != 0 || W / G > 4)) return false;
    return true;
}

int split_rows_per_block(int W, int G) { return (TPB / 64) * (64 / ((W / 4) * G)); }

hipError_t launch_spmm_split(int W, int G, bool proj, int acc, bool smallp, int esize, int64_t nrows,
                             const int32_t* rp, const uint32_t* ent, const void* X, const uint32_t* scale, void* Y,
                             const void* U, uint32_t* partial, int nblocks, ModP mp, hipStream_t st, int pass,
                             uint32_t* carry) {
    if (!split_supported(W, G, proj) || (acc == 1 && !smallp) || (acc == 2 && smallp) || acc < 0 || acc > 2 ||
        (esize == 2 && !smallp) || (esize != 2 && esize != 4) || pass < 0 || pass > 2 || (pass && !carry) ||
        (pass == 1 && proj))
        return hipErrorInvalidValue;
    const int rpb = split_rows_per_block(W, G);
    int64_t tiles = (nrows + rpb - 1) / rpb;
    if (tiles < 1) tiles = 1;
    unsigned grid = proj ? (unsigned)nblocks : (unsigned)tiles;
    if (grid < 1) grid = 1;
    const Args a{nrows, rp, ent, X, scale, Y, U, partial, mp, carry};
    switch (W) {
        case 4: return launch_w<4>(G, proj, acc, smallp, esize, pass, grid, a, st);
        case 8: return launch_w<8>(G, proj, acc, smallp, esize, pass, grid, a, st);
        case 16: return launch_w<16>(G, proj, acc, smallp, esize, pass, grid, a, st);
        case 32: return launch_w<32>(G, proj, acc, smallp, esize, pass, grid, a, st);
        case 64: return launch_w<64>(G, proj, acc, smallp, esize, pass, grid, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bwr
