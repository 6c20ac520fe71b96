// Kernels of the symmetric projection U = V (Section 2.3, "block symmetry":
// with B = D_c A^T D_r A D_c symmetric, S_k = V^T B^k V is symmetric).
//
// Check: with U = V the sequence's symmetry is a property of the products,
// not of how S_k is formed (S_k = (D_c^-1 V)^T X_k with X_k = D_c B^k V), so
// k_sym_check comparing S_k[i][j] with S_k[j][i] checks every term's products.
//
// Gram form (the identities below are standard; the paper does not use them):
// with W_k = B^k V, S_2k = W_k^T W_k and S_2k+1 = (A D_c W_k)^T D_r (A D_c W_k),
// so one application of B gives two terms.  In the iterated quantities
// X_k = D_c W_k and Y_k = D_r A X_k (the first product's output):
//     S_2k   = sum_r d_c[r]^-2 X_k[r] (x) X_k[r]
//     S_2k+1 = sum_r d_r[r]^-1 Y_k[r] (x) Y_k[r]
// k_gram forms such a weighted Gram matrix's partial sums (entries i <= j
// only; the others are mirrored after the reduction by k_mirror).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.h"

namespace bwr {

namespace {

constexpr int TPB = 256;

// partial[b][i W + j] = sum over the rows of block b of w[r] X[r][i] X[r][j] mod p for i <= j (0 for i > j);
// w null: weight 1.  Exact: each product is reduced before the 64-bit sums.
template <int W, bool SMALLP, typename T>
__global__ __launch_bounds__(TPB) void k_gram(int64_t n, const T* __restrict__ X, const uint32_t* __restrict__ w,
                                              uint32_t* __restrict__ partial, int64_t rows_per_block, ModP mp) {
    constexpr int E = W * W;
    constexpr int EPT = E >= TPB ? E / TPB : 1;
    constexpr int R = E >= TPB ? 1 : TPB / E;
    __shared__ uint64_t sh[TPB * EPT];
    const int t = threadIdx.x;
    const int ph = E >= TPB ? 0 : t / E;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    int64_t r1 = r0 + rows_per_block;
    if (r1 > n) r1 = n;
    uint64_t acc[EPT];
    int ii[EPT], cc[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
        const int e = E >= TPB ? t + TPB * q : t % E;
        ii[q] = e / W;
        cc[q] = e % W;
        acc[q] = 0;
    }
    for (int64_t r = r0 + ph; r < r1; r += R) {
        const uint32_t wr = w ? w[r] : 1u;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            if (ii[q] > cc[q]) continue;
            const uint32_t a = X[r * W + ii[q]], b = X[r * W + cc[q]];
            const uint32_t ab = SMALLP ? mulmod16(mp, a, b) : mulmod(mp, a, b);
            acc[q] += SMALLP ? (uint64_t)(ab * wr) : (uint64_t)mulmod(mp, ab, wr);
        }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) sh[t + TPB * q] = acc[q];
    __syncthreads();
    if (R > 1) {
        if (t < E) {
            uint64_t s = 0;
            for (int k = 0; k < R; ++k) s += sh[t + k * E];
            partial[(int64_t)blockIdx.x * E + t] = red64(mp, s);
        }
    } else {
#pragma unroll
        for (int q = 0; q < EPT; ++q) partial[(int64_t)blockIdx.x * E + t + TPB * q] = red64(mp, sh[t + TPB * q]);
    }
}

// S[k][j][i] = S[k][i][j] for i < j, k < nsteps
__global__ __launch_bounds__(TPB) void k_mirror(int64_t nsteps, int32_t s, uint32_t* __restrict__ S) {
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t per = (int64_t)s * s;
    if (idx >= nsteps * per) return;
    const int64_t k = idx / per;
    const int i = (int)((idx % per) / s), j = (int)(idx % s);
    if (i < j) S[k * per + (int64_t)j * s + i] = S[k * per + (int64_t)i * s + j];
}

// bad = 1 if some S[k][i][j] != S[k][j][i]
__global__ __launch_bounds__(TPB) void k_sym_check(int64_t nsteps, int32_t s, const uint32_t* __restrict__ S,
                                                   int32_t* __restrict__ bad) {
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t per = (int64_t)s * s;
    if (idx >= nsteps * per) return;
    const int64_t k = idx / per;
    const int i = (int)((idx % per) / s), j = (int)(idx % s);
    if (i < j && S[k * per + (int64_t)i * s + j] != S[k * per + (int64_t)j * s + i]) atomicOr(bad, 1);
}

// out[r] = d[r]^-power mod p (power 1 or 2), 0 where d[r] = 0 mod p; d null: out[r] = 1
__global__ __launch_bounds__(TPB) void k_inv_diag(int64_t n, const uint32_t* __restrict__ d, ModP mp, int power,
                                                  uint32_t* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (r >= n) return;
    if (!d) {
        out[r] = 1u % mp.p;
        return;
    }
    const uint32_t x = red32(mp, d[r]);
    uint32_t v = x ? powmod(mp, x, mp.p - 2) : 0u;
    if (power == 2) v = mulmod(mp, v, v);
    out[r] = v;
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + TPB - 1) / TPB); }

template <int W, typename T>
hipError_t gram_w(bool smallp, int64_t n, const T* X, const uint32_t* w, uint32_t* partial, int nblocks, ModP mp,
                  hipStream_t st) {
    const int64_t rpb = (n + nblocks - 1) / nblocks;
    if (smallp)
        k_gram<W, true, T><<<nblocks, TPB, 0, st>>>(n, X, w, partial, rpb, mp);
    else
        k_gram<W, false, T><<<nblocks, TPB, 0, st>>>(n, X, w, partial, rpb, mp);
    return hipGetLastError();
}

template <typename T>
hipError_t gram_t(int W, bool smallp, int64_t n, const T* X, const uint32_t* w, uint32_t* partial, int nblocks,
                  ModP mp, hipStream_t st) {
    switch (W) {
        case 1: return gram_w<1, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 2: return gram_w<2, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 4: return gram_w<4, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 8: return gram_w<8, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 16: return gram_w<16, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 32: return gram_w<32, T>(smallp, n, X, w, partial, nblocks, mp, st);
        case 64: return gram_w<64, T>(smallp, n, X, w, partial, nblocks, mp, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_gram(int W, bool smallp, int64_t n, const void* X, int esize, const uint32_t* w, uint32_t* partial,
                       int nblocks, ModP mp, hipStream_t st) {
    if (nblocks < 1) return hipErrorInvalidValue;
    if (esize == 2) return gram_t<uint16_t>(W, smallp, n, (const uint16_t*)X, w, partial, nblocks, mp, st);
    return gram_t<uint32_t>(W, smallp, n, (const uint32_t*)X, w, partial, nblocks, mp, st);
}

hipError_t launch_mirror(int64_t nsteps, int32_t s, uint32_t* S, hipStream_t st) {
    if (nsteps <= 0 || s <= 1) return hipSuccess;
    k_mirror<<<grid_of(nsteps * s * s), TPB, 0, st>>>(nsteps, s, S);
    return hipGetLastError();
}

hipError_t launch_sym_check(int64_t nsteps, int32_t s, const uint32_t* S, int32_t* bad, hipStream_t st) {
    if (nsteps <= 0 || s <= 1) return hipSuccess;
    k_sym_check<<<grid_of(nsteps * s * s), TPB, 0, st>>>(nsteps, s, S, bad);
    return hipGetLastError();
}

hipError_t launch_inv_diag(int64_t n, const uint32_t* d, ModP mp, int power, uint32_t* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_inv_diag<<<grid_of(n), TPB, 0, st>>>(n, d, mp, power, out);
    return hipGetLastError();
}

}  // namespace bwr
