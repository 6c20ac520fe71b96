// gfx950 kernels for the block Wiedemann projection sequence S_k = U^T B^k V
// over GF(p), B = D_c A^T D_r A D_c (Sections 2.2, 2.3 and step 2 of the rank
// algorithm in Section 2.5).
//
// The hot loop is two exact sparse-matrix x block products mod p (the "A^T A u"
// products that take 97-99 % of a step in Table "tab:r-opp"), a diagonal scale
// fused into each product's epilogue, and the U^T projection ("U^T v", done by
// blocks as in Section 2.3).  Everything is integer work bound by memory
// bandwidth; there is no dense contraction to feed the matrix cores except the
// projection, which is tiny.
//
// SpMM mapping (wave64): a row of the output block (W residues) is owned by
// W/4 lanes that each hold 4 columns (one 16-byte gather per non-zero), so a
// wave covers 64*4/W rows and a non-zero costs one index load shared by the
// row's lanes plus one dwordx4 gather per lane.  Sums are delayed: int32
// accumulators when max_len * max|a| * (p-1) < 2^31 (16-bit primes), int64
// otherwise, and one Barrett reduction per output element.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include <type_traits>

#include "kernels.h"
#include "splitmix.h"

namespace bwr {

namespace {

constexpr int TPB = 256;

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ---------------------------------------------------------------- validation
// Row pointers first (without touching the entries): 0 = rp[0] <= ... <= rp[m] = nnz.
__global__ __launch_bounds__(TPB) void k_rowptr_check(int64_t m, int64_t nnz, const int64_t* __restrict__ rp,
                                                      int32_t* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i > m) return;
    int64_t v = rp[i];
    bool ok = v >= 0 && v <= nnz;
    if (i == 0) ok = ok && v == 0;
    if (i == m) ok = ok && v == nnz;
    if (i < m) ok = ok && rp[i + 1] >= v;
    if (!ok) atomicOr(bad, BAD_ROWPTR);
}

__global__ __launch_bounds__(TPB) void k_max_i32(int64_t count, const int32_t* __restrict__ in, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < count) atomicMax(out, in[i]);
}

__global__ __launch_bounds__(TPB) void k_csr_stats(int64_t m, int64_t n, const int64_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ val,
                                                   CsrStats* out) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    int64_t b = rp[i], e = rp[i + 1];
    int32_t bad = 0;
    if (i == 0 && b != 0) bad |= BAD_ROWPTR;
    if (e < b) {
        bad |= BAD_ROWPTR;
        e = b;
    }
    int64_t len = e - b;
    int32_t mx = 0;
    for (int64_t t = b; t < e; ++t) {
        int32_t c = col[t];
        if (c < 0 || (int64_t)c >= n) bad |= BAD_COL;
        int32_t v = val[t];
        int32_t a = v == INT32_MIN ? INT32_MAX : (v < 0 ? -v : v);
        mx = a > mx ? a : mx;
    }
    if (bad) atomicOr(&out->bad, bad);
    atomicMax(&out->max_len, (int32_t)(len > INT32_MAX ? INT32_MAX : len));
    atomicMax(&out->max_abs, mx);
}

// ---------------------------------------------------------------- encoding
__device__ __forceinline__ uint32_t pack_entry(int32_t c, int32_t v) {
    return (uint32_t)c | ((uint32_t)(uint8_t)(int8_t)v << 24);
}

__global__ __launch_bounds__(TPB) void k_pack_rows(int64_t m, const int64_t* __restrict__ rp64,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ val,
                                                   int32_t* __restrict__ rp32, uint32_t* __restrict__ ent) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i > m) return;
    rp32[i] = (int32_t)rp64[i];
    if (i == m) return;
    for (int64_t t = rp64[i]; t < rp64[i + 1]; ++t) ent[t] = pack_entry(col[t], val[t]);
}

__global__ __launch_bounds__(TPB) void k_wide_rows(int64_t m, const int64_t* __restrict__ rp64,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ val,
                                                   ModP mp, int32_t* __restrict__ rp32, int32_t* __restrict__ colw,
                                                   uint32_t* __restrict__ valw) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i > m) return;
    rp32[i] = (int32_t)rp64[i];
    if (i == m) return;
    for (int64_t t = rp64[i]; t < rp64[i + 1]; ++t) {
        colw[t] = col[t];
        valw[t] = reds32(mp, val[t]);
    }
}

__global__ __launch_bounds__(TPB) void k_col_count(int64_t m, const int64_t* __restrict__ rp64,
                                                   const int32_t* __restrict__ col, int32_t* __restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    for (int64_t t = rp64[i]; t < rp64[i + 1]; ++t) atomicAdd(&cnt[col[t]], 1);
}

// Row i of the relabelled CSR is row perm_r[i] of the input with its columns mapped through inv_c
// (rp_out from the host: the scan of the permuted row lengths).
__global__ __launch_bounds__(TPB) void k_permute_csr(int64_t m, const int64_t* __restrict__ rp_out,
                                                     const int32_t* __restrict__ perm_r,
                                                     const int64_t* __restrict__ rp64, const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ val,
                                                     const int32_t* __restrict__ inv_c, int32_t* __restrict__ col_out,
                                                     int32_t* __restrict__ val_out) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    const int64_t o = perm_r[i];
    const int64_t b = rp64[o], e = rp64[o + 1], d = rp_out[i];
    for (int64_t t = b; t < e; ++t) {
        col_out[d + t - b] = inv_c[col[t]];
        val_out[d + t - b] = val[t];
    }
}

// dst[i][c] = src[perm[i]][c] for c < width
__global__ __launch_bounds__(TPB) void k_gather_rows(int64_t rows, int width, const int32_t* __restrict__ perm,
                                                     const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= rows * width) return;
    const int64_t i = idx / width;
    const int c = (int)(idx % width);
    dst[idx] = src[(int64_t)perm[i] * width + c];
}

// Three-phase exclusive scan of int32 counts (totals < 2^31).
constexpr int SCAN_TILE = 1024;

__global__ __launch_bounds__(TPB) void k_scan_tiles(int64_t count, const int32_t* __restrict__ in,
                                                    int32_t* __restrict__ out, int32_t* __restrict__ tile_sum) {
    __shared__ int32_t sh[SCAN_TILE];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    for (int k = threadIdx.x; k < SCAN_TILE; k += TPB) sh[k] = base + k < count ? in[base + k] : 0;
    __syncthreads();
    // each thread scans 4 consecutive elements, then a block scan of the 256 totals
    int32_t v0 = sh[4 * threadIdx.x], v1 = sh[4 * threadIdx.x + 1], v2 = sh[4 * threadIdx.x + 2],
            v3 = sh[4 * threadIdx.x + 3];
    int32_t tot = v0 + v1 + v2 + v3;
    __shared__ int32_t part[TPB];
    part[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < TPB; off <<= 1) {
        int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t excl = part[threadIdx.x] - tot;
    int64_t o = base + 4 * threadIdx.x;
    if (o < count) out[o] = excl;
    if (o + 1 < count) out[o + 1] = excl + v0;
    if (o + 2 < count) out[o + 2] = excl + v0 + v1;
    if (o + 3 < count) out[o + 3] = excl + v0 + v1 + v2;
    if (threadIdx.x == TPB - 1) tile_sum[blockIdx.x] = part[TPB - 1];
}

// single block: exclusive scan of the tile totals in place, grand total at tile_sum[ntiles]
__global__ __launch_bounds__(TPB) void k_scan_totals(int64_t ntiles, int32_t* __restrict__ tile_sum) {
    __shared__ int32_t part[TPB];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < ntiles; base += TPB) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < ntiles ? tile_sum[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < TPB; off <<= 1) {
            int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < ntiles) tile_sum[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == TPB - 1) carry += part[TPB - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ __launch_bounds__(TPB) void k_scan_add(int64_t count, int32_t* __restrict__ out,
                                                  const int32_t* __restrict__ tile_sum, int64_t ntiles) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i < count) out[i] += tile_sum[i / SCAN_TILE];
    if (i == count) out[count] = tile_sum[ntiles];
}

__global__ __launch_bounds__(TPB) void k_scatter_packed_t(int64_t m, const int64_t* __restrict__ rp64,
                                                          const int32_t* __restrict__ col,
                                                          const int32_t* __restrict__ val,
                                                          const int32_t* __restrict__ rpT, int32_t* __restrict__ cursor,
                                                          uint32_t* __restrict__ entT) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    for (int64_t t = rp64[i]; t < rp64[i + 1]; ++t) {
        int32_t c = col[t];
        int32_t pos = rpT[c] + atomicAdd(&cursor[c], 1);
        entT[pos] = pack_entry((int32_t)i, val[t]);
    }
}

__global__ __launch_bounds__(TPB) void k_scatter_wide_t(int64_t m, const int64_t* __restrict__ rp64,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ val, ModP mp,
                                                        const int32_t* __restrict__ rpT, int32_t* __restrict__ cursor,
                                                        int32_t* __restrict__ colT, uint32_t* __restrict__ valT) {
    int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (i >= m) return;
    for (int64_t t = rp64[i]; t < rp64[i + 1]; ++t) {
        int32_t c = col[t];
        int32_t pos = rpT[c] + atomicAdd(&cursor[c], 1);
        colT[pos] = (int32_t)i;
        valT[pos] = reds32(mp, val[t]);
    }
}

// ---------------------------------------------------------------- random blocks and scaling
__global__ __launch_bounds__(TPB) void k_rng_block(uint64_t key, int64_t rows, int32_t s, int32_t ld, ModP mp,
                                                   int diag, uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= rows * (int64_t)ld) return;
    int64_t r = idx / ld;
    int32_t c = (int32_t)(idx - r * ld);
    out[idx] = c < s ? sm_residue(mp, key, (uint64_t)(r * s + c), diag) : 0u;
}

template <typename E>
__global__ __launch_bounds__(TPB) void k_pad_scale(int64_t n, int32_t s, int32_t W, const uint32_t* __restrict__ in,
                                                   const uint32_t* __restrict__ d, int mode, ModP mp,
                                                   E* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= n * (int64_t)W) return;
    int64_t r = idx / W;
    int32_t c = (int32_t)(idx - r * W);
    uint32_t x = 0;
    if (c < s) {
        x = in[r * s + c];
        x = x >= mp.p ? x % mp.p : x;
        if (mode == 1) x = mulmod(mp, x, red32(mp, d[r]));
        else if (mode == 2) x = mulmod(mp, x, invmod(mp, red32(mp, d[r])));
    }
    out[idx] = (E)x;
}

template <typename E>
__global__ __launch_bounds__(TPB) void k_unpad(int64_t n, int32_t s, int32_t W, const E* __restrict__ in,
                                               uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= n * (int64_t)s) return;
    int64_t r = idx / s;
    int32_t c = (int32_t)(idx - r * s);
    out[idx] = in[r * W + c];
}

__global__ __launch_bounds__(TPB) void k_square_diag(int64_t n, const uint32_t* __restrict__ d, ModP mp,
                                                     uint32_t* __restrict__ d2, int32_t* bad) {
    int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (r >= n) return;
    uint32_t x = red32(mp, d[r]);
    if (x == 0) atomicOr(bad, 1);
    d2[r] = mulmod(mp, x, x);
}

// words 32-bit zeros at p (grid-stride), then `tail` zero bytes at t: a memset that is an ordinary kernel
__global__ __launch_bounds__(TPB) void k_fill_zero(uint32_t* __restrict__ p, int64_t words, uint8_t* __restrict__ t,
                                                   int tail) {
    for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < words; i += (int64_t)gridDim.x * TPB) p[i] = 0u;
    if (blockIdx.x == 0 && (int)threadIdx.x < tail) t[threadIdx.x] = 0;
}

__global__ __launch_bounds__(TPB) void k_reduce_vec(int64_t n, const uint32_t* __restrict__ in, ModP mp,
                                                    uint32_t* __restrict__ out) {
    int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (r >= n) return;
    out[r] = red32(mp, in[r]);
}

// ---------------------------------------------------------------- sparse x block mod p
template <int CPL>
struct Vec;
template <>
struct Vec<1> {
    using T = uint32_t;
    static __device__ __forceinline__ void load(const uint32_t* p, uint32_t (&x)[1]) { x[0] = *p; }
    static __device__ __forceinline__ void store(uint32_t* p, const uint32_t (&x)[1]) { *p = x[0]; }
};
template <>
struct Vec<2> {
    static __device__ __forceinline__ void load(const uint32_t* p, uint32_t (&x)[2]) {
        uint2 v = *reinterpret_cast<const uint2*>(p);
        x[0] = v.x;
        x[1] = v.y;
    }
    static __device__ __forceinline__ void store(uint32_t* p, const uint32_t (&x)[2]) {
        *reinterpret_cast<uint2*>(p) = make_uint2(x[0], x[1]);
    }
};
template <>
struct Vec<4> {
    static __device__ __forceinline__ void load(const uint32_t* p, uint32_t (&x)[4]) {
        uint4 v = *reinterpret_cast<const uint4*>(p);
        x[0] = v.x;
        x[1] = v.y;
        x[2] = v.z;
        x[3] = v.w;
    }
    static __device__ __forceinline__ void store(uint32_t* p, const uint32_t (&x)[4]) {
        *reinterpret_cast<uint4*>(p) = make_uint4(x[0], x[1], x[2], x[3]);
    }
};

template <int W>
struct Shape {
    static constexpr int LPR = W >= 4 ? W / 4 : 1;  // lanes per output row
    static constexpr int CPL = W / LPR;             // columns per lane
    static constexpr int RPB = TPB / LPR;           // rows per block
};

template <int W, bool ACC32, bool SMALLP>
__global__ __launch_bounds__(TPB) void k_spmm_packed(int64_t nrows, const int32_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ ent, const uint32_t* __restrict__ X,
                                                     const uint32_t* __restrict__ scale, uint32_t* __restrict__ Y,
                                                     ModP mp) {
    using Sh = Shape<W>;
    constexpr int CPL = Sh::CPL;
    using Acc = typename std::conditional<ACC32, int32_t, int64_t>::type;
    const int64_t g = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t row = g / Sh::LPR;
    const int sub = (int)(g - row * Sh::LPR);
    if (row >= nrows) return;
    const int32_t b = rp[row], e = rp[row + 1];
    Acc acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;
    const uint32_t* Xs = X + sub * CPL;
    int32_t t = b;
    for (; t + 4 <= e; t += 4) {
        uint32_t en[4];
        uint32_t x[4][CPL];
#pragma unroll
        for (int u = 0; u < 4; ++u) en[u] = ent[t + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) Vec<CPL>::load(Xs + (size_t)(en[u] & 0xFFFFFFu) * W, x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int32_t a = (int32_t)en[u] >> 24;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (ACC32) acc[c] += __mul24(a, (int32_t)x[u][c]);
                else acc[c] += (int64_t)a * (int64_t)x[u][c];
            }
        }
    }
    for (; t < e; ++t) {
        uint32_t en0 = ent[t];
        uint32_t x[CPL];
        Vec<CPL>::load(Xs + (size_t)(en0 & 0xFFFFFFu) * W, x);
        int32_t a = (int32_t)en0 >> 24;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            if (ACC32) acc[c] += __mul24(a, (int32_t)x[c]);
            else acc[c] += (int64_t)a * (int64_t)x[c];
        }
    }
    uint32_t out[CPL];
    const uint32_t sc = scale ? scale[row] : 1u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        uint32_t r = ACC32 ? reds32(mp, (int32_t)acc[c]) : reds64(mp, (int64_t)acc[c]);
        out[c] = SMALLP ? mulmod16(mp, r, sc) : mulmod(mp, r, sc);
    }
    Vec<CPL>::store(Y + (size_t)row * W + sub * CPL, out);
}

template <int W>
__global__ __launch_bounds__(TPB) void k_spmm_wide(int64_t nrows, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col, const uint32_t* __restrict__ val,
                                                   const uint32_t* __restrict__ X, const uint32_t* __restrict__ scale,
                                                   uint32_t* __restrict__ Y, ModP mp) {
    using Sh = Shape<W>;
    constexpr int CPL = Sh::CPL;
    const int64_t g = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t row = g / Sh::LPR;
    const int sub = (int)(g - row * Sh::LPR);
    if (row >= nrows) return;
    const int32_t b = rp[row], e = rp[row + 1];
    uint64_t acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;
    const uint32_t* Xs = X + sub * CPL;
    for (int32_t t = b; t < e; ++t) {
        uint32_t x[CPL];
        Vec<CPL>::load(Xs + (size_t)col[t] * W, x);
        uint32_t a = val[t];
        // each reduced product is < p < 2^31, so up to 2^33 of them fit in 64 bits
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += mulmod(mp, a, x[c]);
    }
    uint32_t out[CPL];
    const uint32_t sc = scale ? scale[row] : 1u;
#pragma unroll
    for (int c = 0; c < CPL; ++c) out[c] = mulmod(mp, red64(mp, acc[c]), sc);
    Vec<CPL>::store(Y + (size_t)row * W + sub * CPL, out);
}

// ---------------------------------------------------------------- projection U^T X
// Thread t of a block owns entries e = t + TPB q of the W x W result (E = W^2)
// and, when E < TPB, the row phase t / E.  Partial sums are exact in 64 bits:
// for p <= 2^16 products are < 2^32; otherwise each product is reduced first.
template <int W, bool SMALLP, typename T>
__global__ __launch_bounds__(TPB) void k_project(int64_t n, const T* __restrict__ U, const T* __restrict__ X,
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
        int e = E >= TPB ? t + TPB * q : t % E;
        ii[q] = e / W;
        cc[q] = e % W;
        acc[q] = 0;
    }
    for (int64_t r = r0 + ph; r < r1; r += R) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
            uint32_t u = U[r * W + ii[q]];
            uint32_t x = X[r * W + cc[q]];
            acc[q] += SMALLP ? (uint64_t)(u * x) : (uint64_t)mulmod(mp, u, x);
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

// S_k = sum over the nblocks partials of step k: one block per step; 16 groups of 64
// lanes split the partials (each wave reads 64 consecutive words), then LDS adds the groups.
constexpr int RED_TPB = 1024;
__global__ __launch_bounds__(RED_TPB) void k_reduce_partials(int W, int32_t s, int nblocks,
                                                             const uint32_t* __restrict__ partial, int64_t pstride,
                                                             uint32_t* __restrict__ S, int64_t sstride, ModP mp) {
    __shared__ uint64_t sh[RED_TPB / 64][64];
    const int64_t k = blockIdx.x;
    const int per = s * s;
    const int64_t E = (int64_t)W * W;
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const uint32_t* base = partial + k * pstride;
    for (int e0 = 0; e0 < per; e0 += 64) {
        const int e = e0 + lane;
        uint64_t acc = 0;
        if (e < per) {
            const uint32_t* src = base + (int64_t)(e / s) * W + (e % s);
            for (int b = g; b < nblocks; b += RED_TPB / 64) acc += src[(int64_t)b * E];
        }
        sh[g][lane] = acc;
        __syncthreads();
        if (g == 0 && e < per) {
            uint64_t t = 0;
#pragma unroll
            for (int q = 0; q < RED_TPB / 64; ++q) t += sh[q][lane];
            S[k * sstride * per + e] = red64(mp, t);
        }
        __syncthreads();
    }
}

// Column split of a packed operand: entries with column < mid go to part 0, the others to part 1
// (same order inside each row).
__global__ __launch_bounds__(TPB) void k_split_count(int64_t rows, const int32_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ ent, uint32_t mid,
                                                     int32_t* __restrict__ cnt0, int32_t* __restrict__ cnt1) {
    const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (r >= rows) return;
    int32_t c0 = 0;
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t) c0 += (ent[t] & 0xFFFFFFu) < mid ? 1 : 0;
    cnt0[r] = c0;
    cnt1[r] = rp[r + 1] - rp[r] - c0;
}

__global__ __launch_bounds__(TPB) void k_split_scatter(int64_t rows, const int32_t* __restrict__ rp,
                                                       const uint32_t* __restrict__ ent, uint32_t mid,
                                                       const int32_t* __restrict__ rp0, const int32_t* __restrict__ rp1,
                                                       uint32_t* __restrict__ ent0, uint32_t* __restrict__ ent1) {
    const int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (r >= rows) return;
    int32_t o0 = rp0[r], o1 = rp1[r];
    for (int32_t t = rp[r]; t < rp[r + 1]; ++t) {
        const uint32_t e = ent[t];
        if ((e & 0xFFFFFFu) < mid) ent0[o0++] = e;
        else ent1[o1++] = e;
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_rowptr_check(int64_t m, int64_t nnz, const int64_t* rp, int32_t* bad_dev, hipStream_t st) {
    hipError_t err = launch_fill_zero(bad_dev, sizeof(int32_t), st);
    if (err != hipSuccess) return err;
    k_rowptr_check<<<grid_for(m + 1, TPB), TPB, 0, st>>>(m, nnz, rp, bad_dev);
    return hipGetLastError();
}

hipError_t launch_max_i32(int64_t count, const int32_t* in, int32_t* out_dev, hipStream_t st) {
    hipError_t err = launch_fill_zero(out_dev, sizeof(int32_t), st);
    if (err != hipSuccess || count == 0) return err;
    k_max_i32<<<grid_for(count, TPB), TPB, 0, st>>>(count, in, out_dev);
    return hipGetLastError();
}

hipError_t launch_csr_stats(int64_t m, int64_t n, const int64_t* rp, const int32_t* col, const int32_t* val,
                            CsrStats* out_dev, hipStream_t st) {
    hipError_t err = launch_fill_zero(out_dev, sizeof(CsrStats), st);
    if (err != hipSuccess || m == 0) return err;
    k_csr_stats<<<grid_for(m, TPB), TPB, 0, st>>>(m, n, rp, col, val, out_dev);
    return hipGetLastError();
}

hipError_t launch_pack_rows(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val, int32_t* rp32,
                            uint32_t* ent, hipStream_t st) {
    k_pack_rows<<<grid_for(m + 1, TPB), TPB, 0, st>>>(m, rp64, col, val, rp32, ent);
    return hipGetLastError();
}

hipError_t launch_wide_rows(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val, ModP mp,
                            int32_t* rp32, int32_t* colw, uint32_t* valw, hipStream_t st) {
    k_wide_rows<<<grid_for(m + 1, TPB), TPB, 0, st>>>(m, rp64, col, val, mp, rp32, colw, valw);
    return hipGetLastError();
}

hipError_t launch_col_count(int64_t m, const int64_t* rp64, const int32_t* col, int32_t* cnt, hipStream_t st) {
    if (m == 0) return hipSuccess;
    k_col_count<<<grid_for(m, TPB), TPB, 0, st>>>(m, rp64, col, cnt);
    return hipGetLastError();
}

int64_t scan_tmp_words(int64_t count) { return (count + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t launch_permute_csr(int64_t m, const int64_t* rp_out, const int32_t* perm_r, const int64_t* rp64,
                              const int32_t* col, const int32_t* val, const int32_t* inv_c, int32_t* col_out,
                              int32_t* val_out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_permute_csr<<<grid_for(m, TPB), TPB, 0, st>>>(m, rp_out, perm_r, rp64, col, val, inv_c, col_out, val_out);
    return hipGetLastError();
}

hipError_t launch_gather_rows(int64_t rows, int width, const int32_t* perm, const uint32_t* src, uint32_t* dst,
                              hipStream_t st) {
    if (rows <= 0 || width <= 0) return hipSuccess;
    k_gather_rows<<<grid_for(rows * width, TPB), TPB, 0, st>>>(rows, width, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(int64_t count, const int32_t* in, int32_t* out, int32_t* tmp, hipStream_t st) {
    int64_t ntiles = (count + SCAN_TILE - 1) / SCAN_TILE;
    if (ntiles > 0) {
        k_scan_tiles<<<(unsigned)ntiles, TPB, 0, st>>>(count, in, out, tmp);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    k_scan_totals<<<1, TPB, 0, st>>>(ntiles, tmp);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_scan_add<<<grid_for(count + 1, TPB), TPB, 0, st>>>(count, out, tmp, ntiles);
    return hipGetLastError();
}

hipError_t launch_scatter_packed_t(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val,
                                   const int32_t* rpT, int32_t* cursor, uint32_t* entT, hipStream_t st) {
    if (m == 0) return hipSuccess;
    k_scatter_packed_t<<<grid_for(m, TPB), TPB, 0, st>>>(m, rp64, col, val, rpT, cursor, entT);
    return hipGetLastError();
}

hipError_t launch_scatter_wide_t(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val, ModP mp,
                                 const int32_t* rpT, int32_t* cursor, int32_t* colT, uint32_t* valT, hipStream_t st) {
    if (m == 0) return hipSuccess;
    k_scatter_wide_t<<<grid_for(m, TPB), TPB, 0, st>>>(m, rp64, col, val, mp, rpT, cursor, colT, valT);
    return hipGetLastError();
}

hipError_t launch_rng_block(uint64_t seed, int stream, int64_t rows, int32_t s, int32_t ld, ModP mp, int diag,
                            uint32_t* out, hipStream_t st) {
    int64_t total = rows * (int64_t)ld;
    if (total == 0) return hipSuccess;
    k_rng_block<<<grid_for(total, TPB), TPB, 0, st>>>(sm_key(seed, stream), rows, s, ld, mp, diag, out);
    return hipGetLastError();
}

hipError_t launch_pad_scale(int64_t n, int32_t s, int32_t W, const uint32_t* in, const uint32_t* d, int mode,
                            ModP mp, void* out, int esize, hipStream_t st) {
    int64_t total = n * (int64_t)W;
    if (total == 0) return hipSuccess;
    if (esize == 2)
        k_pad_scale<uint16_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, in, d, mode, mp, (uint16_t*)out);
    else
        k_pad_scale<uint32_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, in, d, mode, mp, (uint32_t*)out);
    return hipGetLastError();
}

hipError_t launch_unpad(int64_t n, int32_t s, int32_t W, const void* in, int esize, uint32_t* out, hipStream_t st) {
    int64_t total = n * (int64_t)s;
    if (total == 0) return hipSuccess;
    if (esize == 2)
        k_unpad<uint16_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, (const uint16_t*)in, out);
    else
        k_unpad<uint32_t><<<grid_for(total, TPB), TPB, 0, st>>>(n, s, W, (const uint32_t*)in, out);
    return hipGetLastError();
}

hipError_t launch_square_diag(int64_t n, const uint32_t* d, ModP mp, uint32_t* d2, int32_t* bad, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_square_diag<<<grid_for(n, TPB), TPB, 0, st>>>(n, d, mp, d2, bad);
    return hipGetLastError();
}

hipError_t launch_reduce_vec(int64_t n, const uint32_t* in, ModP mp, uint32_t* out, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_reduce_vec<<<grid_for(n, TPB), TPB, 0, st>>>(n, in, mp, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
    if (bytes == 0) return hipSuccess;
    const int64_t words = (int64_t)(bytes / 4);
    const int64_t tail = (int64_t)(bytes % 4);
    const int64_t n = std::max<int64_t>(words, tail ? 1 : 0);
    const int64_t blocks = std::min<int64_t>((n + TPB - 1) / TPB, 65536);
    k_fill_zero<<<(unsigned)std::max<int64_t>(blocks, 1), TPB, 0, st>>>(reinterpret_cast<uint32_t*>(p), words,
                                                                       reinterpret_cast<uint8_t*>(p) + 4 * words,
                                                                       (int)tail);
    return hipGetLastError();
}

template <int W>
static hipError_t spmm_packed_w(bool acc32, bool smallp, int64_t nrows, const int32_t* rp, const uint32_t* ent,
                                const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st) {
    unsigned grid = grid_for(nrows, Shape<W>::RPB);
    if (acc32)
        k_spmm_packed<W, true, true><<<grid, TPB, 0, st>>>(nrows, rp, ent, X, scale, Y, mp);
    else if (smallp)
        k_spmm_packed<W, false, true><<<grid, TPB, 0, st>>>(nrows, rp, ent, X, scale, Y, mp);
    else
        k_spmm_packed<W, false, false><<<grid, TPB, 0, st>>>(nrows, rp, ent, X, scale, Y, mp);
    return hipGetLastError();
}

hipError_t launch_spmm_packed(int W, bool acc32, bool smallp, int64_t nrows, const int32_t* rp, const uint32_t* ent,
                              const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    if (acc32 && !smallp) return hipErrorInvalidValue;
    switch (W) {
        case 1: return spmm_packed_w<1>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 2: return spmm_packed_w<2>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 4: return spmm_packed_w<4>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 8: return spmm_packed_w<8>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 16: return spmm_packed_w<16>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 32: return spmm_packed_w<32>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        case 64: return spmm_packed_w<64>(acc32, smallp, nrows, rp, ent, X, scale, Y, mp, st);
        default: return hipErrorInvalidValue;
    }
}

template <int W>
static hipError_t spmm_wide_w(int64_t nrows, const int32_t* rp, const int32_t* col, const uint32_t* val,
                              const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st) {
    k_spmm_wide<W><<<grid_for(nrows, Shape<W>::RPB), TPB, 0, st>>>(nrows, rp, col, val, X, scale, Y, mp);
    return hipGetLastError();
}

hipError_t launch_spmm_wide(int W, int64_t nrows, const int32_t* rp, const int32_t* col, const uint32_t* val,
                            const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st) {
    if (nrows == 0) return hipSuccess;
    switch (W) {
        case 1: return spmm_wide_w<1>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 2: return spmm_wide_w<2>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 4: return spmm_wide_w<4>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 8: return spmm_wide_w<8>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 16: return spmm_wide_w<16>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 32: return spmm_wide_w<32>(nrows, rp, col, val, X, scale, Y, mp, st);
        case 64: return spmm_wide_w<64>(nrows, rp, col, val, X, scale, Y, mp, st);
        default: return hipErrorInvalidValue;
    }
}

int proj_blocks(int64_t n, int W) {
    (void)W;
    int64_t b = (n + 255) / 256;
    if (b > 512) b = 512;
    if (b < 1) b = 1;
    return (int)b;
}

template <int W, typename T>
static hipError_t project_w(bool smallp, int64_t n, const T* U, const T* X, uint32_t* partial, int nblocks, ModP mp,
                            hipStream_t st) {
    int64_t rpb = (n + nblocks - 1) / nblocks;
    if (smallp)
        k_project<W, true, T><<<nblocks, TPB, 0, st>>>(n, U, X, partial, rpb, mp);
    else
        k_project<W, false, T><<<nblocks, TPB, 0, st>>>(n, U, X, partial, rpb, mp);
    return hipGetLastError();
}

template <typename T>
static hipError_t project_t(int W, bool smallp, int64_t n, const T* U, const T* X, uint32_t* partial, int nblocks,
                            ModP mp, hipStream_t st) {
    switch (W) {
        case 1: return project_w<1, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 2: return project_w<2, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 4: return project_w<4, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 8: return project_w<8, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 16: return project_w<16, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 32: return project_w<32, T>(smallp, n, U, X, partial, nblocks, mp, st);
        case 64: return project_w<64, T>(smallp, n, U, X, partial, nblocks, mp, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_project(int W, bool smallp, int64_t n, const void* U, const void* X, int esize, uint32_t* partial,
                          int nblocks, ModP mp, hipStream_t st) {
    if (esize == 2)
        return project_t<uint16_t>(W, smallp, n, (const uint16_t*)U, (const uint16_t*)X, partial, nblocks, mp, st);
    return project_t<uint32_t>(W, smallp, n, (const uint32_t*)U, (const uint32_t*)X, partial, nblocks, mp, st);
}

hipError_t launch_reduce_partials(int W, int32_t s, int nblocks, int64_t nsteps, const uint32_t* partial, uint32_t* S,
                                  ModP mp, hipStream_t st, int64_t pstride, int64_t sstride) {
    if (nsteps <= 0 || s <= 0) return hipSuccess;
    if (pstride <= 0) pstride = (int64_t)nblocks * W * W;
    k_reduce_partials<<<(unsigned)nsteps, RED_TPB, 0, st>>>(W, s, nblocks, partial, pstride, S, sstride, mp);
    return hipGetLastError();
}

}  // namespace bwr

namespace bwr {

hipError_t launch_split_operand(int64_t rows, const int32_t* rp, const uint32_t* ent, uint32_t mid, int32_t* cnt0,
                                int32_t* cnt1, int32_t* tmp, int32_t* rp0, int32_t* rp1, uint32_t* ent0, uint32_t* ent1,
                                hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    k_split_count<<<grid_for(rows, TPB), TPB, 0, st>>>(rows, rp, ent, mid, cnt0, cnt1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_exclusive_scan(rows, cnt0, rp0, tmp, st);
    if (e == hipSuccess) e = launch_exclusive_scan(rows, cnt1, rp1, tmp, st);
    if (e != hipSuccess) return e;
    k_split_scatter<<<grid_for(rows, TPB), TPB, 0, st>>>(rows, rp, ent, mid, rp0, rp1, ent0, ent1);
    return hipGetLastError();
}

}  // namespace bwr
