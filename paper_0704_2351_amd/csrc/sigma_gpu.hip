// Sigma-basis on the device: PM-Basis (the algorithm Section 2.4 relies on)
// with polynomial-matrix products through number-theoretic transforms modulo
// FFT primes c 2^k + 1 and the Chinese remainder theorem (Section 2.4), and
// M-Basis leaves, all stream-ordered so that the recursion never waits on
// the host.
//
// Layouts: a polynomial matrix is [row][col][coef] (each entry contiguous),
// residues uint32.  Transform buffers are [prime][poly][N].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include "sigma_gpu.h"

namespace bwr {

namespace {

constexpr int TPB = 256;
constexpr int LDS_LOG = 12;  // transform segments of 4096 points live in LDS

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
    uint32_t qt = __umulhi(a, wp);
    uint32_t r = a * w - qt * q;
    return r >= q ? r - q : r;
}

__device__ __forceinline__ uint32_t addq(uint32_t a, uint32_t b, uint32_t q) {
    uint32_t s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ uint32_t subq(uint32_t a, uint32_t b, uint32_t q) { return a >= b ? a - b : a + q - b; }

// Montgomery arithmetic modulo an odd p < 2^31 (R = 2^32), for short inverse chains.
struct Mont {
    uint32_t p, pinv_neg, r2;  // -p^-1 mod 2^32, R^2 mod p
};

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, const Mont& M) {
    const uint64_t t = (uint64_t)a * b;
    const uint32_t m = (uint32_t)t * M.pinv_neg;
    const uint64_t u = (t + (uint64_t)m * M.p) >> 32;
    return u >= M.p ? (uint32_t)(u - M.p) : (uint32_t)u;
}

// a^-1 mod p by Fermat's little theorem, in Montgomery form internally
__device__ __forceinline__ uint32_t mont_inv(uint32_t a, const Mont& M) {
    uint32_t x = mont_mul(a, M.r2, M);  // a R
    uint32_t r = mont_mul(1u, M.r2, M);  // R
    uint32_t e = M.p - 2;
    while (e) {
        if (e & 1) r = mont_mul(r, x, M);
        x = mont_mul(x, x, M);
        e >>= 1;
    }
    return mont_mul(r, 1u, M);
}

__device__ __forceinline__ uint32_t shoup_pre_dev(uint32_t w, uint32_t p) {
    return (uint32_t)(((uint64_t)w << 32) / p);
}

// ------------------------------------------------------------------ loading into transform buffers
// dst[t][b][x] = src_b[x] mod q_t for x < len, 0 for len <= x < N.  Polynomial b of a
// matrix with `len` coefficients per entry starts at src + b * ld.
__global__ __launch_bounds__(TPB) void k_load_polys(const uint32_t* __restrict__ src, int64_t ld, int64_t len,
                                                    int64_t off, int nb, int64_t N, int T, NttConsts c,
                                                    uint32_t* __restrict__ dst) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    int64_t total = (int64_t)T * nb * N;
    if (idx >= total) return;
    int64_t x = idx % N;
    int64_t b = (idx / N) % nb;
    int t = (int)(idx / (N * nb));
    uint32_t v = 0;
    if (x < len) {
        v = src[b * ld + off + x];
        uint32_t q = c.q[t];
        v = v >= q ? v - q : v;
    }
    dst[idx] = v;
}

// ------------------------------------------------------------------ NTT stages
// Forward: decimation in frequency (natural in, bit-reversed out).
// One radix-2 stage with butterfly span `half` over global memory.
__global__ __launch_bounds__(TPB) void k_dif_stage(uint32_t* __restrict__ a, int64_t N, int64_t half, int nb, int T,
                                                   NttConsts c, const uint32_t* __restrict__ tw) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    int64_t per = N >> 1;
    int64_t total = (int64_t)T * nb * per;
    if (idx >= total) return;
    int64_t bf = idx % per;
    int64_t poly = idx / per;
    int t = (int)(poly / nb);
    uint32_t q = c.q[t];
    const uint32_t* w = tw + (size_t)t * c.tw_stride * 2;
    int64_t blk = bf / half, j = bf % half;
    uint32_t* x = a + poly * N + blk * 2 * half + j;
    uint32_t u = x[0], v = x[half];
    x[0] = addq(u, v, q);
    x[half] = mul_shoup(subq(u, v, q), w[half + j], w[c.tw_stride + half + j], q);
}

// Inverse: decimation in time (bit-reversed in, natural out), one stage.
__global__ __launch_bounds__(TPB) void k_dit_stage(uint32_t* __restrict__ a, int64_t N, int64_t half, int nb, int T,
                                                   NttConsts c, const uint32_t* __restrict__ itw) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    int64_t per = N >> 1;
    int64_t total = (int64_t)T * nb * per;
    if (idx >= total) return;
    int64_t bf = idx % per;
    int64_t poly = idx / per;
    int t = (int)(poly / nb);
    uint32_t q = c.q[t];
    const uint32_t* w = itw + (size_t)t * c.tw_stride * 2;
    int64_t blk = bf / half, j = bf % half;
    uint32_t* x = a + poly * N + blk * 2 * half + j;
    uint32_t u = x[0];
    uint32_t v = mul_shoup(x[half], w[half + j], w[c.tw_stride + half + j], q);
    x[0] = addq(u, v, q);
    x[half] = subq(u, v, q);
}

// The stages whose butterflies stay inside contiguous segments of S = 2^sl
// points, done in LDS: forward runs spans S/2 .. 1, inverse runs 1 .. S/2.
template <bool FORWARD>
__global__ __launch_bounds__(TPB) void k_ntt_lds(uint32_t* __restrict__ a, int64_t N, int sl, int nb, int T,
                                                 NttConsts c, const uint32_t* __restrict__ tw) {
    __shared__ uint32_t sh[1 << LDS_LOG];
    const int S = 1 << sl;
    const int64_t segs_per_poly = N >> sl;
    const int64_t seg = blockIdx.x;
    const int64_t poly = seg / segs_per_poly;
    const int t = (int)(poly / nb);
    const uint32_t q = c.q[t];
    const uint32_t* w = tw + (size_t)t * c.tw_stride * 2;
    uint32_t* base = a + poly * N + (seg % segs_per_poly) * S;
    for (int i = threadIdx.x; i < S; i += TPB) sh[i] = base[i];
    __syncthreads();
    for (int st = 0; st < sl; ++st) {
        const int half = FORWARD ? (S >> 1) >> st : 1 << st;
        for (int bf = threadIdx.x; bf < (S >> 1); bf += TPB) {
            const int blk = bf / half, j = bf % half;
            const int i0 = blk * 2 * half + j;
            uint32_t u = sh[i0], v = sh[i0 + half];
            if (FORWARD) {
                sh[i0] = addq(u, v, q);
                sh[i0 + half] = mul_shoup(subq(u, v, q), w[half + j], w[c.tw_stride + half + j], q);
            } else {
                v = mul_shoup(v, w[half + j], w[c.tw_stride + half + j], q);
                sh[i0] = addq(u, v, q);
                sh[i0 + half] = subq(u, v, q);
            }
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < S; i += TPB) base[i] = sh[i];
}

// ------------------------------------------------------------------ pointwise products
// C[t][i][l][x] = sum_j A[t][i][j][x] B[t][j][l][x] mod q_t; a thread owns (t, i, 8 columns, x).
constexpr int PW_COLS = 8;

__global__ __launch_bounds__(TPB) void k_pointwise(const uint32_t* __restrict__ A, const uint32_t* __restrict__ B,
                                                   uint32_t* __restrict__ C, int r, int k, int c, int64_t N, int T,
                                                   NttConsts cs) {
    const int cgroups = (c + PW_COLS - 1) / PW_COLS;
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    int64_t total = (int64_t)T * r * cgroups * N;
    if (idx >= total) return;
    int64_t x = idx % N;
    int64_t rest = idx / N;
    int lg = (int)(rest % cgroups);
    rest /= cgroups;
    int i = (int)(rest % r);
    int t = (int)(rest / r);
    const uint32_t q = cs.q[t];
    const ModP mq = cs.mq[t];
    const uint32_t* At = A + (size_t)t * r * k * N;
    const uint32_t* Bt = B + (size_t)t * k * c * N;
    uint64_t lo[PW_COLS], hi[PW_COLS];
#pragma unroll
    for (int u = 0; u < PW_COLS; ++u) lo[u] = hi[u] = 0;
    const int l0 = lg * PW_COLS;
    for (int j = 0; j < k; ++j) {
        const uint64_t a = At[((size_t)i * k + j) * N + x];
        if (!a) continue;
#pragma unroll
        for (int u = 0; u < PW_COLS; ++u) {
            if (l0 + u < c) {
                uint64_t pr = a * Bt[((size_t)j * c + l0 + u) * N + x];
                lo[u] += pr & 0xffffffffu;
                hi[u] += pr >> 32;
            }
        }
    }
    const uint32_t r32 = cs.r32[t];
#pragma unroll
    for (int u = 0; u < PW_COLS; ++u)
        if (l0 + u < c)
            C[((size_t)t * r * c + (size_t)i * c + l0 + u) * N + x] =
                addq(red64(mq, lo[u]), mulmod(mq, red64(mq, hi[u]), r32), q);
    (void)q;
}

// ------------------------------------------------------------------ CRT
// out[e][x - lo] for x in [lo, hi): residues scaled by N^-1 mod q_t, Garner, then mod p.
__global__ __launch_bounds__(TPB) void k_crt(const uint32_t* __restrict__ C, int npoly, int64_t N, int64_t lo,
                                             int64_t W, int T, NttConsts cs, ModP mp, uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)npoly * W) return;
    int64_t e = idx / W, x = idx % W + lo;
    uint32_t a[3];
    for (int t = 0; t < T; ++t) {
        uint32_t v = C[((size_t)t * npoly + e) * N + x];
        a[t] = mul_shoup(v, cs.ninv[t], cs.ninvp[t], cs.q[t]);
    }
    uint32_t v;
    if (T == 1) {
        v = red32(mp, a[0]);
    } else {
        const uint32_t q0 = cs.q[0], q1 = cs.q[1];
        uint32_t a0m1 = a[0] >= q1 ? a[0] - q1 : a[0];
        uint32_t t1 = mulmod(cs.mq[1], subq(a[1], a0m1, q1), cs.inv01);
        v = addmod(mp, red32(mp, a[0]), mulmod(mp, cs.q0p, red32(mp, t1)));
        if (T == 3) {
            const uint32_t q2 = cs.q[2];
            uint32_t x01 = addq(a[0] >= q2 ? a[0] - q2 : a[0], mulmod(cs.mq[2], q0 >= q2 ? q0 - q2 : q0, t1), q2);
            uint32_t t2 = mulmod(cs.mq[2], subq(a[2], x01, q2), cs.inv012);
            v = addmod(mp, v, mulmod(mp, cs.q01p, red32(mp, t2)));
        }
    }
    out[idx] = v;
}

// ------------------------------------------------------------------ schoolbook window product mod p
__global__ __launch_bounds__(TPB) void k_schoolbook(const uint32_t* __restrict__ A, int64_t lenA,
                                                    const uint32_t* __restrict__ B, int64_t lenB, int r, int k, int c,
                                                    int64_t lo, int64_t W, ModP mp, uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)r * c * W) return;
    int64_t x = idx % W + lo;
    int64_t e = idx / W;
    int i = (int)(e / c), l = (int)(e % c);
    uint64_t acc_lo = 0, acc_hi = 0;
    for (int j = 0; j < k; ++j) {
        const uint32_t* a = A + ((size_t)i * k + j) * lenA;
        const uint32_t* b = B + ((size_t)j * c + l) * lenB;
        int64_t t0 = x - (lenB - 1);
        if (t0 < 0) t0 = 0;
        int64_t t1 = x < lenA - 1 ? x : lenA - 1;
        for (int64_t t = t0; t <= t1; ++t) {
            uint64_t pr = (uint64_t)a[t] * b[x - t];
            acc_lo += pr & 0xffffffffu;
            acc_hi += pr >> 32;
        }
    }
    out[idx] = addmod(mp, red64(mp, acc_lo), mulmod(mp, red64(mp, acc_hi), red64(mp, (uint64_t)1 << 32)));
}

// ------------------------------------------------------------------ M-Basis leaf
// One workgroup: order-sigma sigma-basis of G (m x n, entries of length ldG,
// coefficients 0 .. sigma-1), starting from the shifted degrees d (device).
// P (m x m, entries of length ldP >= sigma + 1) is written; d is updated.
// The residual series R = P G mod x^sigma and P live in LDS.
//
// Each order k: rows are ranked by (shifted degree, index); repeatedly the
// lowest-ranked row not yet examined whose residual coefficient k is non-zero
// becomes a pivot on its first non-zero column, and that column is eliminated
// from every later-ranked row (the same eliminations, in the same order, as
// processing the rows one by one); then the pivot rows are multiplied by x.
constexpr int LEAF_TPB = 512;

__global__ __launch_bounds__(LEAF_TPB) void k_mbasis_leaf(const uint32_t* __restrict__ G, int64_t ldG, int m, int n,
                                                          int sigma, int64_t* __restrict__ d,
                                                          uint32_t* __restrict__ P, int64_t ldP, ModP mp, Mont mt) {
    extern __shared__ uint32_t smem[];
    const int sp = sigma + 1;
    uint32_t* R = smem;                        // [m][n][sigma]
    uint32_t* Pl = R + m * n * sigma;          // [m][m][sp]
    int* perm = (int*)(Pl + m * m * sp);       // rows by (d, index)
    int* rank_of = perm + m;
    uint32_t* fac = (uint32_t*)(rank_of + m);  // elimination factors per row
    uint32_t* facp = fac + m;                  // their Shoup constants
    int* pdeg = (int*)(facp + m);
    int* fnz = pdeg + m;                       // first non-zero column of R[r][.][k], n if none
    __shared__ int64_t dl[128];
    __shared__ int is_piv[128];
    __shared__ int s_best, s_pos;
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += LEAF_TPB) {
        dl[i] = d[i];
        pdeg[i] = 0;
    }
    for (int e = tid; e < m * n * sigma; e += LEAF_TPB) {
        int k = e % sigma, rc = e / sigma;
        R[e] = G[(size_t)rc * ldG + k];
    }
    for (int e = tid; e < m * m * sp; e += LEAF_TPB) {
        int k = e % sp, rc = e / sp;
        Pl[e] = (k == 0 && rc / m == rc % m) ? 1u : 0u;
    }
    if (tid == 0) s_best = INT_MAX;
    __syncthreads();
    for (int k = 0; k < sigma; ++k) {
        for (int i = tid; i < m; i += LEAF_TPB) {
            int rk = 0;
            for (int j = 0; j < m; ++j) rk += (dl[j] < dl[i] || (dl[j] == dl[i] && j < i)) ? 1 : 0;
            rank_of[i] = rk;
            perm[rk] = i;
            is_piv[i] = 0;
            int f = n;
            for (int cc = n - 1; cc >= 0; --cc)
                if (R[(i * n + cc) * sigma + k]) f = cc;
            fnz[i] = f;
        }
        if (tid == 0) s_pos = 0;
        __syncthreads();
        for (;;) {
            for (int r = tid; r < m; r += LEAF_TPB)
                if (rank_of[r] >= s_pos && fnz[r] < n) atomicMin(&s_best, rank_of[r]);
            __syncthreads();
            const int best = s_best;
            if (best == INT_MAX) break;
            const int q = perm[best];
            const int c = fnz[q];
            // factors of the later rows with a non-zero in the pivot column
            for (int r = tid; r < m; r += LEAF_TPB) {
                uint32_t v = rank_of[r] > best ? R[(r * n + c) * sigma + k] : 0u;
                uint32_t f = v ? mp.p - mulmod(mp, v, mont_inv(R[(q * n + c) * sigma + k], mt)) : 0u;
                fac[r] = f;
                facp[r] = f ? shoup_pre_dev(f, mp.p) : 0u;
            }
            __syncthreads();
            const int rl = sigma - k;
            for (int e = tid; e < m * n * rl; e += LEAF_TPB) {
                int r = e / (n * rl);
                uint32_t f = fac[r];
                if (!f) continue;
                int rem = e - r * n * rl;
                int cc = rem / rl, kk = k + rem % rl;
                uint32_t src = R[(q * n + cc) * sigma + kk];
                if (src)
                    R[(r * n + cc) * sigma + kk] =
                        addq(R[(r * n + cc) * sigma + kk], mul_shoup(src, f, facp[r], mp.p), mp.p);
            }
            const int pl = pdeg[q] + 1;
            for (int e = tid; e < m * m * pl; e += LEAF_TPB) {
                int r = e / (m * pl);
                uint32_t f = fac[r];
                if (!f) continue;
                int rem = e - r * m * pl;
                int cc = rem / pl, kk = rem % pl;
                uint32_t src = Pl[(q * m + cc) * sp + kk];
                if (src)
                    Pl[(r * m + cc) * sp + kk] = addq(Pl[(r * m + cc) * sp + kk], mul_shoup(src, f, facp[r], mp.p), mp.p);
            }
            __syncthreads();
            for (int r = tid; r < m; r += LEAF_TPB) {
                if (fac[r]) {
                    if (pdeg[q] > pdeg[r]) pdeg[r] = pdeg[q];
                    int f = n;
                    for (int cc = n - 1; cc >= 0; --cc)
                        if (R[(r * n + cc) * sigma + k]) f = cc;
                    fnz[r] = f;
                }
            }
            if (tid == 0) {
                is_piv[q] = 1;
                s_pos = best + 1;
                s_best = INT_MAX;
            }
            __syncthreads();
        }
        // multiply the pivot rows by x
        for (int e = tid; e < m * n; e += LEAF_TPB) {
            int r = e / n;
            if (!is_piv[r]) continue;
            uint32_t* x = R + e * sigma;
            for (int kk = sigma - 1; kk > k; --kk) x[kk] = x[kk - 1];
            x[k] = 0;
        }
        for (int e = tid; e < m * m; e += LEAF_TPB) {
            int r = e / m;
            if (!is_piv[r]) continue;
            uint32_t* x = Pl + e * sp;
            for (int kk = pdeg[r] + 1; kk > 0; --kk) x[kk] = x[kk - 1];
            x[0] = 0;
        }
        __syncthreads();
        for (int r = tid; r < m; r += LEAF_TPB)
            if (is_piv[r]) {
                pdeg[r] += 1;
                dl[r] += 1;
            }
        __syncthreads();
    }
    for (int e = tid; e < m * m * sp; e += LEAF_TPB) {
        int k = e % sp, rc = e / sp;
        P[(size_t)rc * ldP + k] = Pl[e];
    }
    for (int i = tid; i < m; i += LEAF_TPB) d[i] = dl[i];
}

// G[r][c][k] = S[k][r][c] for r < s, k < L; -1 (mod p) at r = s + c, k = 0; 0 elsewhere.
__global__ __launch_bounds__(TPB) void k_build_G(const uint32_t* __restrict__ S, int64_t L, int s, uint32_t p,
                                                 uint32_t* __restrict__ G, int64_t len) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)2 * s * s * len) return;
    int64_t k = idx % len;
    int64_t rc = idx / len;
    int r = (int)(rc / s), c = (int)(rc % s);
    uint32_t v = 0;
    if (r < s) {
        if (k < L) v = S[((size_t)k * s + r) * s + c];
    } else if (k == 0 && r - s == c) {
        v = p - 1;
    }
    G[idx] = v;
}

}  // namespace

hipError_t gpu_build_G(const uint32_t* S, int64_t L, int s, uint32_t p, uint32_t* G, int64_t len, hipStream_t st) {
    k_build_G<<<grid_for((int64_t)2 * s * s * len, TPB), TPB, 0, st>>>(S, L, s, p, G, len);
    return hipGetLastError();
}

size_t mbasis_leaf_lds(int m, int n, int sigma) {
    return sizeof(uint32_t) * ((size_t)m * n * sigma + (size_t)m * m * (sigma + 1)) + sizeof(int) * 6 * (size_t)m;
}

hipError_t gpu_load_polys(const uint32_t* src, int64_t ld, int64_t len, int64_t off, int nb, int64_t N, int T,
                          const NttConsts& c, uint32_t* dst, hipStream_t st) {
    int64_t total = (int64_t)T * nb * N;
    k_load_polys<<<grid_for(total, TPB), TPB, 0, st>>>(src, ld, len, off, nb, N, T, c, dst);
    return hipGetLastError();
}

hipError_t gpu_ntt(uint32_t* a, int lg, int nb, int T, const NttConsts& c, const uint32_t* tw, const uint32_t* itw,
                   bool forward, hipStream_t st) {
    const int64_t N = (int64_t)1 << lg;
    const int sl = lg < LDS_LOG ? lg : LDS_LOG;
    const int64_t bfl = (int64_t)T * nb * (N >> 1);
    const int64_t segs = (int64_t)T * nb * (N >> sl);
    if (forward) {
        for (int l = lg; l > sl; --l) {
            k_dif_stage<<<grid_for(bfl, TPB), TPB, 0, st>>>(a, N, (int64_t)1 << (l - 1), nb, T, c, tw);
        }
        if (sl > 0) k_ntt_lds<true><<<(unsigned)segs, TPB, 0, st>>>(a, N, sl, nb, T, c, tw);
    } else {
        if (sl > 0) k_ntt_lds<false><<<(unsigned)segs, TPB, 0, st>>>(a, N, sl, nb, T, c, itw);
        for (int l = sl + 1; l <= lg; ++l) {
            k_dit_stage<<<grid_for(bfl, TPB), TPB, 0, st>>>(a, N, (int64_t)1 << (l - 1), nb, T, c, itw);
        }
    }
    return hipGetLastError();
}

hipError_t gpu_pointwise(const uint32_t* A, const uint32_t* B, uint32_t* C, int r, int k, int c, int64_t N, int T,
                         const NttConsts& cs, hipStream_t st) {
    int64_t total = (int64_t)T * r * ((c + PW_COLS - 1) / PW_COLS) * N;
    k_pointwise<<<grid_for(total, TPB), TPB, 0, st>>>(A, B, C, r, k, c, N, T, cs);
    return hipGetLastError();
}

hipError_t gpu_crt(const uint32_t* C, int npoly, int64_t N, int64_t lo, int64_t W, int T, const NttConsts& cs,
                   ModP mp, uint32_t* out, hipStream_t st) {
    k_crt<<<grid_for((int64_t)npoly * W, TPB), TPB, 0, st>>>(C, npoly, N, lo, W, T, cs, mp, out);
    return hipGetLastError();
}

hipError_t gpu_schoolbook(const uint32_t* A, int64_t lenA, const uint32_t* B, int64_t lenB, int r, int k, int c,
                          int64_t lo, int64_t W, ModP mp, uint32_t* out, hipStream_t st) {
    k_schoolbook<<<grid_for((int64_t)r * c * W, TPB), TPB, 0, st>>>(A, lenA, B, lenB, r, k, c, lo, W, mp, out);
    return hipGetLastError();
}

hipError_t gpu_mbasis_leaf(const uint32_t* G, int64_t ldG, int m, int n, int sigma, int64_t* d, uint32_t* P,
                           int64_t ldP, ModP mp, hipStream_t st) {
    size_t lds = mbasis_leaf_lds(m, n, sigma);
    Mont mt;
    mt.p = mp.p;
    uint32_t inv = 1;  // p^-1 mod 2^32 by Newton iteration (p odd)
    for (int i = 0; i < 5; ++i) inv *= 2u - mp.p * inv;
    mt.pinv_neg = 0u - inv;
    const uint64_t r1 = ((uint64_t)1 << 32) % mp.p;
    mt.r2 = (uint32_t)((r1 * r1) % mp.p);
    k_mbasis_leaf<<<1, LEAF_TPB, lds, st>>>(G, ldG, m, n, sigma, d, P, ldP, mp, mt);
    return hipGetLastError();
}

}  // namespace bwr
