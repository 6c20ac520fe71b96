// Sigma-basis on the device: PM-Basis (the algorithm Section 2.4 relies on)
// with polynomial-matrix products through number-theoretic transforms modulo
// FFT primes c 2^k + 1 and the Chinese remainder theorem (Section 2.4), and
// M-Basis leaves, all stream-ordered so that the recursion never waits on
// the host.
//
// Layouts: a polynomial matrix is [row][col][coef] (each entry contiguous),
// residues uint32; a batch of matrices (one per target prime, same shape) is
// [batch][row][col][coef].  Transform buffers are [FFT prime][poly][N], the
// polys of a batch in batch order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>
#include <mutex>
#include <vector>

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

// ------------------------------------------------------------------ CRT
// out[e][x - lo] for x in [lo, hi): residues scaled by N^-1 mod q_t, Garner, then mod the prime of
// poly e's batch (per_batch polys each).
__global__ __launch_bounds__(TPB) void k_crt(const uint32_t* __restrict__ C, int npoly, int per_batch, int64_t N,
                                             int64_t lo, int64_t W, int T, NttConsts cs, PrimeBatch pb,
                                             uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)npoly * W) return;
    int64_t e = idx / W, x = idx % W + lo;
    const int b = (int)(e / per_batch);
    const ModP mp = pb.mp[b];
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
        v = addmod(mp, red32(mp, a[0]), mulmod(mp, cs.q0p[b], red32(mp, t1)));
        if (T == 3) {
            const uint32_t q2 = cs.q[2];
            uint32_t x01 = addq(a[0] >= q2 ? a[0] - q2 : a[0], mulmod(cs.mq[2], q0 >= q2 ? q0 - q2 : q0, t1), q2);
            uint32_t t2 = mulmod(cs.mq[2], subq(a[2], x01, q2), cs.inv012);
            v = addmod(mp, v, mulmod(mp, cs.q01p[b], red32(mp, t2)));
        }
    }
    out[idx] = v;
}

// ------------------------------------------------------------------ pointwise products
// C[t][i][l][x] = sum_j A[t][i][j][x] B[t][j][l][x] mod q_t over the transform points x, a 4 x 4 tile of
// (i, l) per thread and transform point: per inner index j the thread loads 4 values of A and 4 of B for
// 16 products, summed in 64 bits and reduced every 3 terms (3 (q - 1)^2 + q < 2^64 for q < 2^31).
constexpr int PW_TILE = 4;
__global__ __launch_bounds__(TPB) void k_pointwise_tiled(const uint32_t* __restrict__ A,
                                                         const uint32_t* __restrict__ B, uint32_t* __restrict__ C,
                                                         int r, int k, int c, int nbatch, int64_t N, int T,
                                                         NttConsts cs) {
    const int rt = (r + PW_TILE - 1) / PW_TILE, ct = (c + PW_TILE - 1) / PW_TILE;
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)T * nbatch * rt * ct * N) return;
    const int64_t x = idx % N;
    int64_t rest = idx / N;
    const int lt = (int)(rest % ct);
    rest /= ct;
    const int it = (int)(rest % rt);
    rest /= rt;
    const int b = (int)(rest % nbatch);
    const int t = (int)(rest / nbatch);
    const ModP mq = cs.mq[t];
    const uint32_t* At = A + ((size_t)t * nbatch + b) * r * k * N;
    const uint32_t* Bt = B + ((size_t)t * nbatch + b) * k * c * N;
    C += (size_t)b * r * c * N;
    const int i0 = it * PW_TILE, l0 = lt * PW_TILE;
    uint64_t acc[PW_TILE][PW_TILE];
#pragma unroll
    for (int a = 0; a < PW_TILE; ++a)
#pragma unroll
        for (int b = 0; b < PW_TILE; ++b) acc[a][b] = 0;
    int pending = 0;
    for (int j = 0; j < k; ++j) {
        uint64_t av[PW_TILE], bv[PW_TILE];
#pragma unroll
        for (int a = 0; a < PW_TILE; ++a) av[a] = i0 + a < r ? At[((size_t)(i0 + a) * k + j) * N + x] : 0u;
#pragma unroll
        for (int b = 0; b < PW_TILE; ++b) bv[b] = l0 + b < c ? Bt[((size_t)j * c + l0 + b) * N + x] : 0u;
#pragma unroll
        for (int a = 0; a < PW_TILE; ++a)
#pragma unroll
            for (int b = 0; b < PW_TILE; ++b) acc[a][b] += av[a] * bv[b];
        if (++pending == 3) {
            pending = 0;
#pragma unroll
            for (int a = 0; a < PW_TILE; ++a)
#pragma unroll
                for (int b = 0; b < PW_TILE; ++b) acc[a][b] = red64(mq, acc[a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < PW_TILE; ++a)
#pragma unroll
        for (int b = 0; b < PW_TILE; ++b)
            if (i0 + a < r && l0 + b < c)
                C[((size_t)t * nbatch * r * c + (size_t)(i0 + a) * c + l0 + b) * N + x] = red64(mq, acc[a][b]);
}

// ------------------------------------------------------------------ schoolbook window product mod p
__global__ __launch_bounds__(TPB) void k_schoolbook(const uint32_t* __restrict__ A, int64_t lenA,
                                                    const uint32_t* __restrict__ B, int64_t lenB, int r, int k, int c,
                                                    int64_t lo, int64_t W, PrimeBatch pb,
                                                    uint32_t* __restrict__ out) {
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)pb.n * r * c * W) return;
    int64_t x = idx % W + lo;
    int64_t e = idx / W;
    const int bt = (int)(e / ((int64_t)r * c));
    e %= (int64_t)r * c;
    const ModP mp = pb.mp[bt];
    A += (size_t)bt * r * k * lenA;
    B += (size_t)bt * k * c * lenB;
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

// Schoolbook window product with the operands in LDS: one workgroup per (output row i, group of SB_COLS
// output columns) loads A[i][.] and B[.][columns] once, then each thread forms output coefficients from LDS.
constexpr int SB_COLS = 8;
__global__ __launch_bounds__(TPB) void k_schoolbook_lds(const uint32_t* __restrict__ A, int64_t lenA,
                                                        const uint32_t* __restrict__ B, int64_t lenB, int r, int k,
                                                        int c, int64_t lo, int64_t W, PrimeBatch pb,
                                                        uint32_t* __restrict__ out) {
    extern __shared__ uint32_t lds[];
    const int groups = (c + SB_COLS - 1) / SB_COLS;
    const int bt = (int)(blockIdx.x / ((unsigned)r * groups));
    const int blk = (int)(blockIdx.x % ((unsigned)r * groups));
    const ModP mp = pb.mp[bt];
    A += (size_t)bt * r * k * lenA;
    B += (size_t)bt * k * c * lenB;
    out += (size_t)bt * r * c * W;
    const int i = blk / groups, l0 = (blk % groups) * SB_COLS;
    const int nl = c - l0 < SB_COLS ? c - l0 : SB_COLS;
    uint32_t* As = lds;                      // [k][lenA]
    uint32_t* Bs = lds + (size_t)k * lenA;   // [k][nl][lenB]
    for (int64_t e = threadIdx.x; e < (int64_t)k * lenA; e += TPB) As[e] = A[(size_t)i * k * lenA + e];
    for (int64_t e = threadIdx.x; e < (int64_t)k * nl * lenB; e += TPB) {
        const int64_t j = e / (nl * lenB), rem = e % (nl * lenB);
        Bs[e] = B[((size_t)j * c + l0) * lenB + rem];
    }
    __syncthreads();
    const uint32_t r32 = red64(mp, (uint64_t)1 << 32);
    for (int64_t o = threadIdx.x; o < (int64_t)nl * W; o += TPB) {
        const int l = (int)(o / W);
        const int64_t x = o % W + lo;
        int64_t t0 = x - (lenB - 1);
        if (t0 < 0) t0 = 0;
        const int64_t t1 = x < lenA - 1 ? x : lenA - 1;
        uint64_t acc_lo = 0, acc_hi = 0;
        for (int j = 0; j < k; ++j) {
            const uint32_t* a = As + (size_t)j * lenA;
            const uint32_t* b = Bs + ((size_t)j * nl + l) * lenB;
            for (int64_t t = t0; t <= t1; ++t) {
                const uint64_t pr = (uint64_t)a[t] * b[x - t];
                acc_lo += pr & 0xffffffffu;
                acc_hi += pr >> 32;
            }
        }
        out[((size_t)i * c + l0 + l) * W + (x - lo)] = addmod(mp, red64(mp, acc_lo), mulmod(mp, red64(mp, acc_hi), r32));
    }
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

__global__ __launch_bounds__(LEAF_TPB) void k_mbasis_leaf(const uint32_t* __restrict__ G, int64_t ldG, int64_t gbs,
                                                          int m, int n, int sigma, int64_t* __restrict__ d,
                                                          uint32_t* __restrict__ P, int64_t ldP, int64_t pbs,
                                                          PrimeBatch pb) {
    extern __shared__ uint32_t smem[];
    // batch element of this workgroup: its matrices, degrees and prime
    const ModP mp = pb.mp[blockIdx.x];
    G += blockIdx.x * gbs;
    P += blockIdx.x * pbs;
    d += (int64_t)blockIdx.x * m;
    Mont mt;
    mt.p = mp.p;
    {
        uint32_t inv = 1;  // p^-1 mod 2^32 by Newton iteration (p odd)
        for (int i = 0; i < 5; ++i) inv *= 2u - mp.p * inv;
        mt.pinv_neg = 0u - inv;
        const uint32_t r1 = (uint32_t)((((uint64_t)1) << 32) % mp.p);
        mt.r2 = mulmod(mp, r1, r1);
    }
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

// ------------------------------------------------------------------ M-Basis leaf, one transform per order
// The same basis as k_mbasis_leaf, organised for fewer passes over LDS.  At
// order k only the residual coefficient E = R[., ., k] (m x n) decides the
// pivots, so the eliminations run on E alone while their row operations are
// collected in an m x m matrix T; one parallel pass then applies T (and the
// multiplication of the pivot rows by x) to the rest of the residual window
// and to P.  The eliminations are fraction-free: a row eliminated by pivot
// value v is multiplied by v instead of dividing the pivot row by v, so no
// inverse is needed inside the loop.  Every row of the result is then its
// exact counterpart times the product lambda of the pivot values that
// touched it (the zero pattern, hence every pivot choice and degree, is the
// same); lambda is tracked per row and divided out once when the leaf ends,
// so the output equals the eager per-pivot elimination entry for entry.
//
// Phase A (the waves holding T columns; each repeats the E elimination): lane
// (row r = lane / LPRW, part = lane % LPRW) keeps columns part + LPRW i of its
// row of E and T in registers.  Values of the pivot row come through
// v_readlane (its lanes are known to the whole wave); the pivot-column value
// of the lane's own row comes from a DPP broadcast inside its lane group.
// Phase B (all threads): one thread per output column (c, kk) of the residual
// window (orders k+1 .. sigma-1) or of P (degrees 0 .. k+1) loads the m
// entries of that column and of the column before it once, then forms every
// row r of T times the (shifted, for pivot rows) column with double-precision
// FMAs; all products and sums stay below 2^53, so they are exact (residues of
// large primes are split into 16-bit halves first).
constexpr int LEAF2_TPB = 512;

template <int M>
struct LeafLanes {
    static constexpr int q = 64 / M;
    static constexpr int LPRW = q >= 32 ? 32 : q >= 16 ? 16 : q >= 8 ? 8 : q >= 4 ? 4 : q >= 2 ? 2 : 1;
};

// x mod p for 0 <= x < 2^53 held exactly in a double
__device__ __forceinline__ uint32_t dmod(double x, double pd, double pinv) {
    double q = floor(x * pinv);
    double r = fma(-q, pd, x);
    if (r < 0) r += pd;
    if (r >= pd) r -= pd;
    return (uint32_t)r;
}

// (u * a + v * b) mod p for residues, in exact double arithmetic: products of
// residues below 2^16 fit directly; larger residues a, b are split into 16-bit
// halves so that every partial sum stays below 2^53.
template <bool SMALLP>
__device__ __forceinline__ uint32_t comb2(uint32_t u, uint32_t a, uint32_t v, uint32_t b, double pd, double pinv) {
    if (SMALLP) return dmod(fma((double)u, (double)a, (double)v * (double)b), pd, pinv);
    const double du = (double)u, dv = (double)v;
    const double hi = fma(du, (double)(a >> 16), dv * (double)(b >> 16));        // < 2^48
    const double lo = fma(du, (double)(a & 0xffffu), dv * (double)(b & 0xffffu));  // < 2^48
    return dmod(fma((double)dmod(hi, pd, pinv), 65536.0, (double)dmod(lo, pd, pinv)), pd, pinv);
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// value of lane (lane / LPRW) * LPRW + sp (the same group of LPRW lanes)
template <int LPRW>
__device__ __forceinline__ uint32_t group_bcast(uint32_t v, int sp) {
    if constexpr (LPRW == 1) {
        return v;
    } else if constexpr (LPRW == 2) {
        return sp == 0 ? (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xA0, 0xF, 0xF, false)
                       : (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xF5, 0xF, 0xF, false);
    } else if constexpr (LPRW == 4) {
        switch (sp) {
            case 0: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x00, 0xF, 0xF, false);
            case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x55, 0xF, 0xF, false);
            case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xAA, 0xF, 0xF, false);
            default: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xFF, 0xF, 0xF, false);
        }
    } else {
        const int lane = (int)(threadIdx.x & 63);
        return (uint32_t)__shfl((int)v, (lane / LPRW) * LPRW + sp, 64);
    }
}

template <int S, bool SMALLP>
__global__ __launch_bounds__(LEAF2_TPB) void k_mbasis_leaf2(const uint32_t* __restrict__ G, int64_t ldG, int64_t gbs,
                                                           int sigma, int64_t* __restrict__ d,
                                                           uint32_t* __restrict__ P, int64_t ldP, int64_t pbs,
                                                           PrimeBatch pb) {
    constexpr int M = 2 * S, N = S;
    // batch element of this workgroup: its matrices, degrees and prime
    const ModP mp = pb.mp[blockIdx.x];
    G += blockIdx.x * gbs;
    P += blockIdx.x * pbs;
    d += (int64_t)blockIdx.x * M;
    constexpr int LPRW = LeafLanes<M>::LPRW;
    constexpr int EC = (N + LPRW - 1) / LPRW;       // E columns per lane
    constexpr int TS = (M + LPRW - 1) / LPRW;       // T column slots per row
    constexpr int NWA = TS < LEAF2_TPB / 64 ? TS : LEAF2_TPB / 64;  // waves of phase A
    constexpr int TSW = (TS + NWA - 1) / NWA;       // T slots per lane of a phase-A wave
    extern __shared__ uint32_t smem[];
    const int sp = sigma + 1;
    // ping-pong buffers by offset from the LDS base (an array of pointers would lose the LDS address space)
    const int RS = M * N * sigma, PS = M * M * sp;
    __shared__ double Td[M * M];
    __shared__ uint32_t lamS[M], linv[M];
    __shared__ int pv[M];
    __shared__ int64_t dl[M];
    const int tid = threadIdx.x;
    const double pd = (double)mp.p, pinv = 1.0 / (double)mp.p;
    for (int i = tid; i < M; i += LEAF2_TPB) {
        dl[i] = d[i];
        lamS[i] = 1u;
    }
    for (int e = tid; e < M * N * sigma; e += LEAF2_TPB) {
        const int k = e % sigma, rc = e / sigma;
        smem[e] = G[(size_t)rc * ldG + k];
    }
    for (int e = tid; e < 2 * M * M * sp; e += LEAF2_TPB) {
        const int k = e % sp, rc = (e / sp) % (M * M);
        smem[2 * RS + e] = (e < PS && k == 0 && rc / M == rc % M) ? 1u : 0u;  // P0 = I, P1 = 0
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    for (int k = 0; k < sigma; ++k) {
        const uint32_t* Rc = smem + (k & 1) * RS;
        uint32_t* Rn = smem + ((k + 1) & 1) * RS;
        const uint32_t* Pc = smem + 2 * RS + (k & 1) * PS;
        uint32_t* Pn = smem + 2 * RS + ((k + 1) & 1) * PS;
        if (wave < NWA) {
            const int r = lane / LPRW, part = lane % LPRW;
            const bool valid = r < M;
            const int rr = valid ? r : 0;
            uint32_t e[EC], t[TSW];
#pragma unroll
            for (int i = 0; i < EC; ++i) {
                const int col = part + LPRW * i;
                e[i] = (valid && col < N) ? Rc[(rr * N + col) * sigma + k] : 0u;
            }
#pragma unroll
            for (int u = 0; u < TSW; ++u) {
                const int j = part + LPRW * (wave + NWA * u);
                t[u] = (valid && j == r) ? 1u : 0u;
            }
            int rk = 0;
            const int64_t dr = dl[rr];
            for (int j = 0; j < M; ++j) rk += (dl[j] < dr || (dl[j] == dr && j < rr)) ? 1 : 0;
            uint32_t lam = 1u;
            int isp = 0;
            for (int pos = 0; pos < M; ++pos) {
                const uint64_t bal = __ballot(valid && part == 0 && rk == pos);
                if (bal == 0) continue;  // every rank is taken by exactly one row
                const int ql = (int)__ffsll((unsigned long long)bal) - 1;  // first lane of the row at pos
                uint32_t mk = 0;
#pragma unroll
                for (int i = 0; i < EC; ++i) {
                    const int col = part + LPRW * i;
                    if (col < N && e[i]) mk |= 1u << col;
                }
                uint32_t mq = 0;
#pragma unroll
                for (int x = 0; x < LPRW; ++x) mq |= readlane_u32(mk, ql + x);
                if (mq == 0) continue;
                const int c = __ffs(mq) - 1;
                const int slot = c / LPRW, spart = c % LPRW;
                uint32_t sel = 0;
#pragma unroll
                for (int i = 0; i < EC; ++i)
                    if (i == slot) sel = e[i];
                const uint32_t piv = readlane_u32(sel, ql + spart);
                const uint32_t fr = group_bcast<LPRW>(sel, spart);
                const bool elim = valid && rk > pos && fr != 0u;
                const uint32_t fneg = fr ? mp.p - fr : 0u;  // eliminated row: piv * row - fr * pivot row
                // pivot-row values at this lane's columns, then every update at once (no branches,
                // so the independent chains interleave)
                uint32_t qe[EC], qt[TSW];
#pragma unroll
                for (int i = 0; i < EC; ++i) {
                    qe[i] = 0;
#pragma unroll
                    for (int x = 0; x < LPRW; ++x) {
                        const uint32_t v = readlane_u32(e[i], ql + x);
                        qe[i] = part == x ? v : qe[i];
                    }
                }
#pragma unroll
                for (int u = 0; u < TSW; ++u) {
                    qt[u] = 0;
#pragma unroll
                    for (int x = 0; x < LPRW; ++x) {
                        const uint32_t v = readlane_u32(t[u], ql + x);
                        qt[u] = part == x ? v : qt[u];
                    }
                }
#pragma unroll
                for (int i = 0; i < EC; ++i) {
                    const uint32_t nv = comb2<SMALLP>(piv, e[i], fneg, qe[i], pd, pinv);
                    e[i] = elim ? nv : e[i];
                }
#pragma unroll
                for (int u = 0; u < TSW; ++u) {
                    const uint32_t nv = comb2<SMALLP>(piv, t[u], fneg, qt[u], pd, pinv);
                    t[u] = elim ? nv : t[u];
                }
                {
                    const uint32_t nv = comb2<SMALLP>(piv, lam, 0u, 0u, pd, pinv);
                    lam = elim ? nv : lam;
                }
                if (lane == ql) isp = 1;
            }
            if (valid) {
#pragma unroll
                for (int u = 0; u < TSW; ++u) {
                    const int j = part + LPRW * (wave + NWA * u);
                    if (j < M && wave + NWA * u < TS) Td[r * M + j] = (double)t[u];
                }
                if (wave == 0 && part == 0) {
                    pv[r] = isp;
                    lamS[r] = mulmod(mp, lamS[r], lam);
                }
            }
        }
        __syncthreads();
        // phase B: one thread per input column kk' of the residual window
        // (orders k .. sigma-1) or of P (degrees 0 .. k): Y[r] = sum_j T[r][j] X[j][kk'],
        // stored at order kk' + 1 for pivot rows (multiplied by x), kk' otherwise.
        const int nkR = sigma - k;   // residual inputs k .. sigma-1
        const int nkP = k + 1;       // P inputs 0 .. k (degree <= k after k orders)
        const int nR = N * nkR, nP = M * nkP;
        // rows of a column split over two threads when that fills the block better
        const int rsplit = (nR + nP) * 2 <= LEAF2_TPB + LEAF2_TPB / 2 ? 2 : 1;
        const int rows_per = M / rsplit;
        for (int w = tid; w < (nR + nP) * rsplit; w += LEAF2_TPB) {
            const int idx = w / rsplit, r0 = (w % rsplit) * rows_per;
            const bool isR = idx < nR;
            int c, kq;
            if (isR) {
                c = idx / nkR;
                kq = k + idx % nkR;
            } else {
                c = (idx - nR) / nkP;
                kq = (idx - nR) % nkP;
            }
            const uint32_t* src = isR ? Rc + c * sigma + kq : Pc + c * sp + kq;
            uint32_t* dst = isR ? Rn + c * sigma + kq : Pn + c * sp + kq;
            const int ld = isR ? N * sigma : M * sp;  // stride between rows
            const int lim = isR ? sigma : sp;         // first order past the buffer
            double xh[M], xl[SMALLP ? 1 : M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const uint32_t a = src[j * ld];
                if (SMALLP) {
                    xh[j] = (double)a;
                } else {
                    xh[j] = (double)(a >> 16);
                    xl[j] = (double)(a & 0xffffu);
                }
            }
#pragma unroll 4
            for (int r = r0; r < r0 + rows_per; ++r) {
                const double* tr = Td + r * M;
                double ah = 0.0, al = 0.0;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    ah = fma(tr[j], xh[j], ah);
                    if (!SMALLP) al = fma(tr[j], xl[j], al);
                }
                uint32_t v;
                if (SMALLP) {
                    v = dmod(ah, pd, pinv);
                } else {
                    v = dmod(fma((double)dmod(ah, pd, pinv), 65536.0, (double)dmod(al, pd, pinv)), pd, pinv);
                }
                const int sh = pv[r];
                if (kq + sh < lim && (isR ? kq + sh > k : true)) dst[r * ld + sh] = v;
                if (!isR && sh && kq == 0) dst[r * ld] = 0u;  // a pivot row has no constant term
            }
        }
        for (int i = tid; i < M; i += LEAF2_TPB) dl[i] += pv[i];
        __syncthreads();
    }
    for (int i = tid; i < M; i += LEAF2_TPB) {
        linv[i] = invmod(mp, lamS[i]);
        d[i] = dl[i];
    }
    __syncthreads();
    const uint32_t* Pf = smem + 2 * RS + (sigma & 1) * PS;
    for (int e = tid; e < M * M * sp; e += LEAF2_TPB) {
        const int k = e % sp, rc = e / sp;
        P[(size_t)rc * ldP + k] = mulmod(mp, Pf[e], linv[rc / M]);
    }
}

// G[r][c][k] = S[k][r][c] for r < s, k < L; -1 (mod p) at r = s + c, k = 0; 0 elsewhere;
// written for the coefficients k0 <= k < k1 of every entry.
__global__ __launch_bounds__(TPB) void k_build_G(const uint32_t* __restrict__ S, int64_t L, int s, uint32_t p,
                                                 uint32_t* __restrict__ G, int64_t len, int64_t k0, int64_t k1) {
    const int64_t span = k1 - k0;
    int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= (int64_t)2 * s * s * span) return;
    int64_t k = k0 + idx % span;
    int64_t rc = idx / span;
    int r = (int)(rc / s), c = (int)(rc % s);
    uint32_t v = 0;
    if (r < s) {
        if (k < L) v = S[((size_t)k * s + r) * s + c];
    } else if (k == 0 && r - s == c) {
        v = p - 1;
    }
    G[rc * len + k] = v;
}

// dst[r * dld + x] = src[r * sld + x] for x < width, r < nrows (strided copies as plain loads and stores)
__global__ __launch_bounds__(TPB) void k_copy_rows(uint32_t* __restrict__ dst, int64_t dld, const uint32_t* __restrict__ src,
                                                   int64_t sld, int64_t width, int64_t nrows) {
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    if (idx >= width * nrows) return;
    const int64_t r = idx / width, x = idx % width;
    dst[r * dld + x] = src[r * sld + x];
}

// Generator rows: out[(i * s + c) * olen + k] = P[(rows[i] * m + c) * ld + k] for k <= delta_i (zero above),
// and bad = 1 if any coefficient of those entries above delta_i (up to len) is non-zero.
__global__ __launch_bounds__(TPB) void k_extract_rows(const uint32_t* __restrict__ P, int64_t ld, int64_t len, int m,
                                                      int s, GenRows gr, int64_t olen, uint32_t* __restrict__ out,
                                                      int32_t* __restrict__ bad) {
    const int64_t idx = (int64_t)blockIdx.x * TPB + threadIdx.x;
    const int64_t span = len > olen ? len : olen;
    if (idx >= (int64_t)s * s * span) return;
    const int64_t k = idx % span;
    const int e = (int)(idx / span), i = e / s, c = e % s;
    const uint32_t v = k < len ? P[((int64_t)gr.row[i] * m + c) * ld + k] : 0u;
    if (k < olen) out[(int64_t)e * olen + k] = k <= gr.delta[i] ? v : 0u;
    if (k > gr.delta[i] && v) atomicOr(bad, 1);
}

}  // namespace

hipError_t gpu_copy_rows(uint32_t* dst, int64_t dld, const uint32_t* src, int64_t sld, int64_t width, int64_t nrows,
                         hipStream_t st) {
    if (width <= 0 || nrows <= 0) return hipSuccess;
    k_copy_rows<<<grid_for(width * nrows, TPB), TPB, 0, st>>>(dst, dld, src, sld, width, nrows);
    return hipGetLastError();
}

hipError_t gpu_extract_rows(const uint32_t* P, int64_t ld, int64_t len, int m, int s, const GenRows& gr, int64_t olen,
                            uint32_t* out, int32_t* bad, hipStream_t st) {
    const int64_t span = len > olen ? len : olen;
    if (s <= 0 || span <= 0) return hipSuccess;
    k_extract_rows<<<grid_for((int64_t)s * s * span, TPB), TPB, 0, st>>>(P, ld, len, m, s, gr, olen, out, bad);
    return hipGetLastError();
}

namespace {

}  // namespace

hipError_t gpu_build_G(const uint32_t* S, int64_t L, int s, uint32_t p, uint32_t* G, int64_t len, int64_t k0,
                       int64_t k1, hipStream_t st) {
    if (k0 < 0 || k1 > len || k0 >= k1) return k0 == k1 ? hipSuccess : hipErrorInvalidValue;
    k_build_G<<<grid_for((int64_t)2 * s * s * (k1 - k0), TPB), TPB, 0, st>>>(S, L, s, p, G, len, k0, k1);
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

hipError_t gpu_pointwise(const uint32_t* A, const uint32_t* B, uint32_t* C, int r, int k, int c, int nbatch,
                         int64_t N, int T, const NttConsts& cs, hipStream_t st) {
    const int64_t tiles =
        (int64_t)T * nbatch * ((r + PW_TILE - 1) / PW_TILE) * ((c + PW_TILE - 1) / PW_TILE) * N;
    k_pointwise_tiled<<<grid_for(tiles, TPB), TPB, 0, st>>>(A, B, C, r, k, c, nbatch, N, T, cs);
    return hipGetLastError();
}

hipError_t gpu_crt(const uint32_t* C, int npoly, int per_batch, int64_t N, int64_t lo, int64_t W, int T,
                   const NttConsts& cs, const PrimeBatch& pb, uint32_t* out, hipStream_t st) {
    if (per_batch < 1 || npoly > per_batch * pb.n) return hipErrorInvalidValue;
    k_crt<<<grid_for((int64_t)npoly * W, TPB), TPB, 0, st>>>(C, npoly, per_batch, N, lo, W, T, cs, pb, out);
    return hipGetLastError();
}

hipError_t gpu_schoolbook(const uint32_t* A, int64_t lenA, const uint32_t* B, int64_t lenB, int r, int k, int c,
                          int64_t lo, int64_t W, const PrimeBatch& pb, uint32_t* out, hipStream_t st) {
    if (pb.n < 1 || pb.n > SIGMA_BATCH_MAX) return hipErrorInvalidValue;
    const int nl = c < SB_COLS ? c : SB_COLS;
    const size_t lds = sizeof(uint32_t) * ((size_t)k * lenA + (size_t)k * nl * lenB);
    if (lds <= 48 * 1024 && r > 0 && c > 0 && W > 0) {
        const unsigned grid = (unsigned)pb.n * (unsigned)r * (unsigned)((c + SB_COLS - 1) / SB_COLS);
        k_schoolbook_lds<<<grid, TPB, lds, st>>>(A, lenA, B, lenB, r, k, c, lo, W, pb, out);
        return hipGetLastError();
    }
    k_schoolbook<<<grid_for((int64_t)pb.n * r * c * W, TPB), TPB, 0, st>>>(A, lenA, B, lenB, r, k, c, lo, W, pb, out);
    return hipGetLastError();
}

size_t mbasis_leaf2_lds(int m, int n, int sigma) {
    return sizeof(uint32_t) * (2 * (size_t)m * n * sigma + 2 * (size_t)m * m * (sigma + 1));
}

namespace {

// Raises the kernel's dynamic-LDS limit to at least lds on the current device.  The limit only grows, under a
// lock, so that threads launching leaves of different orders side by side never lower it below what another
// thread's launch needs.
template <int S, bool SMALLP>
hipError_t leaf2_allow_lds(size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    static std::mutex mu;
    static std::vector<size_t> allowed;  // per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)allowed.size() <= dev) allowed.resize(dev + 1, 0);
    if (lds <= allowed[dev]) return hipSuccess;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mbasis_leaf2<S, SMALLP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) allowed[dev] = lds;
    return e;
}

template <int S, bool SMALLP>
hipError_t leaf2_launch(const uint32_t* G, int64_t ldG, int64_t gbs, int sigma, int64_t* d, uint32_t* P, int64_t ldP,
                        int64_t pbs, const PrimeBatch& pb, hipStream_t st) {
    const size_t lds = mbasis_leaf2_lds(2 * S, S, sigma);
    hipError_t e = leaf2_allow_lds<S, SMALLP>(lds);
    if (e != hipSuccess) return e;
    k_mbasis_leaf2<S, SMALLP><<<(unsigned)pb.n, LEAF2_TPB, lds, st>>>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb);
    return hipGetLastError();
}

template <int S>
hipError_t leaf2_s(const uint32_t* G, int64_t ldG, int64_t gbs, int sigma, int64_t* d, uint32_t* P, int64_t ldP,
                   int64_t pbs, const PrimeBatch& pb, hipStream_t st) {
    if (pb.small()) return leaf2_launch<S, true>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
    if (pb.large()) return leaf2_launch<S, false>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
    return hipErrorInvalidValue;  // a batch is all 16-bit primes or all larger ones
}

}  // namespace

hipError_t gpu_mbasis_leaf(const uint32_t* G, int64_t ldG, int64_t gbs, int m, int n, int sigma, int64_t* d,
                           uint32_t* P, int64_t ldP, int64_t pbs, const PrimeBatch& pb, hipStream_t st) {
    if (pb.n < 1 || pb.n > SIGMA_BATCH_MAX) return hipErrorInvalidValue;
    if (m == 2 * n && n >= 1 && n <= LEAF2_MAX_S) {
        switch (n) {
            case 1: return leaf2_s<1>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 2: return leaf2_s<2>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 3: return leaf2_s<3>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 4: return leaf2_s<4>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 5: return leaf2_s<5>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 6: return leaf2_s<6>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 7: return leaf2_s<7>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 8: return leaf2_s<8>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 9: return leaf2_s<9>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 10: return leaf2_s<10>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 11: return leaf2_s<11>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 12: return leaf2_s<12>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 13: return leaf2_s<13>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 14: return leaf2_s<14>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 15: return leaf2_s<15>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            case 16: return leaf2_s<16>(G, ldG, gbs, sigma, d, P, ldP, pbs, pb, st);
            default: break;
        }
    }
    size_t lds = mbasis_leaf_lds(m, n, sigma);
    k_mbasis_leaf<<<(unsigned)pb.n, LEAF_TPB, lds, st>>>(G, ldG, gbs, m, n, sigma, d, P, ldP, pbs, pb);
    return hipGetLastError();
}

}  // namespace bwr
