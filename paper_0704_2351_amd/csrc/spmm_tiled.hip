// Two-dimensional tiled sparse x block product mod p (the "A^T A u" operation of
// a sequence step, Table "tab:r-opp"), optionally fused with the U^T projection
// of its output (projections by blocks, Section 2.3).
//
// Why tiles.  A row-parallel product gathers one W-residue row of the input
// block per non-zero, at a random row.  When the block is much larger than an
// XCD's L2 (4 MB), nearly every gather moves a whole cache line from beyond the
// L2 for a 16- or 32-byte row, so the kernel moves many times its algorithmic
// bytes.  Here the output rows are cut into row blocks of R rows and the input
// rows (the columns of the sparse operand) into slabs of C = 2^cb rows, small
// enough that a slab of the block stays in L2.  A workgroup owns one row block
// at a time: its R x W accumulators live in LDS, and it streams the block's
// non-zeros slab by slab, so every workgroup of an XCD gathers from the same
// slab at about the same time and the slab is fetched into that L2 once per
// round of row blocks instead of once per gather.
//
// Row blocks interleave: block b holds rows b, b + nrb, b + 2 nrb, ... (local
// row r is row b + r nrb), so that every block carries about the same number
// of non-zeros whatever the row order (the rows come sorted by length), and
// nrb is a multiple of the persistent grid: the workgroups then start each
// round of blocks together and walk the slabs at the same pace, which is what
// keeps one slab shared in an XCD's L2.
//
// Encoding (built on the device from the packed CSR, tiled_build below): the
// non-zeros of tile (row block b, slab k) are contiguous, tiles in order
// (b, k), entries of a tile in order of local row; tile_ptr[b * K + k] is the
// first entry of the tile (nrb * K + 1 entries).  One uint32 per non-zero:
//     bits [0, vb)          the value, vb-bit two's complement
//     bits [vb, vb + cb)    column inside the slab
//     bits [vb + cb, 32)    row inside the row block
// so the matrix costs 4 bytes per non-zero and no row pointers.
//
// Accumulation: for p <= 2^16 one int32 per output entry (the caller checks
// max row length * max |a| * (p - 1) < 2^31); for larger primes each residue
// is split into 16-bit halves summed in two int32 (the caller checks
// max row length * max |a| * 65535 < 2^31).  Every product is a value of at
// most vb <= 24 bits times a residue or half below 2^16, so it is formed with
// the full-rate 24-bit multiply.  Adds go to LDS with atomic adds
// (integer sums, so their order never changes the result), then one reduction
// mod p, the row scale and a coalesced store per output entry.
//
// Packed accumulators (p <= 2^16): the sums of two adjacent columns share one
// 64-bit word, T = 2^31 + sum_even + 2^32 sum_odd (mod 2^64), words row-major
// (W / 2 per row).  A product pair is added as the signed 64-bit value
// 2^32 a x_odd + a x_even with one 64-bit LDS atomic: since every partial sum
// of a row stays within (-2^31, 2^31), the low half stays within [0, 2^32) and
// never carries into the high half, so sum_even = low - 2^31 and sum_odd = the
// high half exactly, whatever the order of the adds.  An entry's lanes visit
// their column pairs in an order rotated by the entry's index, so the lanes of
// one instruction spread over different LDS banks (measured at 2M x 1M,
// block 16: the first product 19 % faster, the second 4 %, than one 32-bit add
// per column in column-major order).
//
// Projection (PM = 1): after a row block is stored its reduced rows stay in LDS
// and 4 x 4 tiles of the W x W partial U^T Z are accumulated per thread over
// the rows it visits; the threads' tiles then meet in LDS (64-bit sums) and are
// added to the workgroup's running sums, so the tiles occupy registers only
// during the projection; at the end each workgroup writes one W x W partial,
// reduced later by k_reduce_partials.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <vector>

#include "kernels.h"

namespace bwr {

namespace {

constexpr int TT = 1024;  // threads of a tiled workgroup (16 waves: one workgroup per CU, LDS-bound)
constexpr int BTPB = 256;
constexpr int UNMAX = 4;  // entries a lane takes per pass, at most
typedef double dvec4 __attribute__((ext_vector_type(4)));  // accumulators of a 16 x 16 x 4 f64 MFMA
// s_waitcnt operand of gfx9: vmcnt 0 (bits 3:0 and 15:14), expcnt and lgkmcnt left at their maximum (no wait)
constexpr int VMCNT0 = 0x0F70;
constexpr int STAGE_ROWS_MAX = 1024;  // rows of a staged chunk of the matrix-core projection's operands, at most
constexpr int STAGE_PIECES = 4;       // 16-byte (or smaller) pieces a thread holds per staged chunk, at most

// rows of a staged chunk for a kernel that stages rows of row_bytes bytes
constexpr int stage_rows_cap(int row_bytes) {
    const int pieces = row_bytes >= 16 ? row_bytes / 16 : 1;
    return STAGE_PIECES * TT / pieces < STAGE_ROWS_MAX ? STAGE_PIECES * TT / pieces : STAGE_ROWS_MAX;
}

// a register piece of B bytes (staged copies; plain vector types, which stay in registers)
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <int B> struct PieceOf;
template <> struct PieceOf<4> { using T = uint32_t; };
template <> struct PieceOf<8> { using T = u32x2; };
template <> struct PieceOf<16> { using T = u32x4; };

// 4 residues (projection operands)
__device__ __forceinline__ void ld4(const uint32_t* p, uint32_t (&x)[4]) {
    uint4 v = *reinterpret_cast<const uint4*>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
}
__device__ __forceinline__ void ld4(const uint16_t* p, uint32_t (&x)[4]) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    x[0] = v.x & 0xffffu;
    x[1] = v.x >> 16;
    x[2] = v.y & 0xffffu;
    x[3] = v.y >> 16;
}

// NWD consecutive 32-bit words (8, 16 or 32 bytes, aligned)
template <int NWD>
__device__ __forceinline__ void ldw(const void* p, uint32_t (&w)[NWD]) {
    if constexpr (NWD == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        w[0] = v.x;
        w[1] = v.y;
    } else {
        static_assert(NWD % 4 == 0, "8, 16 or 32 bytes");
#pragma unroll
        for (int h = 0; h < NWD / 4; ++h) {
            const uint4 v = reinterpret_cast<const uint4*>(p)[h];
            w[4 * h] = v.x;
            w[4 * h + 1] = v.y;
            w[4 * h + 2] = v.z;
            w[4 * h + 3] = v.w;
        }
    }
}
template <int NWD>
__device__ __forceinline__ void stw(void* p, const uint32_t (&w)[NWD]) {
    if constexpr (NWD == 2) {
        *reinterpret_cast<uint2*>(p) = make_uint2(w[0], w[1]);
    } else {
#pragma unroll
        for (int h = 0; h < NWD / 4; ++h)
            reinterpret_cast<uint4*>(p)[h] = make_uint4(w[4 * h], w[4 * h + 1], w[4 * h + 2], w[4 * h + 3]);
    }
}

// residue c of a lane's packed words
template <typename E>
__device__ __forceinline__ uint32_t residue(const uint32_t* w, int c) {
    if constexpr (sizeof(E) == 2)
        return (w[c >> 1] >> ((c & 1) * 16)) & 0xffffu;
    else
        return w[c];
}
template <typename E>
__device__ __forceinline__ void put_residue(uint32_t* w, int c, uint32_t y) {
    if constexpr (sizeof(E) == 2)
        w[c >> 1] |= y << ((c & 1) * 16);
    else
        w[c] = y;
}

// W: padded block width; E: stored residue type; SPLIT: 16-bit halves (p > 2^16); PM: fused projection of the
// output Z: 0 none, 1 U^T Z (U from memory), 2 the weighted Gram matrix Z^T diag(wgt) Z (symmetric.hip's form).
// Dynamic LDS: NACC * RS int32 accumulators (NACC = W, or 2 W with SPLIT), then K + 1 tile pointers; with
// a projection at least W * W * 8 bytes for the final partial sums.
//
// A lane owns the CPL = min(W, 16 bytes of residues) columns q CPL .. of an entry: the LPE lanes of an entry
// load the consecutive 16-byte pieces of its gathered row in one instruction, which the memory pipeline
// serves as one access per row (measured at 2M x 1M, block 16: 3-5 % faster than one lane loading the
// 32-byte row in two instructions).  A pass takes un (1 .. UNMAX) entries per lane, whose words were loaded
// one pass ahead; its gathers go out one after another, each after the lane's loads before it have arrived.
// More gathers in flight measured slower: with all four of a pass outstanding together, 383 and 455 us per
// product at 2M x 1M, block 16, against 287 and 309 us one at a time.  The random 16-byte gathers are bound
// by the memory pipeline's miss handling, which more outstanding requests per CU congest.
template <int W, typename E, bool SPLIT, int PM>
__global__ __launch_bounds__(TT) void k_spmm_tiled(int64_t nrows, int64_t nrb, int K, int R, int RS, int cb,
                                                   int vb, const uint32_t* __restrict__ tile_ptr,
                                                   const uint32_t* __restrict__ ent, const E* __restrict__ X,
                                                   const uint32_t* __restrict__ scale, E* __restrict__ Y,
                                                   const E* __restrict__ U, const uint32_t* __restrict__ wgt,
                                                   uint32_t* __restrict__ partial, int un, int sr, ModP mp) {
    constexpr bool PROJ = PM != 0;
    extern __shared__ __align__(16) int32_t lds[];
    constexpr int NACC = SPLIT ? 2 * W : W;
    constexpr int CPL = W < 16 / (int)sizeof(E) ? W : 16 / (int)sizeof(E);
    constexpr int LPE = W / CPL;                 // lanes per entry
    constexpr int EPI = TT / LPE;                // entries per pass of the workgroup
    constexpr int NWD = CPL * (int)sizeof(E) / 4;  // words a lane gathers per entry
    constexpr int WB = W / 4;                    // 4 x 4 tiles of the projection partial per side
    constexpr int NT = WB * WB;
    constexpr int NG = TT / NT;                  // row groups of the projection
    static_assert(W >= 4 && W <= 64 && (W & (W - 1)) == 0, "W must be a power of two in 4..64");
    constexpr bool PK = !SPLIT;                  // packed 64-bit pairs, row-major (see the header)
    // projection on the matrix cores for residues below 2^16 and W <= 32 (NTL 16-wide tiles per side)
    constexpr bool MFP = PROJ && !SPLIT && W <= 32;
    constexpr int NTL = W >= 16 ? W / 16 : 1;
    constexpr int NP = CPL / 2;                  // column pairs of a lane
    constexpr int WPP = NWD / NP;                // gathered words per column pair (1 or 2)
    constexpr uint32_t BIAS = 0x80000000u;
    // a staged row (U row, or weight) is PPR pieces of PB bytes; a thread copies at most SPT pieces per chunk
    constexpr int SRB = PM == 1 ? W * (int)sizeof(E) : 4;
    constexpr int PB = SRB >= 16 ? 16 : SRB;
    constexpr int PPR = SRB / PB;
    constexpr int SRM = stage_rows_cap(SRB);
    constexpr int SPT = MFP ? (SRM * PPR + TT - 1) / TT : 1;
    using Piece = typename PieceOf<PB>::T;
    // grouped epilogue loads (EG rows' scale factors a thread loads together) where registers allow
    constexpr bool GE = !SPLIT && W <= 32;
    constexpr int EG = GE ? 4 : 1;
    static_assert(!PK || (CPL % 2 == 0 && (NP & (NP - 1)) == 0), "packed pairs need an even power-of-two CPL");
    int32_t* acc = lds;
    unsigned long long* acc64 = reinterpret_cast<unsigned long long*>(lds);
    uint32_t* tp = reinterpret_cast<uint32_t*>(lds + NACC * RS);
    // LDS index of the reduced value of column c of local row r (kept in place of the accumulators)
    auto zix = [&](int c, int r) { return PK ? r * W + c : c * RS + r; };
    // staging of the matrix-core projection's operands (sr > 0): the U rows (PM 1) or weights (PM 2) of sr rows
    // at a time, after the tile pointers, 16-byte aligned
    unsigned char* const stage =
        reinterpret_cast<unsigned char*>(lds) + ((((size_t)NACC * RS + K + 1) * sizeof(int32_t) + 15) & ~(size_t)15);
    const int q = threadIdx.x % LPE;
    const int es = threadIdx.x / LPE;
    const uint32_t cmask = (1u << cb) - 1u;
    const int vsh = 32 - vb;
    const int rsh = cb + vb;
    const int pt = threadIdx.x % NT, pg = threadIdx.x / NT;
    const int pti = pt / WB, ptj = pt % WB;

    using PAcc = typename std::conditional<SPLIT, uint32_t, uint64_t>::type;
    // the workgroup's W x W projection sums over its row blocks, entry threadIdx.x + h TT in tot[h]
    constexpr int NTOT = (W * W + TT - 1) / TT;
    unsigned long long tot[NTOT];
#pragma unroll
    for (int h = 0; h < NTOT; ++h) tot[h] = 0;

    const uint32_t EPS = (uint32_t)un * EPI;  // entries per pass
    for (int64_t rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
        int4* acc4 = reinterpret_cast<int4*>(acc);
        if constexpr (PK) {
            for (int i = threadIdx.x; i < R * W / 4; i += TT) acc4[i] = make_int4((int)BIAS, 0, (int)BIAS, 0);
        } else {
            for (int i = threadIdx.x; i < NACC * RS / 4; i += TT) acc4[i] = make_int4(0, 0, 0, 0);
        }
        for (int i = threadIdx.x; i <= K; i += TT) tp[i] = tile_ptr[rb * K + i];
        __syncthreads();
        const uint32_t end = tp[K];
        uint32_t e0 = tp[0] + (uint32_t)es;
        uint32_t wn[UNMAX];
#pragma unroll
        for (int u = 0; u < UNMAX; ++u) {
            const uint32_t idx = e0 + u * EPI;
            wn[u] = (u < un && idx < end) ? __builtin_nontemporal_load(ent + idx) : 0u;
        }
        // the slab of an entry: k advances (a lane's entries only move forward through the row block's
        // tiles); knext caches tp[k + 1]
        int k = 0;
        uint32_t knext = tp[1];
        for (; e0 < end; e0 += EPS) {
            uint32_t w[UNMAX];
#pragma unroll
            for (int u = 0; u < UNMAX; ++u) w[u] = wn[u];
#pragma unroll
            for (int u = 0; u < UNMAX; ++u) {
                const uint32_t idx = e0 + EPS + u * EPI;
                wn[u] = (u < un && idx < end) ? __builtin_nontemporal_load(ent + idx) : 0u;
            }
            uint32_t xv[UNMAX][NWD];
#pragma unroll
            for (int u = 0; u < UNMAX; ++u) {
                const uint32_t idx = e0 + u * EPI;
                if (u < un && idx < end) {
                    while (idx >= knext) knext = tp[++k + 1];
                    const size_t xr = ((size_t)k << cb) + ((w[u] >> vb) & cmask);
                    // one gather of a lane in flight at a time (see the header)
                    __builtin_amdgcn_s_waitcnt(VMCNT0);
                    ldw<NWD>(X + xr * W + q * CPL, xv[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < UNMAX; ++u) {
                if (u < un && e0 + u * EPI < end) {
                    const int lr = (int)(w[u] >> rsh);
                    const int32_t a = (int32_t)(w[u] << vsh) >> vsh;
                    if constexpr (PK) {
                        // rotate the lane's pairs by the entry's index (selects on registers), then pair j of
                        // the rotated order is the lane's pair (j + rot) mod NP
                        const int rot = (int)(es + u * EPI) & (NP - 1);
                        uint32_t* v = xv[u];
#pragma unroll
                        for (int b = 1; b < NP; b <<= 1) {
                            uint32_t t[NWD];
#pragma unroll
                            for (int h = 0; h < NWD; ++h) t[h] = v[(h + b * WPP) % NWD];
#pragma unroll
                            for (int h = 0; h < NWD; ++h) v[h] = (rot & b) ? t[h] : v[h];
                        }
                        unsigned long long* rowp = acc64 + (size_t)lr * (W / 2) + q * NP;
#pragma unroll
                        for (int j = 0; j < NP; ++j) {
                            const int32_t lo = __mul24(a, (int32_t)residue<E>(v, 2 * j));
                            const int32_t hi = __mul24(a, (int32_t)residue<E>(v, 2 * j + 1));
                            const int64_t d = (int64_t)((uint64_t)(uint32_t)hi << 32) + (int64_t)lo;
                            atomicAdd(rowp + ((j + rot) & (NP - 1)), (unsigned long long)d);
                        }
                    } else {
#pragma unroll
                        for (int c = 0; c < CPL; ++c) {
                            const uint32_t x = residue<E>(xv[u], c);
                            atomicAdd(&acc[(q * CPL + c) * RS + lr], __mul24(a, (int32_t)(x & 0xffffu)));
                            atomicAdd(&acc[(W + q * CPL + c) * RS + lr], __mul24(a, (int32_t)(x >> 16)));
                        }
                    }
                }
            }
        }
        __syncthreads();
        // reduce, scale, store: lane (row, column group), so consecutive lanes store consecutive rows
        // rows of block rb: rb, rb + nrb, rb + 2 nrb, ... (local row r is row rb + r nrb)
        const int nr = (int)((nrows - rb + nrb - 1) / nrb);
        uint32_t* zl = reinterpret_cast<uint32_t*>(acc);
        // staged projection: chunks of cs rows; a thread's pieces of a chunk are all loaded before any is written
        // to LDS, so a chunk costs one memory latency (on gfx9 a wait for a load also waits for earlier stores)
        const int cs = sr > 0 ? (sr < SRM ? sr : SRM) : nr;
        Piece pc[SPT];
        // (every piece is loaded: indices past the chunk repeat its last piece, so no load waits in a branch)
        auto stage_load = [&](int c0, int c1) {
            const int n = (c1 - c0) * PPR;
#pragma unroll
            for (int h = 0; h < SPT; ++h) {
                const int i = threadIdx.x + h * TT < n ? threadIdx.x + h * TT : n - 1;
                const int64_t row = rb + (int64_t)(c0 + i / PPR) * nrb;
                if constexpr (PM == 1)
                    pc[h] = reinterpret_cast<const Piece*>(U + (size_t)row * W)[i % PPR];
                else
                    pc[h] = wgt[row];
            }
        };
        auto stage_store = [&](int c0, int c1) {
#pragma unroll
            for (int h = 0; h < SPT; ++h) {
                const int i = threadIdx.x + h * TT;
                if (i < (c1 - c0) * PPR) reinterpret_cast<Piece*>(stage)[i] = pc[h];
            }
        };
        // row r, column group qq of the block (i = r LPE + qq): reduce, scale by sc, store, keep the result for
        // the projection
        const int ne = nr * LPE;
        auto epi_row = [&](int i, uint32_t sc) {
            const int r = i / LPE, qq = i % LPE;
            const int64_t row = rb + (int64_t)r * nrb;
            uint32_t yw[NWD];
#pragma unroll
            for (int h = 0; h < NWD; ++h) yw[h] = 0;
            if constexpr (PK) {
                // the lane's NP words, read before the reduced values overwrite them in place
                unsigned long long pw[NP];
#pragma unroll
                for (int j = 0; j < NP; ++j) pw[j] = acc64[(size_t)r * (W / 2) + qq * NP + j];
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const unsigned long long t = pw[c / 2];
                    const int32_t sum = (c & 1) ? (int32_t)(uint32_t)(t >> 32) : (int32_t)((uint32_t)t - BIAS);
                    const uint32_t y = mulmod16(mp, reds32(mp, sum), sc);
                    put_residue<E>(yw, c, y);
                    if constexpr (PROJ) zl[zix(qq * CPL + c, r)] = y;
                }
            } else {
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    const int idx = (qq * CPL + c) * RS + r;
                    const uint32_t red =
                        reds64(mp, (int64_t)acc[(W + qq * CPL + c) * RS + r] * 65536 + (int64_t)acc[idx]);
                    const uint32_t y = mulmod(mp, red, sc);
                    put_residue<E>(yw, c, y);
                    if constexpr (PROJ) zl[idx] = y;
                }
            }
            stw<NWD>(Y + (size_t)row * W + qq * CPL, yw);
        };
        if constexpr (!GE) {
            // (kernels without registers to spare: one factor at a time)
            for (int i = threadIdx.x; i < ne; i += TT) epi_row(i, scale ? scale[rb + (int64_t)(i / LPE) * nrb] : 1u);
        } else {
            // EG rows of a thread per group, their scale factors loaded together (indices past the block repeat
            // its last row); the first group's factors and the first staged chunk are loaded before any wait
            uint32_t scv[EG];
            auto scale_group = [&](int i0) {
                if (scale) {
#pragma unroll
                    for (int h = 0; h < EG; ++h) {
                        const int i = i0 + h * TT < ne ? i0 + h * TT : ne - 1;
                        scv[h] = scale[rb + (int64_t)(i / LPE) * nrb];
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < EG; ++h) scv[h] = 1u;
                }
            };
            if (MFP && sr > 0 && scale && ne > 0) {
                // every address first, then every load, in every lane (a uniform branch: lanes past the block
                // load its last row's factor and do not use it)
                const int c1 = cs < nr ? cs : nr, n = c1 * PPR;
                const uint32_t* sa[EG];
                const Piece* pa[SPT];
#pragma unroll
                for (int h = 0; h < EG; ++h) {
                    const int i = (int)threadIdx.x + h * TT < ne ? (int)threadIdx.x + h * TT : ne - 1;
                    sa[h] = scale + rb + (int64_t)(i / LPE) * nrb;
                }
#pragma unroll
                for (int h = 0; h < SPT; ++h) {
                    const int i = (int)threadIdx.x + h * TT < n ? (int)threadIdx.x + h * TT : n - 1;
                    const int64_t row = rb + (int64_t)(i / PPR) * nrb;
                    if constexpr (PM == 1)
                        pa[h] = reinterpret_cast<const Piece*>(U + (size_t)row * W) + i % PPR;
                    else
                        pa[h] = reinterpret_cast<const Piece*>(wgt + row);
                }
#pragma unroll
                for (int h = 0; h < EG; ++h) scv[h] = *sa[h];
#pragma unroll
                for (int h = 0; h < SPT; ++h) pc[h] = *pa[h];
            } else {
                if ((int)threadIdx.x < ne) scale_group(threadIdx.x);
                if constexpr (MFP)
                    if (sr > 0) stage_load(0, cs < nr ? cs : nr);
            }
            for (int i0 = threadIdx.x; i0 < ne; i0 += EG * TT) {
                if (i0 != (int)threadIdx.x) scale_group(i0);
                // one row at a time (register pressure), each taking the next preloaded factor
#pragma unroll 1
                for (int h = 0; h < EG; ++h) {
                    if (i0 + h * TT >= ne) break;
                    const uint32_t sc = scv[0];
#pragma unroll
                    for (int g = 0; g + 1 < EG; ++g) scv[g] = scv[g + 1];
                    epi_row(i0 + h * TT, sc);
                }
            }
        }
        if constexpr (PROJ && MFP) {
            // the block's partial as a dense contraction on the matrix cores: D (16 x 16 per tile pair) +=
            // A (16 x 4) B (4 x 16) with A = the U (or weighted Z) values of 4 rows, transposed, and B = their
            // reduced rows; lane l holds A[l % 16][l / 16] and B[l / 16][l % 16], i.e. both at row l / 16,
            // column l % 16 of the 4 rows, and D[l / 16 + 4 i][l % 16] in its i-th accumulator.  Residues
            // are below 2^16, so every product and every sum over the row block (fewer than 2^21 rows) is an
            // integer below 2^53, exact in double precision.
            const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6, cc = ln & 15, kk = ln >> 4;
            dvec4 dacc[NTL][NTL];
#pragma unroll
            for (int tm = 0; tm < NTL; ++tm)
#pragma unroll
                for (int tn = 0; tn < NTL; ++tn) dacc[tm][tn] = dvec4{0.0, 0.0, 0.0, 0.0};
            // the products over rows c0 .. c1 - 1, their U rows (or weights) from the staged chunk (ST) or from
            // memory
            auto rows_mfma = [&](auto staged, int c0, int c1) {
                constexpr bool ST = decltype(staged)::value;
                // QD row quads of the wave per step: their LDS reads all go out before the first product (rows
                // past the chunk read its last row and contribute 0), and the products alternate between two
                // accumulator sets, so a step pays one LDS latency for QD products (one quad for W = 32: its
                // four tiles leave no registers for more)
                constexpr int QD = NTL == 1 ? 4 : 1;
                dvec4 dacc2[NTL][NTL];
#pragma unroll
                for (int tm = 0; tm < NTL; ++tm)
#pragma unroll
                    for (int tn = 0; tn < NTL; ++tn) dacc2[tm][tn] = dvec4{0.0, 0.0, 0.0, 0.0};
                for (int rbase = c0 + wv * 4; rbase < c1; rbase += QD * (TT / 64) * 4) {
                    double av[QD][NTL], bv[QD][NTL];
#pragma unroll
                    for (int d = 0; d < QD; ++d) {
                        const int r0 = rbase + d * (TT / 64) * 4 + kk;
                        const bool in = r0 < c1;
                        const int r = in ? r0 : c1 - 1;
#pragma unroll
                        for (int t = 0; t < NTL; ++t) {
                            const int c = t * 16 + cc;
                            uint32_t uu = 0, zz = 0;
                            if (c < W) {
                                zz = zl[zix(c, r)];
                                if constexpr (PM == 1)
                                    uu = ST ? (uint32_t)reinterpret_cast<const E*>(stage)[(r - c0) * W + c]
                                            : (uint32_t)U[(size_t)(rb + (int64_t)r * nrb) * W + c];
                                else
                                    uu = mulmod16(mp, ST ? reinterpret_cast<const uint32_t*>(stage)[r - c0]
                                                         : wgt[rb + (int64_t)r * nrb], zz);
                            }
                            av[d][t] = in ? (double)uu : 0.0;
                            bv[d][t] = (double)zz;
                        }
                    }
#pragma unroll
                    for (int d = 0; d < QD; ++d)
#pragma unroll
                        for (int tm = 0; tm < NTL; ++tm)
#pragma unroll
                            for (int tn = 0; tn < NTL; ++tn) {
                                if (d & 1)
                                    dacc2[tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d][tm], bv[d][tn],
                                                                                          dacc2[tm][tn], 0, 0, 0);
                                else
                                    dacc[tm][tn] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[d][tm], bv[d][tn],
                                                                                         dacc[tm][tn], 0, 0, 0);
                            }
                }
                if constexpr (QD > 1) {
#pragma unroll
                    for (int tm = 0; tm < NTL; ++tm)
#pragma unroll
                        for (int tn = 0; tn < NTL; ++tn) dacc[tm][tn] += dacc2[tm][tn];
                }
            };
            if (sr > 0) {
                // chunk c is copied to LDS while chunk c + 1's loads are in flight, so the loads of every chunk
                // after the first overlap the products of the one before
                stage_store(0, cs < nr ? cs : nr);
                __syncthreads();
                for (int c0 = 0; c0 < nr; c0 += cs) {
                    const int c1 = c0 + cs < nr ? c0 + cs : nr;
                    const int c2 = c1 + cs < nr ? c1 + cs : nr;
                    if (c1 < nr) stage_load(c1, c2);
                    rows_mfma(std::true_type{}, c0, c1);
                    if (c1 < nr) {
                        __syncthreads();  // the chunk's staged rows are read before the next chunk's copy
                        stage_store(c1, c2);
                        __syncthreads();
                    }
                }
            } else {
                __syncthreads();
                rows_mfma(std::false_type{}, 0, nr);
            }
            // the waves' tiles meet in W x W 64-bit LDS sums (over the reduced rows, now read)
            __syncthreads();
            unsigned long long* red = reinterpret_cast<unsigned long long*>(lds);
            for (int e = threadIdx.x; e < W * W; e += TT) red[e] = 0;
            __syncthreads();
#pragma unroll
            for (int tm = 0; tm < NTL; ++tm)
#pragma unroll
                for (int tn = 0; tn < NTL; ++tn)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int mrow = tm * 16 + kk + 4 * i, ncol = tn * 16 + cc;
                        if (mrow < W && ncol < W)
                            atomicAdd(&red[mrow * W + ncol], (unsigned long long)dacc[tm][tn][i]);
                    }
            __syncthreads();
#pragma unroll
            for (int h = 0; h < NTOT; ++h)
                if (threadIdx.x + h * TT < W * W) tot[h] += red[threadIdx.x + h * TT];
        } else if constexpr (PROJ) {
            // 4 x 4 tiles of this row block's partial per thread (live only here, not in the gather loop)
            PAcc pacc[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) pacc[a][b] = 0;
            __syncthreads();
            // 4 rows per round, their U loads issued together
            for (int r0 = pg; r0 < nr; r0 += 4 * NG) {
                uint32_t u[4][4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = r0 + j * NG;
                    if (r >= nr) continue;
                    if constexpr (PM == 1) {
                        ld4(U + (size_t)(rb + (int64_t)r * nrb) * W + pti * 4, u[j]);
                    } else {
                        // Gram form: u = wgt[row] * z_i, from this block's own output in LDS
                        const uint32_t wr = wgt[rb + (int64_t)r * nrb];
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            const uint32_t zi = zl[zix(pti * 4 + a, r)];
                            u[j][a] = SPLIT ? mulmod(mp, wr, zi) : mulmod16(mp, wr, zi);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int r = r0 + j * NG;
                    if (r >= nr) break;
                    uint32_t z[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b) z[b] = zl[zix(ptj * 4 + b, r)];
#pragma unroll
                    for (int a = 0; a < 4; ++a)
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            if constexpr (SPLIT)
                                pacc[a][b] = addmod(mp, pacc[a][b], mulmod(mp, u[j][a], z[b]));
                            else
                                pacc[a][b] += (uint64_t)(u[j][a] * z[b]);
                        }
                }
            }
            // the threads' tiles meet in W x W 64-bit LDS sums (over the reduced rows, now read)
            __syncthreads();
            unsigned long long* red = reinterpret_cast<unsigned long long*>(lds);
            for (int e = threadIdx.x; e < W * W; e += TT) red[e] = 0;
            __syncthreads();
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    atomicAdd(&red[(pti * 4 + a) * W + ptj * 4 + b], (unsigned long long)pacc[a][b]);
            __syncthreads();
#pragma unroll
            for (int h = 0; h < NTOT; ++h)
                if (threadIdx.x + h * TT < W * W) tot[h] += red[threadIdx.x + h * TT];
        }
        __syncthreads();
    }
    if constexpr (PROJ) {
        // one W x W partial per workgroup
#pragma unroll
        for (int h = 0; h < NTOT; ++h)
            if (threadIdx.x + h * TT < W * W)
                partial[(size_t)blockIdx.x * W * W + threadIdx.x + h * TT] = red64(mp, tot[h]);
    }
}

// ---- encoding ----

// cnt[(b * K + k) * R + lr] = entries of row b + lr nrb in slab k
__global__ __launch_bounds__(BTPB) void k_tile_count(int64_t rows, int64_t nrb, const int32_t* __restrict__ rp,
                                                     const uint32_t* __restrict__ ent, int K, int R, int cb,
                                                     int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * BTPB + threadIdx.x;
    if (i >= rows) return;
    const int64_t b = i % nrb;
    const int lr = (int)(i / nrb);
    for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
        const uint32_t col = ent[t] & 0xFFFFFFu;
        atomicAdd(&cnt[(b * K + (col >> cb)) * R + lr], 1);
    }
}

// tile_ptr[t] = pos[t * R] for t <= ntiles (pos holds ntiles * R + 1 entries)
__global__ __launch_bounds__(BTPB) void k_tile_ptrs(int64_t ntiles, int R, const int32_t* __restrict__ pos,
                                                    uint32_t* __restrict__ tile_ptr) {
    const int64_t t = (int64_t)blockIdx.x * BTPB + threadIdx.x;
    if (t <= ntiles) tile_ptr[t] = (uint32_t)pos[t * R];
}

// one thread per row: its entries go to the next free places of their (row block, slab, local row) runs, in
// the row's order (each run belongs to one row, so the order is deterministic)
__global__ __launch_bounds__(BTPB) void k_tile_scatter(int64_t rows, int64_t nrb, const int32_t* __restrict__ rp,
                                                       const uint32_t* __restrict__ ent, int K, int R, int cb,
                                                       int vb, int32_t* __restrict__ pos, uint32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BTPB + threadIdx.x;
    if (i >= rows) return;
    const int64_t b = i % nrb;
    const int lr = (int)(i / nrb);
    const uint32_t cmask = (1u << cb) - 1u, vmask = (1u << vb) - 1u;
    for (int32_t t = rp[i]; t < rp[i + 1]; ++t) {
        const uint32_t w = ent[t];
        const uint32_t col = w & 0xFFFFFFu;
        const int32_t a = (int32_t)w >> 24;
        const int64_t slot = (b * K + (col >> cb)) * R + lr;
        const int32_t p = pos[slot];
        pos[slot] = p + 1;
        out[p] = ((uint32_t)lr << (cb + vb)) | ((col & cmask) << vb) | ((uint32_t)a & vmask);
    }
}

// Raises a kernel's dynamic-LDS limit on the current device to the device maximum, once (under a lock).
hipError_t allow_max_lds(const void* fn, size_t want) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& d : done)
        if (d.first == fn && d.second == dev) return hipSuccess;
    int mx = 0;
    e = hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if ((size_t)mx < want) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, mx);
    if (e == hipSuccess) done.emplace_back(fn, dev);
    return e;
}

// Largest dynamic LDS of a workgroup on the current device (cached per device).
size_t device_max_lds() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
    if (!cache[dev] && hipDeviceGetAttribute(&cache[dev], hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 65536;
    return (size_t)cache[dev];
}

template <int W, typename E, bool SPLIT, int PM>
hipError_t launch_t(const TiledOperand& t, const void* X, const uint32_t* scale, void* Y, const void* U,
                    const uint32_t* wgt, uint32_t* partial, const TiledLaunch& L, ModP mp, hipStream_t st) {
    size_t lds = tiled_lds_bytes(W, SPLIT, PM != 0, t.R, t.K);
    // the matrix-core projection stages its operands in the LDS the accumulators leave free: chunks of sr rows
    // (a multiple of 64, at most stage_rows_cap; none when fewer than 64 rows fit: direct loads)
    int sr = 0;
    if constexpr (PM != 0 && !SPLIT && W <= 32) {
        if (!getenv("BWR_TILED_NO_STAGE")) {
            const size_t base = (((size_t)W * (t.R + 1) + t.K + 1) * 4 + 15) & ~(size_t)15;
            const size_t per_row = PM == 1 ? (size_t)W * sizeof(E) : sizeof(uint32_t);
            const size_t mx = device_max_lds();
            sr = (int)std::min<size_t>(stage_rows_cap((int)per_row), mx > base ? (mx - base) / per_row : 0) & ~63;
            if (sr > 0) lds = std::max(lds, base + (size_t)sr * per_row);
        }
    }
    hipError_t e = allow_max_lds(reinterpret_cast<const void*>(&k_spmm_tiled<W, E, SPLIT, PM>), lds);
    if (e != hipSuccess || L.grid == 0) return e;  // grid 0: only raise the LDS limit (before a graph capture)
    k_spmm_tiled<W, E, SPLIT, PM><<<(unsigned)L.grid, TT, lds, st>>>(
        t.rows, t.nrb, t.K, t.R, t.R + 1, t.cb, t.vb, t.tile_ptr, t.ent, (const E*)X, scale, (E*)Y, (const E*)U,
        wgt, partial, L.un, sr, mp);
    return hipGetLastError();
}

template <int W, typename E, bool SPLIT>
hipError_t launch_m(const TiledOperand& t, int pmode, const void* X, const uint32_t* scale, void* Y, const void* U,
                    const uint32_t* wgt, uint32_t* partial, const TiledLaunch& L, ModP mp, hipStream_t st) {
    switch (pmode) {
        case 0: return launch_t<W, E, SPLIT, 0>(t, X, scale, Y, U, wgt, partial, L, mp, st);
        case 1: return launch_t<W, E, SPLIT, 1>(t, X, scale, Y, U, wgt, partial, L, mp, st);
        case 2: return launch_t<W, E, SPLIT, 2>(t, X, scale, Y, U, wgt, partial, L, mp, st);
        default: return hipErrorInvalidValue;
    }
}

template <int W>
hipError_t launch_w(const TiledOperand& t, int pmode, bool split, int esize, const void* X, const uint32_t* scale,
                    void* Y, const void* U, const uint32_t* wgt, uint32_t* partial, const TiledLaunch& L, ModP mp,
                    hipStream_t st) {
    if (esize == 2) {
        if (split) return hipErrorInvalidValue;
        return launch_m<W, uint16_t, false>(t, pmode, X, scale, Y, U, wgt, partial, L, mp, st);
    }
    if (split) return launch_m<W, uint32_t, true>(t, pmode, X, scale, Y, U, wgt, partial, L, mp, st);
    return launch_m<W, uint32_t, false>(t, pmode, X, scale, Y, U, wgt, partial, L, mp, st);
}

}  // namespace

size_t tiled_lds_bytes(int W, bool split, bool proj, int R, int K) {
    const size_t nacc = (size_t)(split ? 2 * W : W);
    size_t b = sizeof(int32_t) * (nacc * (size_t)(R + 1) + (size_t)K + 1);
    if (proj) b = std::max<size_t>(b, (size_t)W * W * sizeof(uint64_t));
    return (b + 15) & ~(size_t)15;
}

int tiled_threads() { return TT; }

hipError_t launch_tiled_build(int64_t rows, int64_t nrb, const int32_t* rp, const uint32_t* ent, int K, int R,
                              int cb, int vb, int32_t* cnt, int32_t* pos, int32_t* scan_tmp, uint32_t* tile_ptr,
                              uint32_t* out, hipStream_t st) {
    if (nrb < 1 || nrb * (int64_t)R < rows) return hipErrorInvalidValue;
    const int64_t ntiles = nrb * K;
    const int64_t count = ntiles * R;
    hipError_t e = launch_fill_zero(cnt, sizeof(int32_t) * (size_t)std::max<int64_t>(count, 1), st);
    if (e != hipSuccess) return e;
    const unsigned g = (unsigned)std::max<int64_t>(1, (rows + BTPB - 1) / BTPB);
    if (rows > 0) {
        k_tile_count<<<g, BTPB, 0, st>>>(rows, nrb, rp, ent, K, R, cb, cnt);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = launch_exclusive_scan(count, cnt, pos, scan_tmp, st)) != hipSuccess) return e;
    k_tile_ptrs<<<(unsigned)((ntiles + 1 + BTPB - 1) / BTPB), BTPB, 0, st>>>(ntiles, R, pos, tile_ptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rows > 0) {
        k_tile_scatter<<<g, BTPB, 0, st>>>(rows, nrb, rp, ent, K, R, cb, vb, pos, out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t prepare_spmm_tiled(const TiledOperand& t, int W, int pmode, bool split, int esize) {
    if (esize != 2 && esize != 4) return hipErrorInvalidValue;
    const ModP mp = ModP::make(split ? 2147483647u : 65521u);
    const TiledLaunch L{};  // grid 0
    switch (W) {
        case 4: return launch_w<4>(t, pmode, split, esize, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, L, mp, 0);
        case 8: return launch_w<8>(t, pmode, split, esize, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, L, mp, 0);
        case 16: return launch_w<16>(t, pmode, split, esize, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, L, mp, 0);
        case 32: return launch_w<32>(t, pmode, split, esize, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, L, mp, 0);
        case 64: return launch_w<64>(t, pmode, split, esize, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, L, mp, 0);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spmm_tiled(const TiledOperand& t, int W, int pmode, bool split, int esize, const void* X,
                             const uint32_t* scale, void* Y, const void* U, const uint32_t* wgt, uint32_t* partial,
                             const TiledLaunch& L, ModP mp, hipStream_t st) {
    if (L.grid < 1 || L.un < 1 || L.un > UNMAX || t.R < 1 || t.nrb < 1 ||
        t.nrb * (int64_t)t.R < t.rows || t.K < 1 || t.cb < 1 || t.vb < 2 || t.vb > 24 || t.rb + t.cb + t.vb > 32 ||
        (1LL << t.rb) < t.R || pmode < 0 || pmode > 2 || (pmode == 1 && (!U || !partial)) ||
        (pmode == 2 && (!wgt || !partial)) || (esize != 2 && esize != 4) || split != (mp.p > 65536u))
        return hipErrorInvalidValue;
    switch (W) {
        case 4: return launch_w<4>(t, pmode, split, esize, X, scale, Y, U, wgt, partial, L, mp, st);
        case 8: return launch_w<8>(t, pmode, split, esize, X, scale, Y, U, wgt, partial, L, mp, st);
        case 16: return launch_w<16>(t, pmode, split, esize, X, scale, Y, U, wgt, partial, L, mp, st);
        case 32: return launch_w<32>(t, pmode, split, esize, X, scale, Y, U, wgt, partial, L, mp, st);
        case 64: return launch_w<64>(t, pmode, split, esize, X, scale, Y, U, wgt, partial, L, mp, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace bwr
