// Launchers for the gfx950 kernels of the block Wiedemann sequence.
//
// Device layouts (all row-major, residues uint32 in [0, p)):
//   packed CSR   rp[nrows + 1] (int32), ent[nnz] (uint32) with
//                ent = column | (uint8)value << 24 (columns < 2^24, |value| <= 127)
//   wide CSR     rp[nrows + 1] (int32), col[nnz] (int32), val[nnz] (uint32 residue)
//   blocks       X[n][W], Y[m][W] with W the padded block width (1..64, power of two);
//                padding columns are zero and stay zero
//   S            S[k][s][s]
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modp.h"

namespace bwr {

struct CsrStats {
    int32_t bad;       // non-zero: malformed input (see flags below)
    int32_t max_len;   // longest row
    int32_t max_abs;   // largest |value| (saturated at 2^31 - 1)
    int32_t pad;
};
enum : int32_t { BAD_ROWPTR = 1, BAD_COL = 2 };

// Row-pointer check (reads only rp): bad_dev = BAD_ROWPTR unless 0 = rp[0] <= ... <= rp[m] = nnz.
hipError_t launch_rowptr_check(int64_t m, int64_t nnz, const int64_t* rp, int32_t* bad_dev, hipStream_t st);
// out_dev = max(0, max in[i])
hipError_t launch_max_i32(int64_t count, const int32_t* in, int32_t* out_dev, hipStream_t st);
// Input validation and statistics over a device CSR with int64 row pointers (call after the row-pointer check).
hipError_t launch_csr_stats(int64_t m, int64_t n, const int64_t* rp, const int32_t* col,
                            const int32_t* val, CsrStats* out_dev, hipStream_t st);

// Packed encoding of A (rows kept in input order).
hipError_t launch_pack_rows(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val,
                            int32_t* rp32, uint32_t* ent, hipStream_t st);
// Wide encoding of A for one prime: columns copied, values reduced mod p.
hipError_t launch_wide_rows(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val,
                            ModP mp, int32_t* rp32, int32_t* colw, uint32_t* valw, hipStream_t st);

// Transpose support: column histogram, exclusive scan, scatter.
hipError_t launch_col_count(int64_t m, const int64_t* rp64, const int32_t* col, int32_t* cnt, hipStream_t st);
hipError_t launch_exclusive_scan(int64_t count, const int32_t* in, int32_t* out /* count + 1 */,
                                 int32_t* tmp /* >= scan_tmp_words(count) */, hipStream_t st);
int64_t scan_tmp_words(int64_t count);
// Relabelled CSR: row i = input row perm_r[i], columns mapped through inv_c; rp_out (m + 1) given.
hipError_t launch_permute_csr(int64_t m, const int64_t* rp_out, const int32_t* perm_r, const int64_t* rp64,
                              const int32_t* col, const int32_t* val, const int32_t* inv_c, int32_t* col_out,
                              int32_t* val_out, hipStream_t st);
// dst[i][c] = src[perm[i]][c], c < width (uint32 rows)
hipError_t launch_gather_rows(int64_t rows, int width, const int32_t* perm, const uint32_t* src, uint32_t* dst,
                              hipStream_t st);
// Column split of a packed operand (rows x cols, int32 row pointers): part 0 = entries with column < mid,
// part 1 = the rest, each a CSR over the same rows (rp0, rp1: rows + 1 entries; cnt0, cnt1: rows; tmp:
// scan_tmp_words(rows)).  ent0/ent1 must hold the counts the scans produce (at most nnz in all).
hipError_t launch_split_operand(int64_t rows, const int32_t* rp, const uint32_t* ent, uint32_t mid, int32_t* cnt0,
                                int32_t* cnt1, int32_t* tmp, int32_t* rp0, int32_t* rp1, uint32_t* ent0, uint32_t* ent1,
                                hipStream_t st);
hipError_t launch_scatter_packed_t(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val,
                                   const int32_t* rpT, int32_t* cursor, uint32_t* entT, hipStream_t st);
hipError_t launch_scatter_wide_t(int64_t m, const int64_t* rp64, const int32_t* col, const int32_t* val,
                                 ModP mp, const int32_t* rpT, int32_t* cursor, int32_t* colT, uint32_t* valT,
                                 hipStream_t st);

// Random residues from the counter-based SplitMix64 stream (seed, stream):
// out[r * ld + c] = element(r * s + c) for r < rows, c < s (and 0 for s <= c < ld).
hipError_t launch_rng_block(uint64_t seed, int stream, int64_t rows, int32_t s, int32_t ld, ModP mp,
                            int diag, uint32_t* out, hipStream_t st);

// Copy an n x s block into an n x W padded block of esize-byte residues
// (esize 2 needs p <= 2^16), optionally scaled row-wise by d[r] (mode 1) or by
// d[r]^-1 (mode 2); mode 0 copies.  Entries are reduced mod p.
hipError_t launch_pad_scale(int64_t n, int32_t s, int32_t W, const uint32_t* in, const uint32_t* d, int mode,
                            ModP mp, void* out, int esize, hipStream_t st);
// out[r * s + c] = in[r * W + c] for c < s (in: esize-byte residues)
hipError_t launch_unpad(int64_t n, int32_t s, int32_t W, const void* in, int esize, uint32_t* out, hipStream_t st);
// d2[r] = d[r]^2 mod p; also checks d[r] mod p != 0 (bad != 0 otherwise).
hipError_t launch_square_diag(int64_t n, const uint32_t* d, ModP mp, uint32_t* d2, int32_t* bad, hipStream_t st);
// reduce an arbitrary uint32 diagonal into [0, p)
hipError_t launch_reduce_vec(int64_t n, const uint32_t* in, ModP mp, uint32_t* out, hipStream_t st);
// bytes of zeros at p: a kernel, so that code a caller may capture in a graph records no memset node
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// Y[r] = scale[r] * sum_t a_rt X[col_t]  (mod p), for r < nrows.  scale may be null (1).
// acc32: the caller guarantees max_len * max|a| * (p - 1) < 2^31 and p <= 2^16.
hipError_t launch_spmm_packed(int W, bool acc32, bool smallp, int64_t nrows, const int32_t* rp, const uint32_t* ent,
                              const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st);
hipError_t launch_spmm_wide(int W, int64_t nrows, const int32_t* rp, const int32_t* col, const uint32_t* val,
                            const uint32_t* X, const uint32_t* scale, uint32_t* Y, ModP mp, hipStream_t st);

// Projection partials: partial[b][i * W + c] = sum over the rows of block b of U[r][i] X[r][c] mod p.
int proj_blocks(int64_t n, int W);
hipError_t launch_project(int W, bool smallp, int64_t n, const void* U, const void* X, int esize, uint32_t* partial,
                          int nblocks, ModP mp, hipStream_t st);
// S[k sstride][i][j] (i, j < s) = sum_b partial[k pstride + b W^2 + i W + j] mod p, for k < nsteps
// (pstride 0: nblocks W^2, the partials of consecutive steps back to back).
hipError_t launch_reduce_partials(int W, int32_t s, int nblocks, int64_t nsteps, const uint32_t* partial, uint32_t* S,
                                  ModP mp, hipStream_t st, int64_t pstride = 0, int64_t sstride = 1);

}  // namespace bwr

namespace bwr {
// Row-split sparse x block product (spmm.hip): W in {4..64}, G lanes per row
// slice (1..16, power of two), optional fused projection into per-block W x W
// partials (nblocks blocks in a grid-stride loop).
bool split_supported(int W, int G, bool proj);
int split_rows_per_block(int W, int G);
// X, Y, U hold esize-byte residues (2: p <= 2^16, 4: any p).  acc: 1 = int32 sums (p <= 2^16 and
// max row length * max |a| * (p - 1) < 2^31), 2 = 16-bit halves of the residues summed in two int32
// (p > 2^16 and ceil(max row length / G) * max |a| * 65535 < 2^31), 0 = int64 sums.
// pass (32-bit residues only): 0 = whole rows; 1 = first column part, reduced sums to carry (nrows x W,
// no scale, no projection); 2 = second part, carry added before the scale, store and projection.
hipError_t launch_spmm_split(int W, int G, bool proj, int acc, bool smallp, int esize, int64_t nrows,
                             const int32_t* rp, const uint32_t* ent, const void* X, const uint32_t* scale, void* Y,
                             const void* U, uint32_t* partial, int nblocks, ModP mp, hipStream_t st,
                             int pass = 0, uint32_t* carry = nullptr);
}  // namespace bwr

namespace bwr {
// Two-dimensional tiled sparse x block product (spmm_tiled.hip): nrb row blocks of at most R output rows
// (block b holds rows b, b + nrb, ...) accumulated in LDS, the gathered block read slab by slab (C = 2^cb
// block rows per slab) so that a slab stays in an XCD's L2.  Entries: uint32 (local row << (cb + vb)) | (slab column << vb) | (value & (2^vb - 1)), contiguous per
// tile (row block, slab) in that order, tile_ptr[nrb * K + 1].
struct TiledOperand {
    int64_t rows = 0, nrb = 0;
    int K = 0, R = 0, rb = 0, cb = 0, vb = 0;
    const uint32_t* tile_ptr = nullptr;
    const uint32_t* ent = nullptr;
};
// dynamic LDS of one workgroup (accumulators, tile pointers, final projection sums)
size_t tiled_lds_bytes(int W, bool split, bool proj, int R, int K);
int tiled_threads();
// Tiled encoding of a packed operand (rows x cols, int32 row pointers, packed entries with |value| <
// 2^(vb-1)), nrb * R >= rows: cnt and pos hold nrb * K * R (+ 1 for pos) int32, scan_tmp scan_tmp_words(nrb * K * R);
// tile_ptr nrb * K + 1 entries, out nnz entries.
hipError_t launch_tiled_build(int64_t rows, int64_t nrb, const int32_t* rp, const uint32_t* ent, int K, int R,
                              int cb, int vb, int32_t* cnt, int32_t* pos, int32_t* scan_tmp, uint32_t* tile_ptr,
                              uint32_t* out, hipStream_t st);
// Launch shape of a tiled product: grid persistent workgroups (one row block at a time); un (1 .. 4) entries
// each lane takes per pass (their words loaded one pass ahead, their gathers issued one after another).
struct TiledLaunch {
    int grid = 0;
    int un = 4;
};
// Y = scale * (T X) mod p over the tiled operand T.
// split: residues summed as 16-bit halves (required exactly when p > 2^16; the caller guarantees
// max row length * max |a| * 65535 < 2^31), else int32 sums (max row length * max |a| * (p - 1) < 2^31).
// pmode 1: partial[b][i * W + j] (b < grid) = the workgroup's share of sum_r U[r][i] Y[r][j] mod p; pmode 2: of
// sum_r wgt[r] Y[r][i] Y[r][j] (the Gram form of the symmetric projection); pmode 0: no partials.
hipError_t launch_spmm_tiled(const TiledOperand& t, int W, int pmode, bool split, int esize, const void* X,
                             const uint32_t* scale, void* Y, const void* U, const uint32_t* wgt, uint32_t* partial,
                             const TiledLaunch& L, ModP mp, hipStream_t st);
// Raises the dynamic-LDS limit of the kernel that launch_spmm_tiled would launch (done by every launch too;
// call it before a graph capture that will hold the first launch).
hipError_t prepare_spmm_tiled(const TiledOperand& t, int W, int pmode, bool split, int esize);
}  // namespace bwr

namespace bwr {
// Symmetric projection U = V (symmetric.hip).  Weighted Gram partials: partial[b][i W + j] = sum over the rows of
// block b of w[r] X[r][i] X[r][j] mod p for i <= j, 0 for i > j (w null: weight 1; X: esize-byte residues).
hipError_t launch_gram(int W, bool smallp, int64_t n, const void* X, int esize, const uint32_t* w, uint32_t* partial,
                       int nblocks, ModP mp, hipStream_t st);
// S[k][j][i] = S[k][i][j] for i < j (k < nsteps).
hipError_t launch_mirror(int64_t nsteps, int32_t s, uint32_t* S, hipStream_t st);
// *bad |= 1 when some S[k][i][j] != S[k][j][i] (k < nsteps).
hipError_t launch_sym_check(int64_t nsteps, int32_t s, const uint32_t* S, int32_t* bad, hipStream_t st);
// out[r] = d[r]^-power mod p (power 1 or 2), 0 where d[r] = 0 mod p; d null: all 1.
hipError_t launch_inv_diag(int64_t n, const uint32_t* d, ModP mp, int power, uint32_t* out, hipStream_t st);
}  // namespace bwr
