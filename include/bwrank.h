/*
 * bwrank: rank of large sparse integer matrices modulo a prime by the block
 * Wiedemann method, on AMD MI355X (gfx950).
 *
 * Method (Dumas, Elbaz-Vincent, Giorgi, Urbanska, "Parallel computation of the
 * rank of large sparse matrices from algebraic K-theory"):
 *   Section 2.2  the block Wiedemann sequence X A^i Y of s x s matrices;
 *   Section 2.3  preconditioners of the form A^T A and projections by blocks;
 *   Section 2.4  the minimal matrix generator through a sigma-basis (PM-Basis),
 *                polynomial matrix products with FFT primes and the CRT;
 *   Section 2.5  the "Block Wiedemann Rank Algorithm": precondition, compute
 *                S_i = Y^T A~^i Y for i = 0 .. 2n/s + O(1), take the minimal
 *                generator F, return deg det F - codeg det F.
 *   Section 4    (Conclusion, outlook) early termination of the sequence: an option
 *                here (bwr_set_early_termination).
 *
 * Conventions for every entry point:
 *   - Return value 0 (BWR_OK) or a negative error code below; on error nothing
 *     is written to host outputs and bwr_last_error() describes the failure
 *     (thread-local, valid until the next call on the same thread).
 *   - Matrices are CSR with int64 row pointers (m + 1 entries, row_ptr[0] = 0,
 *     non-decreasing, row_ptr[m] = nnz), int32 column indices in [0, n) and
 *     int32 values (any sign; duplicates are summed).  They are read only and
 *     never retained after a call returns.
 *   - Residues are uint32.  Inputs may be any uint32 (they are reduced mod p);
 *     outputs are canonical in [0, p).
 *   - Blocks are row-major: an n x s block X has X[r * s + c].
 *   - "_dev" entry points take device pointers (memory of the current HIP
 *     device) and a hipStream_t passed as void* (NULL = the null stream); they
 *     wait for the work already queued on that stream, run on a library
 *     stream and return when their work has completed.  Every other entry
 *     point takes host pointers.
 *   - The library keeps one non-blocking stream per host thread and device, so
 *     calls made from different host threads run concurrently on the device
 *     (bwr_set_threads must not run while another call is in progress).
 *   - p must be a prime with 3 <= p < 2^31 (BWR_EPRIME otherwise).
 *   - Block sizes s are 1 .. 64.
 */
#ifndef BWRANK_H
#define BWRANK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BWR_OK 0
#define BWR_EINVAL (-1)  /* NULL pointer, bad size, malformed CSR, zero diagonal entry */
#define BWR_EPRIME (-2)  /* p is not a prime in [3, 2^31) */
#define BWR_ENOMEM (-3)  /* device or host allocation failed */
#define BWR_EDEVICE (-4) /* HIP runtime error */
#define BWR_EBUSY (-5)   /* server queue full */
#define BWR_ESHORT (-6)  /* the generator failed on the check terms (sequence too short) */

typedef struct {
    int64_t m, n;            /* rows, columns */
    int64_t nnz;             /* number of stored entries = row_ptr[m] */
    const int64_t* row_ptr;  /* m + 1 */
    const int32_t* col_idx;  /* nnz, 0 <= col < n */
    const int32_t* val;      /* nnz */
} bwr_csr;

/* Timings and sizes of one rank computation (all optional to read). */
typedef struct {
    int64_t rank;         /* the result */
    int64_t nb;           /* dimension B acts on: min(m, n) */
    int32_t s;            /* block size used: min(block, nb) */
    int32_t transposed;   /* 1 when B = D_c A D_r A^T D_c (m < n) */
    int64_t len;          /* sequence terms used for the generator: 2 + ceil(2 nb / s), or the order at which
                           * early termination kept the basis */
    int64_t check_terms;  /* terms past len the generator was verified on */
    int64_t sum_delta;    /* sum of the generator's row degrees */
    double t_encode;      /* seconds: validation and device encoding of A */
    double t_sequence;    /* seconds: the L + check terms on the device */
    double t_sigma;       /* seconds from the end of the sequence to the generator.  On the device when its
                           * leaf fits in LDS (s <= 32), else on the host.  On the device and for L >= 4096
                           * the basis of the earlier orders is computed on a second stream while the
                           * sequence runs (BWR_SIGMA_MIN_CHUNK sets its smallest chunk, 0 disables), so
                           * only the last chunks count here. */
    double t_readout;     /* seconds: check and read-out */
    int32_t sigma_threads;
    int32_t trials;       /* independent draws made (see bwr_set_trials); the other fields describe the draw
                           * that gave the rank, the times are summed over the draws */
    int64_t terms;        /* sequence terms computed: len + check_terms, or more after an early stop
                           * (bwr_set_early_termination) */
} bwr_rank_info;

/* Timings of one batched rank computation. */
typedef struct {
    double t_encode;    /* seconds: upload, validation and encoding of every matrix */
    double t_sequence;  /* wall seconds of the batched phase: sequence steps, with the read-outs of finished
                           jobs overlapped on a pool of host threads (one stream each) */
    double t_sigma;     /* read-out seconds (sigma-basis, check, rank) summed over those threads */
    double t_total;     /* seconds: the whole call */
    int64_t steps;      /* batched steps (one launch per product each) */
    int32_t jobs;       /* (matrix, group of primes) jobs */
    int32_t width;      /* block width of the batch (primes per job x block size, padded) */
    int32_t g1, g2;     /* lanes per row slice of the two products */
    int32_t retries;    /* further draws made by the agreement retry (bwr_set_batch_retry) */
} bwr_batch_info;

/* Library version (major * 10000 + minor * 100 + patch). */
int bwr_version(void);

/* Message for the last non-zero return on this thread ("" if none). */
const char* bwr_last_error(void);

/* 1 if p is a prime in [3, 2^31), else 0 (deterministic Miller-Rabin, bases 2, 7, 61). */
int bwr_is_prime(uint32_t p);

/* Sequence length the rank uses for an nb-dimensional B and block size s:
 * 2 + ceil(2 nb / s) (Section 2.5, step 2: 2n/s + O(1) terms).  -1 if s < 1 or nb < 0. */
int64_t bwr_sequence_length(int64_t nb, int32_t s);

/* Host threads used by the sigma-basis (default: min(hardware threads, 16)). */
int bwr_set_threads(int32_t n);

/* Independent draws per rank computation, 1 .. 64 (default 1), for every rank
 * entry point (bwr_rank_modp, bwr_rank_modp_dev, bwr_rank_modp_batch,
 * bwr_rank_integer, and the server's requests submitted afterwards).  Draw t
 * uses seed + t for U, V, D_r and D_c.  The result of one draw is never above
 * the true rank (Section 2.5: the algorithm errs only by returning less), so
 * the largest result over the draws is kept; a single-matrix computation stops
 * early once a draw reaches min(m, n).  Like bwr_set_threads, it must not run
 * while another call is in progress.  bwr_get_trials returns the setting. */
int bwr_set_trials(int32_t n);
int32_t bwr_get_trials(void);

/* Early termination of the sequence (the outlook of the paper's conclusion,
 * Section 4: the sequence needs about 2 rank / s terms, not 2 min(m, n) / s,
 * when the rank is below min(m, n)).  on = 1 applies to single-matrix ranks
 * (bwr_rank_modp, bwr_rank_modp_dev, bwr_rank_modp_sym(_dev); not
 * bwr_rank_modp_dev_ws, whose generator is computed after the sequence)
 * whose sequence has at least 4096 terms and whose sigma-basis runs on the
 * device: the basis is computed beside the
 * sequence in chunks cut as the terms arrive (max(512, L/32) orders, the
 * first at L/8), and the sequence stops once the generator rows' shifted
 * degrees have not changed over max(128, chunk/8) orders and 4 terms past
 * that order are complete.  The generator of that order is then checked on
 * the 4 terms past it and read out as usual (bwr_rank_info.len is its order,
 * terms the number of terms computed); should that check fail (a stall
 * before the sequence was complete), the draw is made again at the full
 * length.  A stall of that
 * length in a sequence that is not yet complete is a further Monte Carlo
 * event (the check terms past the kept order guard against it).  Off (0) by
 * default.  The matrices that bwr_rank_modp_batch and the server send to
 * their single-matrix lanes use it too; their batched sequences do not, so
 * with it on bwr_rank_modp_batch sends every matrix whose sequence can stop
 * early (at least 4096 terms) to its single-matrix lanes.
 * Returns BWR_EINVAL for other values.
 * Like bwr_set_trials, it must not run while another call is in progress. */
int bwr_set_early_termination(int32_t on);
int32_t bwr_get_early_termination(void);

/* Agreement retry of bwr_rank_modp_batch (and bwr_rank_integer): after the
 * batch, a (matrix, prime) whose rank is below the largest rank of the same
 * matrix at the other primes gets up to n further single-matrix draws (seeds
 * seed + trials, seed + trials + 1, ...), stopping once it reaches that
 * largest rank, and keeps the largest result.  Every draw returns at most the
 * rank mod p (Section 2.5: the error is one-sided), so the result stays a
 * valid Monte Carlo rank mod p; a prime that divides minors of A keeps its
 * lower rank after the n draws.  The draws are made only where the primes
 * disagree, so they cost little beside the batch; with n > 0 a batched rank
 * may exceed bwr_rank_modp's with the same seed.  0 (the default) disables
 * it; n in 0..16, else BWR_EINVAL.  Must not run while another call is in
 * progress. */
int bwr_set_batch_retry(int32_t n);
int32_t bwr_get_batch_retry(void);

/* The random residues the rank draws, from a counter-based SplitMix64
 * (Steele, Lea, Flood 2014): with mix() the SplitMix64 finaliser and
 * gamma = 0x9E3779B97F4A7C15, output(state, i) = mix(state + (i + 1) gamma),
 * key = output(seed, stream) and element i = output(key, i).
 * out[r * s + c] = element(r * s + c) for r < rows, c < s, from stream
 * `stream` (0 = V, 1 = U, 2 = row diagonal, 3 = column diagonal); block
 * entries are h mod p, diagonal entries (diag != 0) 1 + h mod (p - 1).
 * Host computation (the device draws the same values). */
int bwr_random_block(uint64_t seed, int32_t stream, int64_t rows, int32_t s, uint32_t p, int32_t diag,
                     uint32_t* out);

/* The projected sequence (Sections 2.2-2.3): S_k = U^T B^k V mod p for
 * k < len, with B = D_c A^T D_r A D_c (n x n).  d_row (m) and d_col (n) are the
 * diagonals (NULL = identity; d_col entries must be non-zero mod p).  U, V are
 * n x s.  S_out has len * s * s entries: S_out[(k * s + i) * s + j] = S_k[i][j].
 * No transposition: B always acts on GF(p)^n. */
int bwr_sequence(const bwr_csr* A, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                 const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out);

/* Same with every pointer (the CSR arrays included) in device memory. */
int bwr_sequence_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                     const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream);

/* One application of B (the two sparse products and both diagonal scales of
 * a step): Z = D_c A^T D_r A D_c X mod p, X and Z n x s, device memory. */
int bwr_apply_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* X,
                  uint32_t p, int32_t s, uint32_t* Z, void* stream);

/* ---- for callers that cannot allocate -------------------------------------
 * bwr_sequence_dev_noalloc is bwr_sequence_dev for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): every device buffer of the call is carved
 * from a static device array of 256 MiB that the library holds on each GPU
 * it runs on (until the process ends); the call makes no device allocation
 * and instantiates no graph.  Limit: bwr_sequence_workspace(m, n, nnz, s) must
 * not exceed 256 MiB (about 5 M non-zeros at s = 8), else BWR_EINVAL with
 * nothing computed.  Calls on one GPU share its array: they take turns under
 * a lock (calls from several threads on one device run one after another;
 * issued without that lock they would race), and the array keeps the last
 * call's contents, so each call clears what it needs zeroed.  Results equal
 * bwr_sequence_dev's. */
int bwr_sequence_dev_noalloc(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                             const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream);

/* ---- symmetric projection (Section 2.3, block symmetry) -------------------
 * With the symmetric projection U = V the terms S_k = V^T B^k V are symmetric
 * (B = D_c A^T D_r A D_c is symmetric).  bwr_sequence_sym_dev computes them
 * for k < len (V: n x s, device; layouts as bwr_sequence_dev).  gram = 0:
 * each term is formed as (D_c^-1 V)^T X_k like the independent projection
 * and every term is checked to be symmetric on the device (a term that is
 * not: BWR_EDEVICE), a check of the sparse products themselves.  gram = 1:
 * the standard identities S_2k = W_k^T W_k and S_2k+1 = (A D_c W_k)^T D_r
 * (A D_c W_k), W_k = B^k V, give two terms per application of B, so the
 * sequence takes about half the sparse products (the paper does not use
 * them); only the entries i <= j are summed and the others mirrored.
 * bwr_rank_modp_sym(_dev): the rank algorithm (Section 2.5) with this
 * projection (V drawn from the seed as for bwr_rank_modp; draws as set by
 * bwr_set_trials).  The paper notes that the symmetric projection lowers the
 * probability of success; the result is still never above the true rank.
 * When d_row has entries divisible by p the Gram form weighs those rows by
 * 0, which gives the same terms. */
int bwr_sequence_sym_dev(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* V,
                         uint32_t p, int32_t s, int64_t len, int32_t gram, uint32_t* S_out, void* stream);
int bwr_rank_modp_sym(const bwr_csr* A, uint32_t p, int32_t block, uint64_t seed, int32_t gram, int64_t* rank_out,
                      bwr_rank_info* info);
int bwr_rank_modp_sym_dev(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, int32_t gram, void* stream,
                          int64_t* rank_out, bwr_rank_info* info);

/* ---- caller-owned workspace -----------------------------------------------
 * bwr_sequence_dev (Sections 2.2-2.3) and bwr_rank_modp_dev (Section 2.5)
 * with every device buffer of the computation carved from `workspace`, a
 * caller-allocated device region (e.g. a torch tensor) of workspace_bytes,
 * 256-byte aligned: these calls make no device allocation of their own.
 * bwr_sequence_workspace and bwr_rank_workspace return a sufficient size
 * (an upper bound, counted from the buffers the computation carves: the
 * encoded CSR of A and A^T with their relabelled copy, the iterated blocks,
 * the partial sums; for the rank also the draws and the sequence), or 0 for
 * invalid arguments.  Results are identical to the allocating forms.  Inside
 * a workspace the products use the row-split kernels with the heuristic
 * launch plan (no autotuner trials, no tiled encodings) and the rank's
 * sigma-basis runs on the host.  BWR_ENOMEM (nothing computed) if the
 * workspace is too small; BWR_EINVAL if it is NULL or misaligned.  The
 * workspace is the caller's: the call reads and writes it on a library
 * stream after waiting for `stream`, returns once its work is complete, and
 * keeps nothing in it; two calls in flight must not share one workspace. */
size_t bwr_sequence_workspace(int64_t m, int64_t n, int64_t nnz, int32_t s);
/* Device allocations the library has made in this process so far (a count
 * that the workspace forms leave unchanged; for tests and monitoring). */
int64_t bwr_device_allocations(void);
size_t bwr_rank_workspace(int64_t m, int64_t n, int64_t nnz, int32_t block);
int bwr_sequence_dev_ws(const bwr_csr* A_dev, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                        const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* workspace,
                        size_t workspace_bytes, void* stream);
int bwr_rank_modp_dev_ws(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, void* workspace,
                         size_t workspace_bytes, void* stream, int64_t* rank_out, bwr_rank_info* info);

/* ---- a matrix encoded once, for several sequences ------------------------
 * The blackbox of Section 2.3 (B = D_c A^T D_r A D_c) applied many times to
 * one A: bwr_matrix_create_dev validates and encodes the device CSR A once
 * (CSR of A and A^T, rows and columns relabelled by length; the CSR arrays
 * are not retained), and each bwr_matrix_sequence_dev computes
 * S_k = U^T B^k V exactly as bwr_sequence_dev does, without encoding again;
 * the tiled forms of the products that the autotuner picks are built on first
 * use and kept with the matrix.  p: prime the matrix will be used with (only
 * matters when an entry is outside [-127, 127] or a dimension exceeds 2^24:
 * then residues mod p are stored and other primes are refused, BWR_EINVAL).
 * Ownership: the handle owns its device memory until bwr_matrix_destroy,
 * which waits for the device to be idle first.  Sequence calls on one
 * handle may run from several threads at once. */
typedef struct bwr_matrix bwr_matrix;
int bwr_matrix_create_dev(const bwr_csr* A_dev, uint32_t p, void* stream, bwr_matrix** out);
int bwr_matrix_sequence_dev(bwr_matrix* M, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* U,
                            const uint32_t* V, uint32_t p, int32_t s, int64_t len, uint32_t* S_out, void* stream);
/* The symmetric sequence S_k = V^T B^k V of a kept matrix (as bwr_sequence_sym_dev). */
int bwr_matrix_sequence_sym_dev(bwr_matrix* M, const uint32_t* d_row, const uint32_t* d_col, const uint32_t* V,
                                uint32_t p, int32_t s, int64_t len, int32_t gram, uint32_t* S_out, void* stream);
void bwr_matrix_destroy(bwr_matrix* M);

/* Rank of A over GF(p) by the block Wiedemann rank algorithm (Section 2.5):
 * B = D_c A^T D_r A D_c on the smaller side (A and A^T swap when m < n),
 * D_r, D_c, U, V drawn from `seed`, 2 + ceil(2 nb / s) terms plus 4 check
 * terms, sigma-basis generator, rank = deg det F - codeg det F.  Monte Carlo:
 * the result never exceeds the true rank and equals it with high
 * probability.  An all-zero or empty matrix returns 0 without a launch.
 * info may be NULL. */
int bwr_rank_modp(const bwr_csr* A, uint32_t p, int32_t block, uint64_t seed, int64_t* rank_out,
                  bwr_rank_info* info);

/* Same with the CSR arrays in device memory. */
int bwr_rank_modp_dev(const bwr_csr* A_dev, uint32_t p, int32_t block, uint64_t seed, void* stream,
                      int64_t* rank_out, bwr_rank_info* info);

/* Average device time in microseconds (HIP events on `stream`) of the three
 * kernels of one step of the sequence, each launched `iters` times back to
 * back on A (device CSR) with random blocks of width s: us_out[0] = the first
 * sparse product with the row scale (A X, or A^T X when transpose != 0),
 * us_out[1] = the second sparse product with the column scale, us_out[2] =
 * the U^T projection (0 when it is fused into the second product).  If
 * plan_out is not NULL it receives the launch plan the sequence would use:
 * {block width W, row split of the first product, row split of the second,
 * projection fused (0/1), projection blocks, bytes per stored residue,
 * column passes of the first product, column passes of the second, then for
 * each product its two-dimensional tiling: rows per row block (0 = not
 * tiled), log2 of the block rows per slab, workgroups; then for each product
 * the entries each lane of a tiled product takes per pass} (16 int32; row
 * split 0 = the one-row-per-lane kernel).  For measurement; computes nothing
 * the caller keeps. */
int bwr_time_step_kernels_dev(const bwr_csr* A_dev, uint32_t p, int32_t s, int32_t transpose, int32_t iters,
                              void* stream, double* us_out, int32_t* plan_out);

/* Ranks of nmat matrices, each at nprimes primes, with their sequences
 * advanced together: one launch per sparse product per step covers every
 * (matrix, group of primes) job, and the primes of a job share one pass over
 * the matrix (their blocks sit side by side in one block of width
 * primes x block).  Each rank equals bwr_rank_modp(A[j], primes[t], block,
 * seed) exactly: same draws, same sequence, same read-out (unless the
 * agreement retry, bwr_set_batch_retry, raised it with further draws).
 * ranks_out[j * nprimes + t].  Matrices with entries outside [-127, 127] or
 * a dimension above 2^24, and matrices whose side-by-side block (larger
 * dimension x width x bytes per residue) exceeds 2 MB (BWR_BATCH_BLOCK_BYTES),
 * take the single-matrix path, on 2 host threads (BWR_BATCH_SOLO_THREADS; 1
 * when early termination is on, which sends more matrices there) that run
 * beside the batched launches.  When the primes mix 16-bit and larger ones,
 * the 16-bit primes are batched with 16-bit residues and the larger ones take
 * the single-matrix path (BWR_BATCH_SPLIT=0: all primes batched, 32-bit
 * residues).  The sigma-bases of a job's primes run as one batched
 * sigma-basis per prime class (BWR_SIGMA_BATCH=0: one per prime).  info may
 * be NULL. */
int bwr_rank_modp_batch(const bwr_csr* const* A, int32_t nmat, const uint32_t* primes, int32_t nprimes,
                        int32_t block, uint64_t seed, int64_t* ranks_out, bwr_batch_info* info);

/* Rank of A over the integers, probabilistically (Section 2.5): the largest of
 * its ranks modulo the nprimes primes (each in [3, 2^31)), computed as one
 * bwr_rank_modp_batch call.  Each modular rank is at most the rank over Q
 * (Monte Carlo errors are one-sided too), so *rank_out is a lower bound that
 * equals it unless every prime divides every non-zero maximal minor or every
 * solve fails.  ranks_out (nprimes, may be NULL) receives the modular ranks. */
int bwr_rank_integer(const bwr_csr* A, const uint32_t* primes, int32_t nprimes, int32_t block, uint64_t seed,
                     int64_t* rank_out, int64_t* ranks_out);

/* The sequences bwr_rank_modp_batch computes, returned instead of ranked:
 * for matrix j (B on its smaller side, as in bwr_rank_modp) and prime t,
 * S_out[j][(t * len[j] + k) * s * s + i * s + c] = S_k[i][c] for k < len[j],
 * with U, V, D_r, D_c drawn from `seed` as bwr_rank_modp draws them. */
int bwr_sequence_batch(const bwr_csr* const* A, int32_t nmat, const uint32_t* primes, int32_t nprimes, int32_t s,
                       uint64_t seed, const int64_t* len, uint32_t* const* S_out);

/* ---- serving: a continuous-batching rank server ---------------------------
 * A worker thread keeps two batches of sequences running on the current
 * device, each on a stream of its own: requests at primes <= 2^16 (16-bit
 * residues) and the others (32-bit residues).  Each batch advances 64 steps
 * at a time; before queueing an advance the worker waits until the one it
 * queued before has run (BWR_SERVER_AHEAD = K waits for the one queued K
 * advances before, 0 never waits), so a request admitted now starts after at
 * most one advance already on the device.  Submitted requests queue up and
 * join their running batch at the next step
 * boundary while the HBM budget (the summed device bytes of the admitted
 * requests: encoded matrix, blocks and sequence, plus the upload of one being
 * encoded) and the slot count allow.  A finished sequence gets
 * its sigma-basis and read-out and the request is answered; results are
 * identical to bwr_rank_modp(A, p, block, seed).  A request with at least
 * 2^20 non-zeros (BWR_SERVER_SOLO_NNZ; 0 sends every request to the batches)
 * skips the batches: it is ranked by the single-matrix path (autotuned,
 * tiled products) on a lane of its own that runs one such request at a time
 * beside the batches, admitted against the same budget.  Calls on one server
 * are thread-safe. */
typedef struct bwr_server bwr_server;

typedef struct {
    double p50_ms, p99_ms;  /* latency quantiles: answer time - submit time */
    double solves_per_s;    /* answered requests / (last answer - first submit) */
    double busy_s;          /* worker time spent advancing the batch and answering */
    int64_t completed;      /* answered requests */
    int64_t max_queue;      /* largest queue length seen */
    int64_t max_active;     /* largest number of requests in the batch at once */
    int64_t steps;          /* batched steps run */
    int64_t peak_bytes;     /* largest sum, over the requests admitted at once, of their device bytes (encoded
                               matrix, blocks, sequence; plus the upload of one being encoded): at most the
                               budget unless a single request alone was admitted into an idle server */
} bwr_server_stats;

/* Creates a server on the current device (block size 1..32). */
int bwr_server_create(uint64_t hbm_budget_bytes, int32_t max_slots, int32_t block, bwr_server** out);
/* Copies A (host CSR) into host memory and queues the request, with the
 * number of draws bwr_set_trials sets (a request whose best rank so far is
 * below min(m, n) rejoins the queue with the next seed while draws are left).
 * The worker uploads and encodes the matrix when it admits the request, so
 * queued requests hold no device memory.  BWR_ENOMEM if it alone exceeds the
 * budget.  *ticket identifies the request. */
int bwr_server_submit(bwr_server* srv, const bwr_csr* A, uint32_t p, uint64_t seed, uint64_t* ticket);
/* *done = 1 and *rank set once answered (the request's error code otherwise). */
int bwr_server_poll(bwr_server* srv, uint64_t ticket, int32_t* done, int64_t* rank);
/* Blocks until the request is answered. */
int bwr_server_wait(bwr_server* srv, uint64_t ticket, int64_t* rank);
int bwr_server_get_stats(bwr_server* srv, bwr_server_stats* out);
/* Stops the worker (requests still running are abandoned) and frees everything. */
void bwr_server_destroy(bwr_server* srv);

/* Minimal generator of a host sequence S (len x s x s, residues mod p) via
 * the sigma-basis of [S(x); -I] of order len (Section 2.4).  delta_out (s):
 * shifted row degrees; P_out ((max_deg + 1) x s x s, capacity given by
 * P_cap_terms >= len + 1): P_out[(k * s + i) * s + j] = coefficient of x^k in
 * the p-part of generator row i, so that F_i(x) = x^delta_i P_i(1/x)
 * satisfies sum_j F_{i,j} S_{l+j} = 0.  *max_deg_out = max delta. */
int bwr_min_generator(const uint32_t* S, int64_t len, int32_t s, uint32_t p, int64_t* delta_out,
                      uint32_t* P_out, int64_t P_cap_terms, int64_t* max_deg_out);

/* bwr_min_generator on a device sequence S_dev (len x s x s, device memory),
 * with the sigma-basis computed on the device (PM-Basis over NTT/CRT products
 * and M-Basis leaves, s <= 32); delta_out and P_out are host memory. */
int bwr_min_generator_dev(const uint32_t* S_dev, int64_t len, int32_t s, uint32_t p, void* stream,
                          int64_t* delta_out, uint32_t* P_out, int64_t P_cap_terms, int64_t* max_deg_out);

/* bwr_min_generator_dev for n <= 4 device sequences S_dev[b] of one length
 * and block size, sequence b mod p[b], the primes all <= 2^16 or all larger
 * (else BWR_EINVAL): the sigma-bases run as one PM-Basis recursion whose leaf
 * and product launches serve every sequence (Section 2.4; the sequences of
 * one matrix at several primes share their length).  Host outputs per
 * sequence b: delta_out + b s, P_out + b P_cap_terms s s (layout as in
 * bwr_min_generator), max_deg_out[b].  Each result equals
 * bwr_min_generator_dev's for that sequence alone. */
int bwr_min_generators_dev(const uint32_t* const* S_dev, int32_t n, int64_t len, int32_t s, const uint32_t* p,
                           void* stream, int64_t* delta_out, uint32_t* P_out, int64_t P_cap_terms,
                           int64_t* max_deg_out);

/* Rank read-out from a host sequence: generator from the first `len` terms,
 * verified on `check` further terms (S holds len + check terms), then
 * deg det F - codeg det F (Section 2.5, steps 3-4). */
int bwr_rank_from_sequence(const uint32_t* S, int64_t len, int64_t check, int32_t s, uint32_t p,
                           int64_t* rank_out);

/* ---- environment settings ------------------------------------------------
 * Every result is the same under any of these; they select launch plans or
 * turn features off, for measurement and for tests.
 *   BWR_NO_TUNE=1          heuristic launch plans, no autotuner trials
 *   BWR_NO_PLAN_CACHE=1    tune again on every call (plans are otherwise
 *                          kept per matrix shape, width and prime class)
 *   BWR_G1, BWR_G2         lanes per row slice of the first / second product
 *                          (single-matrix path; either one skips tuning)
 *   BWR_E32=1              32-bit residues also for primes <= 2^16
 *   BWR_PARTS=2            two column passes for 32-bit residues;
 *                          BWR_NO_PARTS=1 keeps the tuner from trying them
 *   BWR_NO_O7=1            no 7-wave variant of the fused 8-wide product
 *   BWR_TILED=1            both products in the two-dimensional tiled form
 *                          wherever it applies (no tuning; also used by
 *                          bwr_apply_dev); BWR_TILED=0 keeps the tuner from
 *                          trying it.  BWR_TILED_WGS (workgroups per CU),
 *                          BWR_TILED_SLAB (bytes of the block per slab),
 *                          BWR_TILED_R (row block cap), BWR_TILED_GRID
 *                          (workgroup cap) and BWR_TILED_UN (entries per
 *                          lane per pass, 1-4) pin its geometry;
 *                          BWR_TILED_NO_STAGE=1 makes the fused projection
 *                          load its operands directly instead of staging
 *                          them in LDS
 *   BWR_NO_SORT=1          no length-sorted relabelling of rows and columns
 *   BWR_NO_GRAPH=1         launch every step instead of replaying HIP graphs
 *   BWR_HOST_SIGMA=1       sigma-basis on the host instead of the device
 *   BWR_SIGMA_MIN_CHUNK    see bwr_rank_info.t_sigma
 *   BWR_EARLY_STEP, BWR_EARLY_VERIFY  (tests) the chunk and confirmation
 *                          lengths of early termination; BWR_EARLY_FORCE_AT=c
 *                          keeps the basis at the first cut at or past order
 *                          c, stalled or not.  A generator kept too early
 *                          fails its check, and the draw is then made again
 *                          at the full length
 *   BWR_SIGMA_BATCH, BWR_BATCH_SPLIT, BWR_BATCH_BLOCK_BYTES,
 *   BWR_BATCH_SOLO_THREADS see bwr_rank_modp_batch
 *   BWR_BATCH_G1, BWR_BATCH_G2  lanes per row slice of the batched products
 *   BWR_BATCH_ACC=0        64-bit accumulators in the batched products
 *   BWR_BATCH_BLOCKS       persistent blocks of the batched second product
 *                          (default 2048)
 *   BWR_BATCH_CHUNK        steps per batched graph (even, default 64)
 *   BWR_READOUT_THREADS    host threads reading out finished batched or
 *                          served sequences (default 3)
 *   BWR_SERVER_AHEAD, BWR_SERVER_SOLO_NNZ  see the serving section
 *   BWR_SERVER_FAIL_ADVANCE=k  (tests of error handling) the server's
 *                          advance after k advances reports an error instead
 *                          of launching, once; the requests in its batches
 *                          are answered with that error */

#ifdef __cplusplus
}
#endif

#endif /* BWRANK_H */
