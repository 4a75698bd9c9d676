/*
 * binv.h -- blockwise inversion of partitioned matrices on AMD MI355X (gfx950).
 *
 * The library inverts a non-singular square matrix X partitioned into a k x k
 * grid of blocks whose diagonal blocks are square (Eq. (matx) and the
 * partitioning of §5.1: arbitrary diagonal-block orders m_i with sum m_i = n).
 * It applies Eq. (a) of §3 -- X^-1 from A^-1 and the Schur complement
 * S_A = D - C A^-1 B -- once per diagonal block, in place, exactly as the
 * in-place procedure of §4.2 (invertor_inplace_by_a) does when its recursion
 * is unrolled over the block grid.  For block p:
 *
 *   P      <- W_pp^-1                      pivot-block inversion (the ◊ of
 *                                          Table 3; Gauss-Jordan with partial
 *                                          pivoting inside the block)
 *   W_pj   <- P W_pj,       j != p         row panel  (the -A^-1 B product)
 *   W_ij   <- W_ij - W_ip W_pj, i,j != p   Schur complement / assembly (∼)
 *   W_ip   <- -W_ip P,      i != p         column panel (the -C A^-1 product)
 *   W_pp   <- P
 *
 * which costs 2 b_p n^2 flops per block and exactly 2 n^3 in total.  After
 * the last block W = X^-1.  Like the paper's method, pivoting never crosses
 * block boundaries: a block whose pivot search meets an exact zero makes the
 * call report the matrix as singular (re-partitioning, §3, is the caller's
 * choice).
 *
 * Conventions for every entry point:
 *  - Matrices are row-major float64 in device memory (HBM); `ld*` is the
 *    leading dimension in elements (>= the row length).  A column-major caller
 *    gets the inverse of the transpose, i.e. the transpose of the inverse, and
 *    so a correct inverse too.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *    on it in order; the call returns once the work is enqueued unless
 *    BINV_F_SYNC is set.
 *  - The caller owns and frees every pointer it passes; the library keeps no
 *    reference to them after the enqueued work completes.  Workspace belongs
 *    to the context.  A context must not be used from two host threads at
 *    once, nor on two streams whose work can overlap.
 *  - Functions return a binv_status; binv_last_error() gives a thread-local
 *    message for the last non-OK status.
 */
#ifndef BINV_H
#define BINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BINV_OK = 0,
  BINV_E_INVALID = 1,   /* bad argument (sizes, partition, pointers), or an
                           input matrix holding a NaN or an infinity */
  BINV_E_SINGULAR = 2,  /* an exactly-zero pivot inside a diagonal block */
  BINV_E_NOMEM = 3,     /* device allocation failed */
  BINV_E_NOCONVERGE = 4, /* binv_invert_mixed / binv_poll: the result misses its
                           residual target after the allowed refinement (X
                           still holds the best iterate, info says how close) */
  BINV_E_HIP = 5,       /* a HIP runtime call failed */
  BINV_E_BUSY = 6,      /* binv_poll: the request is not finished yet */
  BINV_E_NOTFOUND = 7   /* binv_poll: unknown (or already collected) ticket */
} binv_status;

typedef enum {
  BINV_PREC_FP64 = 0,       /* plain FP64 blockwise inversion */
  BINV_PREC_MIXED_F32 = 1   /* FP32 sweep + FP64 Newton-Schulz (binv_invert_mixed) */
} binv_prec;

/* Flags for binv_opts.flags. */
#define BINV_F_SYNC 1u    /* synchronize the stream before returning and report
                             BINV_E_SINGULAR from the device-side info word */
#define BINV_F_REFINE_FROM_FP64 8u /* binv_invert_mixed: start the refinement from
                             the plain FP64 sweep instead of the FP32 one */
#define BINV_F_SAMPLED_CHECK 16u /* binv_invert_mixed: accept an iterate on
                             rho estimated from 64 random sign probes (see
                             binv_residual; 4 * 64 * n^2 flops instead of
                             2 n^3) for n >= 192; the full residual is formed
                             only when a Newton-Schulz step needs it */
#define BINV_F_GRAPH 4u  /* capture the call's whole launch sequence in a HIP
                             graph on first use and replay it afterwards.
                             Batched calls: one graph per plan, re-captured
                             when the A, X or info pointers change.
                             binv_invert (one-stream schedule only: with two
                             blocks or more, a call that would use the
                             lookahead, see BINV_F_LOOKAHEAD, gives
                             BINV_E_INVALID): graphs cached in the
                             context (at most 16, least recently used
                             replaced) keyed by n, the leading dimensions, the
                             A, X and info pointers, the flags and the
                             partition; the first call of a key runs eagerly
                             (sizing the workspace), then captures; a key is
                             re-captured when the context's workspace has moved
                             since.  A replay reads A as it is at replay time. */
#define BINV_F_NO_LOOKAHEAD 2u /* run every step on the caller's stream only
                             (the serial schedule). */
#define BINV_F_LOOKAHEAD 64u /* use the lookahead schedule at every order:
                             block p+1's diagonal block is updated first, then
                             block p+1's pivot block is inverted on an internal
                             side stream while the rest of block p's trailing
                             update runs on a second internal stream
                             (CU-masked only if BINV_SIDE_NCU asks for it, see
                             binv_lookahead_cus); the caller's stream waits for
                             both before the call's work ends.  With neither
                             this flag nor BINV_F_NO_LOOKAHEAD the lookahead is
                             used from n = 2048 up (below that the serial
                             schedule measured as fast or faster), and not with
                             BINV_F_PIVOT (serial measured faster); with both,
                             BINV_F_NO_LOOKAHEAD wins.  Results are bitwise
                             identical either way. */

#define BINV_F_PIVOT 32u /* block-row pivoting (binv_invert, and the FP64 sweep of
                             binv_invert_mixed): the b_p rows that form pivot
                             block p are chosen among all rows not yet used as
                             pivots, by tournament selection on the block's
                             columns (strips of 64 columns; leaves of 256
                             consecutive rows, each node keeping the rows that
                             Gauss elimination with partial pivoting picks,
                             four nodes merging into one); the chosen rows take
                             the block's position and a final column
                             permutation undoes the moves.  The row panel is
                             formed by the pivot block's own 64-wide
                             Gauss-Jordan sub-steps instead of a product with
                             its explicit inverse.  This extends the
                             re-blocking remedy of §3 (Eqs. (b) and (c) are
                             Eq. (a) on a block-row permuted matrix) to any
                             non-singular input, the permutation
                             counter-example of §3 included, with the
                             residual of Gauss-Jordan with partial pivoting.
                             Needs every block order <= 2047 and n <= 32768
                             (BINV_E_INVALID otherwise). */

typedef struct {
  int32_t k;            /* number of diagonal blocks when `part` is given */
  const int32_t* part;  /* host array of k diagonal-block orders summing to n,
                           or NULL to use `block` */
  int32_t block;        /* uniform diagonal-block order when part == NULL;
                           the last block takes the remainder; 0 = 512 */
  uint32_t flags;       /* BINV_F_* */
} binv_opts;

typedef struct binv_ctx binv_ctx;

/* Create a context on HIP device `device`.  It owns the panel workspace,
 * which grows to the largest problem seen and is released by binv_destroy. */
binv_status binv_create(binv_ctx** ctx, int device);
binv_status binv_destroy(binv_ctx* ctx);

/* Invert the n x n matrix A (row-major, leading dimension lda) into X
 * (leading dimension ldx).  X == A with ldx == lda inverts in place
 * (§4.2); otherwise A is left unchanged (§4.1's out-of-place form).
 *
 * d_info: optional device pointer to one int64 the call sets to 0, to the
 *         1-based global row of the first pivot (in block order) that was
 *         exactly zero, or to -1 when A holds a NaN or an infinity (checked
 *         as A is copied into X, or in a pass of its own in place); X is then
 *         undefined.  With BINV_F_SYNC the status is BINV_E_SINGULAR or
 *         BINV_E_INVALID in those cases.
 * opts:   may be NULL (uniform blocks of 512, asynchronous).
 * Errors: BINV_E_INVALID for n < 0, ld < n, a partition that does not sum to
 *         n or has a non-positive order, NULL matrices with n > 0, or
 *         overlapping A and X that are not the same matrix. */
binv_status binv_invert(binv_ctx* ctx, int64_t n, const double* A, int64_t lda,
                        double* X, int64_t ldx, const binv_opts* opts,
                        void* stream, int64_t* d_info);

/* Steps [p_begin, p_end) of binv_invert's blockwise sweep, in place on W
 * (n x n, leading dimension ldw, device): the stepid of §5 as a resumable
 * control variable for this sweep.  Step p applies Eq. (a) for diagonal block
 * p (pivot inversion, row panel, Schur update with the column panel), so
 * after steps 0..p the working matrix holds the partial sweep of the leading
 * block L = blocks 0..p (§4.2's in-place procedure, stopped there):
 *   [[ L^-1,       L^-1 B       ],
 *    [ -C L^-1,    D - C L^-1 B ]]   (B, C, D the rest of A)
 * and after step k-1 (k = number of blocks) W = A^-1.  W must hold A before
 * step 0 and exactly the state the previous range left before any later
 * range: the library keeps nothing between calls, so the state may be copied
 * out (to the host, a file) and copied back, to this or another device
 * buffer, and the sweep resumed later.  Results are bitwise those of
 * binv_invert for every way of cutting [0, k) into ranges.  opts as for
 * binv_invert (same partition on every call); BINV_F_PIVOT is rejected (the
 * pivoted sweep's row order would be state too).  p_end < 0 means k.  d_info
 * (optional device int64): set to 0 when p_begin == 0, then the 1-based row of
 * the first exactly-zero pivot (kept across calls); when NULL, an internal
 * word cleared by every call, so only the call's own steps are reported.
 * BINV_F_SYNC: return BINV_E_SINGULAR once that word is set.  Errors: BINV_E_INVALID for a range
 * outside 0 <= p_begin <= p_end <= k and the argument errors of
 * binv_invert. */
binv_status binv_sweep_steps(binv_ctx* ctx, int64_t n, double* W, int64_t ldw, const binv_opts* opts,
                             int32_t p_begin, int32_t p_end, void* stream, int64_t* d_info);

/* Out-of-core inversion: W (n x n, row-major, leading dimension ldw) lives
 * in HOST memory and is inverted in place by binv_invert's blockwise sweep
 * while the device holds only the current block's panels and two slabs of
 * rows, so n may exceed what the device memory holds (§5's design constraint
 * of blocks kept outside memory, with the work done in a predefined sequence
 * of steps).  Step p copies block p's rows and column panel to the device,
 * inverts the pivot block and forms the row panel there, then streams every
 * slab of rows in, applies the trailing update to it and copies it back,
 * alternating two device streams so the copies of one slab overlap the
 * update of the other.  device_bytes bounds the call's device memory:
 * 8 (4 b n + b^2 + 4 (64 b + 4096)) + 256 bytes for the panels (b = the
 * largest block order) plus 16 n bytes per row of slab height (rounded down
 * to a multiple of 128 rows when at least 128); BINV_E_INVALID below one row.
 * The result is bitwise that of binv_invert.  Page-locked host memory
 * (hipHostMalloc) makes the copies asynchronous; pageable memory works too.
 * Synchronous.  *singular_row (may be NULL): 0, or the 1-based row of the
 * first exactly-zero pivot (status BINV_E_SINGULAR; W is then undefined).
 * opts as for binv_invert (BINV_F_GRAPH, BINV_F_LOOKAHEAD and BINV_F_NO_LOOKAHEAD have no
 * effect); BINV_F_PIVOT and blocks of order > 2047 give BINV_E_INVALID.  The
 * host matrix is not checked for NaN or infinity. */
binv_status binv_invert_host(binv_ctx* ctx, int64_t n, double* W, int64_t ldw, const binv_opts* opts,
                             size_t device_bytes, void* stream, int64_t* singular_row);

/* binv_invert for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The same blockwise sweep as binv_invert with BINV_F_NO_LOOKAHEAD (bitwise
 * the same result), on the caller's stream only, whose workspace (the panels
 * and, when d_info is NULL, the info word) is a static 64 MiB array that the
 * library holds on every device it runs on until the process ends.  It calls
 * no hipMalloc, hipFree or other allocating routine and creates no stream or
 * event.  The workspace needed, in doubles, is
 *   32 + 2 b n + b^2 + 512 b + 32768   (b = the largest block order),
 * which must fit in 64 MiB (n = 7168 with b = 512, or
 * n = 16384 with b = 224); larger problems are rejected with BINV_E_INVALID
 * and a message giving the size they need.  Every call on one device shares
 * that device's array, so calls whose work can overlap on one device (two
 * streams, two host threads) race and corrupt each other; the array keeps the
 * last call's contents, and a call writes every element it reads before
 * reading it (the info word is cleared first).  Arguments, the in-place
 * rule, d_info and BINV_F_SYNC are as for binv_invert; BINV_F_PIVOT and
 * blocks of order > 2047 give BINV_E_INVALID; BINV_F_NO_LOOKAHEAD is implied.
 * binv_create looks up each device's copy of the array; BINV_E_HIP if that
 * failed. */
binv_status binv_invert_noalloc(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                                const binv_opts* opts, void* stream, int64_t* d_info);

/* ---------------------------------------------------------------------------
 * Mixed precision: the same blockwise sweep on an FP32 working copy (row
 * panels and Schur updates on FP32 MFMA with FP32 accumulation, every pivot
 * block inverted in FP64), then Newton-Schulz refinement in FP64 on the
 * original matrix, X <- X + X (I - A X), until rho = ||A X - I||_F / sqrt(n)
 * is at most `target`.  FP64 and the device are used for the pivot blocks, the
 * residual I - A X and its norm.
 * --------------------------------------------------------------------------- */
typedef struct {
  double rho;              /* rho of the returned X, computed in FP64 on the GPU */
  double rho_steps[8];     /* rho of each successive iterate: the FP32 sweep's
                              (if it fell back), the starting sweep's, then
                              after each Newton-Schulz step; a last entry not
                              below the one before it is a step that was formed
                              and rejected (X keeps the better iterate) */
  int32_t refine_steps;    /* Newton-Schulz steps accepted into X */
  int32_t fell_back;       /* 1: the FP32 sweep's rho was >= 0.5 (Newton-Schulz
                              would not converge), so the FP64 sweep was used
                              as the starting point */
  int32_t converged;       /* 1: rho <= target */
  int32_t sampled;         /* 1: rho is the random-probe estimate
                              (BINV_F_SAMPLED_CHECK); 0: the full residual */
  int32_t rho_count;       /* entries of rho_steps that were filled */
} binv_info;

/* rho = ||A X - I||_F / sqrt(n) of a given X: the residual norm check (a6 of
 * the hot path) on its own, A and X FP64 row-major on ctx's device.  flags 0:
 * the full residual I - A X (an n x n x n FP64 GEMM, 2 n^3 flops) and its
 * norm.  BINV_RESID_ESTIMATE: the mean of ||(A X - I) z||^2 over 64 random
 * sign vectors z (Hutchinson's estimator of the squared Frobenius norm, as
 * A (X z) - z: two n x n x 64 products), an unbiased estimate of rho^2 whose
 * relative standard deviation is at most sqrt(2/64) however the error is
 * spread over the rows; orders below 192 always take the full residual.  The
 * probes are a fixed function of n, so equal inputs give equal results.
 * Uses ctx's workspace (n^2 doubles); synchronizes `stream` and writes *rho.
 * Errors: BINV_E_INVALID (NULL pointers, n < 0, ld < n, unknown flags). */
#define BINV_RESID_ESTIMATE 1u
#define BINV_RESID_COMPENSATED 2u /* the full residual formed with an error-free
                             split of the operands (Ozaki, Ogita, Oishi and
                             Rump 2012): A split by rows and X by columns into a
                             leading part of (52 - ceil(log2 n)) / 2 bits and
                             the rest, so that I - A1 X1 is exact in FP64 and
                             R = (I - A1 X1) - A2 X1 - A X2 carries rounding
                             errors about 2^-bits of a plain FP64 residual's;
                             three n^3 FP64 GEMMs, 4 n^2 doubles of extra
                             workspace.  binv_invert_mixed always forms its
                             residuals this way. */
binv_status binv_residual(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, const double* X, int64_t ldx,
                          uint32_t flags, void* stream, double* rho);
/* The compensated residual matrix itself: R = I - A X (n x n, ld ldr, device)
 * as binv_residual forms it with BINV_RESID_COMPENSATED, and rho.  Synchronous.
 * Errors: BINV_E_INVALID (NULL pointers, n < 0, ld < n). */
binv_status binv_residual_matrix(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, const double* X,
                                 int64_t ldx, double* R, int64_t ldr, void* stream, double* rho);

/* Invert A (FP64, row-major, lda) into X (ldx); X must not overlap A, which
 * is read again by the refinement.  opts: the partition (as binv_invert) and
 * the flags BINV_F_LOOKAHEAD, BINV_F_NO_LOOKAHEAD, BINV_F_REFINE_FROM_FP64, BINV_F_SAMPLED_CHECK.
 * Refinement stops
 * once rho <= target (target <= 0 means 1e-10), after max_refine steps
 * (< 0 means 5, at most 6), or when rho stops decreasing.  Because the sweep
 * never pivots across diagonal blocks, its error can grow on nonsymmetric
 * inputs; the refinement repairs that whenever the start has rho < 0.5.
 * The call is synchronous: it reads each residual norm back to decide the
 * next step, and fills *info (may be NULL).  Returns BINV_E_INVALID when A
 * holds a NaN or an infinity, BINV_E_SINGULAR for an exactly-zero pivot, and
 * BINV_E_NOCONVERGE when the result misses the target (X then holds the
 * iterate with the smallest rho, reported in info->rho). */
binv_status binv_invert_mixed(binv_ctx* ctx, int64_t n, const double* A, int64_t lda, double* X, int64_t ldx,
                              const binv_opts* opts, double target, int32_t max_refine, void* stream,
                              binv_info* info);

/* ---------------------------------------------------------------------------
 * Batched inversion of many small, uneven matrices.
 *
 * A plan fixes `count` matrices of orders m[i] in 1..256, packed back to back
 * in one buffer: matrix i is row-major with leading dimension m[i] and starts
 * at element sum_{j<i} m[j]^2.  Matrix i is split into k[i] diagonal blocks
 * (k == NULL: one block) whose orders are part[s_i .. s_i + k[i]) with s_i the
 * running sum of k (part == NULL: floor(m/k) each, the remainder added one by
 * one to the last blocks).  Each matrix is inverted by the same blockwise
 * elimination as binv_invert, with pivoting inside its diagonal blocks only;
 * orders up to 192 run in registers, one Gauss-Jordan pass per matrix; blocks
 * larger than 128 of a matrix of order > 192 are split in near-equal pieces
 * of at most 128, and such a matrix is swept block step by block step.  Host
 * arrays are read during binv_batch_create only.  The plan keeps device
 * copies of its tables and a workspace of about (128^2 + 256 m) doubles per
 * matrix of order > 192; it belongs to `ctx`'s
 * device and is released by binv_batch_destroy.
 * Errors: BINV_E_INVALID for an order outside 1..256, k[i] outside 1..m[i] or
 * block orders that do not sum to m[i]; BINV_E_NOMEM.
 * --------------------------------------------------------------------------- */
typedef struct binv_batch binv_batch;

binv_status binv_batch_create(binv_ctx* ctx, int64_t count, const int32_t* m, const int32_t* k,
                              const int32_t* part, binv_batch** plan);
binv_status binv_batch_destroy(binv_batch* plan);

/* Number of matrices, packed elements and algorithmic flops (2 sum m^3). */
binv_status binv_batch_query(const binv_batch* plan, int64_t* count, int64_t* total_elems, double* flops);

/* Invert every matrix of the plan: A and X are device buffers of the plan's
 * packed size (X == A inverts in place; otherwise they must not overlap).
 * d_info: device int32[count]; entry i becomes 0, or the 1-based row (within
 * matrix i) of its first exactly-zero pivot, in which case X's matrix i is
 * undefined.  flags: BINV_F_GRAPH, BINV_F_SYNC.  Stream-ordered on `stream`. */
binv_status binv_invert_batched(binv_batch* plan, const double* A, double* X, int32_t* d_info, uint32_t flags,
                                void* stream);

/* The paper's parallel algorithm (§5) on every matrix of a plan, instead of
 * the blockwise sweep: each matrix's diagonal blocks (a power-of-two count
 * N_k, orders 1..4; binv_level_partition gives the scheme of §5.1) are
 * inverted bottom-up by Eq. (ad) over N_s = 2 N_k - 1 steps whose work the
 * step number fixes (Tables 4 and 5): the closed-form inverses of the
 * diagonal blocks (◊), the products -A^-1 B and -D^-1 C (→, ←), the Schur
 * complements S_A and S_D (∼), which are inverted by the same scheme one
 * level down in the provisional sets of §5.3, and the products with their
 * inverses (↑, ↓).  No pivoting: every diagonal block and Schur complement
 * met must be invertible (SPD inputs guarantee it).  It costs
 * n^3 (3 - 1/N_k) flops for uniform blocks against the sweep's 2 n^3.  One
 * workgroup per matrix with M_inv and the provisional sets on chip; orders
 * are launched in classes (<= 8, 16, 32, 45, 52, 64), one launch each.
 * A, X, d_info and in-place use as for binv_invert_batched; d_info[i] is the
 * 1-based first row of the first block (earliest step, then lowest block)
 * whose determinant was exactly zero.  flags: BINV_F_SYNC (BINV_F_GRAPH is
 * accepted and has no effect: the call is one launch per order class).
 * Errors: BINV_E_INVALID for an order > 64, a block count that is not a
 * power of two, a block order > 4, or the inverse's on-chip part (m^2, or
 * a^2 + d^2 for orders above 32 with a, d the orders of the top level's
 * halves) plus the provisional sets above 19968 doubles (156 KB of LDS; no
 * such partition of an order <= 64 reaches it); checked on the first call,
 * naming the matrix. */
binv_status binv_invert_batched_levels(binv_batch* plan, const double* A, double* X, int32_t* d_info,
                                       uint32_t flags, void* stream);

/* The partition of §5.1 (Table 2): N_k = 2^(floor(log2 m) - 1) diagonal
 * blocks (1 for m < 4) of orders floor(m / N_k), the remainder added one by
 * one to the last blocks, so every order is 2, 3 or 4 for m >= 2.  Writes N_k
 * to *k and, if part is not NULL, the orders to part[0 .. N_k) (capacity:
 * its length).  Host only.  Errors: BINV_E_INVALID for m < 1, k NULL or a
 * capacity below N_k. */
binv_status binv_level_partition(int32_t m, int32_t capacity, int32_t* k, int32_t* part);

/* Autotuner for the register-resident tiers (orders <= 192).  Each tier has
 * several launch shapes (rows per lane, columns per wave, waves per matrix,
 * matrices per workgroup) that compute bitwise-identical results; this call
 * runs every shape of every non-empty tier `reps` times (>= 1) on the plan's
 * own matrices (A -> X, d_info as for binv_invert_batched, which it leaves
 * holding a valid inversion), times each with HIP events on `stream`, and
 * keeps the fastest in the plan.  The choice is also remembered in `ctx` by
 * tier and by the power of two of the tier's matrix count, and plans created
 * later on that context start from it.  Synchronous.  chosen (may be NULL):
 * int32[6], the shape index per tier (-1 for an empty tier); ms (may be
 * NULL): double[6 * 4], the best time of each (tier, shape), 0 when not run
 * (tiers up to orders 8, 16, 32, 64, 128, 192 have 4, 4, 4, 4, 3 and 2
 * shapes; the fifth tier's third shape is its first compiled for two
 * workgroups per CU). */
binv_status binv_batch_tune(binv_batch* plan, const double* A, double* X, int32_t* d_info, int32_t reps,
                            void* stream, int32_t* chosen, double* ms);

/* rho_i = ||A_i X_i - I||_F / sqrt(m_i) of every matrix of the plan, computed
 * in FP64 on the device (one workgroup per matrix, 2 m_i^3 flops) into
 * d_rho[i] (device double[count]).  Stream-ordered; A and X as for
 * binv_invert_batched. */
binv_status binv_batch_residual(binv_batch* plan, const double* A, const double* X, double* d_rho, void* stream);

/* Launch shape of (tier, shape index): {rows per lane, columns per wave,
 * waves per matrix, matrices per workgroup}.  BINV_E_INVALID for an index the
 * tier does not have. */
binv_status binv_batch_shape(int32_t tier, int32_t shape, int32_t out[4]);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of inversion requests of mixed orders.
 *
 * binv_submit copies A (a host or device pointer; the caller may reuse it at
 * once) and returns a ticket; it never waits for other requests.  A device A
 * (complete: the copy is not ordered after the caller's streams, so the
 * caller synchronizes the stream that produced A first)
 * is copied straight into the request's device state when the budget has
 * room at that moment (the memory is charged from then on); otherwise A is
 * staged in host memory until admission.  A scheduler thread admits queued requests in FIFO
 * order while the server's HBM budget (bytes of device memory held for
 * admitted, not yet collected requests, including their working panels) and
 * in-flight limit allow.  Admitted requests of order <= 256 are grouped into
 * rounds of shared batched launches: orders <= 192 one Gauss-Jordan pass each
 * in registers (pivoting over the whole matrix), orders 193..256 swept block
 * step by block step with blocks of at most 128 (one launch per step for
 * every such request of the round); a mixed request that starts from the FP32
 * sweep (see BINV_SERVER_STRICT_PRECISION) and every larger request is
 * inverted by the blockwise sweep on worker threads with their own streams,
 * so their work overlaps on the device: orders >= 4096 one at a time on the
 * first worker (with the lookahead schedule), the others on any worker
 * (BINV_SERVER_WORKERS in the environment sets the worker count, default 2).
 * Every request run by a worker ends with the FP64 residual check against its
 * target (binv_invert_mixed with BINV_F_SAMPLED_CHECK unless the server was
 * created with BINV_SERVER_FULL_CHECK) and is refined only when the check
 * fails; the check asks for half the target (it carries rounding error and,
 * as an estimate, a spread of its own), info->converged reports rho <= target.
 * BINV_PREC_FP64 starts from the FP64 sweep; BINV_PREC_MIXED_F32 from
 * the FP32 sweep under the policy of BINV_SERVER_STRICT_PRECISION below.
 * Requests run in a round are inverted in FP64, then checked on their full
 * residual and refined by up to three Newton-Schulz steps where they miss
 * their target (info->sampled = 0).
 * binv_poll returns BINV_E_BUSY until the request is done; then it copies X
 * (also when the status is BINV_E_NOCONVERGE: the request missed its target
 * and X is its best iterate)
 * (n x n row-major, host or device pointer, may be NULL), fills *info and
 * *times (either may be NULL), releases the request's device memory and
 * forgets the ticket.  A finished request keeps its memory until it is
 * polled; the server then keeps the block for reuse by later requests (at
 * most a quarter of the budget in cached blocks, freed by
 * binv_server_destroy).  Everything the server holds counts against the
 * budget, cached blocks and the workspace of its worker contexts included;
 * to admit a request it frees cached blocks and idle workers' workspace
 * before waiting.  Errors: BINV_E_NOMEM from binv_submit when the request alone
 * exceeds the budget; BINV_E_SINGULAR (and the other codes) from binv_poll
 * for a request that failed.
 * --------------------------------------------------------------------------- */
typedef struct binv_server binv_server;

typedef struct {
  double queue_ms;   /* submit -> admission */
  double total_ms;   /* submit -> result ready (latency) */
} binv_request_times;

#define BINV_SERVER_STRICT_PRECISION 1u /* mixed requests always start from the
                             FP32 sweep (default: only when the target is
                             >= 1e-6, within the FP32 sweep's reach; below
                             that one Newton-Schulz step costs two FP64 GEMMs
                             of the sweep's size, more than the FP64 sweep it
                             would save, so they start from the FP64 sweep) */
#define BINV_SERVER_FULL_CHECK 2u /* gate on the full residual instead of the
                             64-row sampled estimate (BINV_F_SAMPLED_CHECK) */
binv_status binv_server_create(int device, size_t hbm_budget_bytes, int32_t max_inflight, uint32_t flags,
                               binv_server** server);
binv_status binv_submit(binv_server* server, int64_t n, const double* A, int a_is_device, int32_t prec,
                        double target, uint64_t* ticket);
binv_status binv_poll(binv_server* server, uint64_t ticket, double* X, int x_is_device, binv_info* info,
                      binv_request_times* times);
/* Completion queue: the oldest finished, not yet collected ticket (in the
 * order requests finished), waiting up to wait_us microseconds for one;
 * BINV_E_BUSY if none.  The ticket stays valid for binv_poll, which collects
 * it; a ticket collected without this call is skipped here. */
binv_status binv_next_done(binv_server* server, int64_t wait_us, uint64_t* ticket);

/* Device bytes the server holds or has reserved (request blocks of admitted
 * requests and those kept for reuse, the workspace its worker contexts and
 * its small-request round buffers have grown to, and the workspace reserved
 * for requests still running), the most ever held (never above the budget),
 * and requests finished so far.  Any pointer may be NULL. */
binv_status binv_server_stats(binv_server* server, size_t* used_bytes, size_t* peak_bytes, int64_t* completed);
/* Stops the scheduler, lets running requests finish, frees everything. */
binv_status binv_server_destroy(binv_server* server);

/* Per-phase kernel timing, for measurement.  Phases: */
#define BINV_PHASE_PIVOT 0   /* pivot-block inversion (leaf kernels, sub-sweeps) */
#define BINV_PHASE_ROW 1     /* row panel GEMM */
#define BINV_PHASE_SCHUR 2   /* Schur trailing update GEMM (all tiles; under
                                lookahead all but the next block's diagonal
                                block, on the trailing-update stream, which is
                                CU-masked only when CUs are reserved) */
#define BINV_PHASE_OTHER 3   /* copies and panel saves */
#define BINV_PHASE_BAND 4    /* lookahead: Schur update of the next block's
                                diagonal block, before the fork */
#define BINV_PHASE_SMALL 5   /* batched: register-resident tiers (orders <= 192) */
#define BINV_PHASE_TAIL 6    /* lookahead: the part of the trailing update that
                                follows the pivot chain on the side stream */
#define BINV_NPHASE 7

typedef struct {
  double ms[BINV_NPHASE];        /* summed device time of the timed launches */
  int64_t launches[BINV_NPHASE]; /* number of timed launches */
  double flops[BINV_NPHASE];     /* summed algorithmic flops of those launches
                                    (2 K per output element contracted) */
} binv_timing;

/* CUs reserved for the lookahead's pivot chain (creating the lookahead's
 * streams if no call has yet): nres / 8 on each of the 8 XCDs (nres = 8
 * unless BINV_SIDE_NCU says otherwise; 0 there disables the mask), the
 * trailing update's stream being CU-masked to the rest.  0 means no mask: the
 * device refused it or it is disabled, and the pivot chain competes with the
 * trailing update for every CU (the result is the same).  A CU-masked stream
 * holds a hardware queue of its own for the context's lifetime; a process that
 * overlaps work on many streams of its own (as binv_server does) has fewer
 * queues to share while such a context exists.  Errors: BINV_E_INVALID,
 * BINV_E_HIP. */
binv_status binv_lookahead_cus(binv_ctx* ctx, int32_t* reserved);

/* Record a pair of hipEvents around every later launch of the phases whose
 * bit (1 << BINV_PHASE_*) is set in `phase_mask` (0 turns timing off), on the
 * stream that launch runs on.  Top-level launches only: the sub-sweep of a
 * large pivot block counts as one BINV_PHASE_PIVOT interval. */
binv_status binv_set_timing(binv_ctx* ctx, uint32_t phase_mask);

/* Wait for the recorded events, add their intervals to *out (which the caller
 * zeroes first), and forget them. */
binv_status binv_get_timing(binv_ctx* ctx, binv_timing* out);

/* Thread-local description of the last error (never NULL). */
const char* binv_last_error(void);

/* Library version string. */
const char* binv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BINV_H */
