/*
 * lpcg.h -- C ABI of the learned-preconditioner PCG library (liblpcg.so) for
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves sparse SPD systems A x = b from discretised second-order
 * PDEs (paper: Preliminaries, "Discretization") with preconditioned conjugate
 * gradient (Appendix, algorithm "PCG") and the preconditioner P = L L^T, where
 * L is lower triangular on the pattern of tril(A) (Method, "Learning
 * Preconditioners").  L comes from a message-passing GNN over the matrix graph
 * (Method, "Architecture"; technical-details appendix) or from the IC(0) and
 * Jacobi baselines (Experiments, baselines).  Training-side entry points give
 * the data loss sum ||L L^T x - b||^2 (Method, equation loss_Ab), its gradient,
 * the network's reverse mode and an Adam step.
 *
 * Conventions for every entry point
 *  - All array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 *    tensors) unless a comment says "host".  The caller owns them.
 *  - Indices are int32; CSR rows have ascending, unique column indices and the
 *    diagonal stored; the pattern must be structurally symmetric.
 *  - Work is enqueued on the given stream.  Entry points documented as
 *    "synchronous" wait for their stream before returning; the others return
 *    as soon as the work is enqueued.
 *  - Return value: LPCG_OK or one of the LPCG_E* codes below; a message is
 *    available from lpcg_last_error() (thread-local).  No C++ exception ever
 *    crosses this interface and the library never aborts the process.
 *  - L is stored in lower CSR order (rows ascending, columns ascending, the
 *    diagonal last in each row), FP32.  "Ut" denotes the same values in the
 *    CSR order of U = L^T (rows ascending, diagonal first).
 */
#ifndef LPCG_H
#define LPCG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- status */
#define LPCG_OK          0
#define LPCG_EINVAL      1  /* bad argument / pattern (unsorted, no diagonal, not symmetric) */
#define LPCG_EHIP        2  /* a HIP runtime call failed */
#define LPCG_ENOTCONV    3  /* PCG hit maxit; x holds the last iterate */
#define LPCG_EBREAKDOWN  4  /* PCG p^T A p <= 0 or non-finite; IC(0) pivot <= 0 */
#define LPCG_ENONFINITE  5  /* a predicted factor has a non-finite or non-positive diagonal */
#define LPCG_ENOMEM      6  /* device allocation failed / workspace too small */

/* Message of the last failing call on this thread ("" if none). */
const char *lpcg_last_error(void);
/* Library version string. */
const char *lpcg_version(void);

/* ------------------------------------------------------------- matrices */
/* Sparse square matrix in CSR, device pointers.  val may be NULL where only
 * the pattern is needed. */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *rowptr; /* [n+1] */
    const int32_t *colind; /* [nnz] */
    const double *val;     /* [nnz] FP64 */
} lpcg_csr;

/* Opaque handle: one sparsity pattern (possibly a block-diagonal batch of
 * independent systems), its derived structure, a copy of A's values and the
 * solver's work vectors.  Owned by the library. */
typedef struct lpcg_system lpcg_system;

typedef struct {
    int32_t n, nnz, nnz_l;       /* nnz_l = stored entries of tril(A) */
    int32_t nlev_fwd, nlev_bwd;  /* level counts of the L and L^T solves */
    int32_t max_width_fwd, max_width_bwd; /* largest level */
    int32_t nsys;                /* systems in the batch (1 if not batched) */
    int32_t ordering;            /* LPCG_ORDER_* the system was analysed with */
    int32_t ncolors;             /* colours of LPCG_ORDER_COLOR (0 otherwise) */
} lpcg_info;

/* Row orderings.  NATURAL keeps A's numbering (the factor lives on tril(A)).
 * COLOR renumbers the rows before everything else: first-fit colouring in
 * row order on the lower-triangle graph (colour(i) = smallest colour no
 * neighbour j < i has), then rows sorted by (system of the batch, colour),
 * ascending inside a colour.  The library then works on P A P^T: the factor
 * lives on tril(P A P^T) and each triangular solve has at most as many
 * levels as there are colours (2, red-black, on grid graphs).  This is a
 * solver-side choice outside the paper; it changes the preconditioner that a
 * given factor pattern can express, not the system solved.
 *
 * Numbering contract for a COLOR system: vectors indexed by rows of the
 * problem (b, x, the x/y of lpcg_spmv, the rhs/y of lpcg_sptrsv, x and b of
 * lpcg_llt_loss) are in the caller's ORIGINAL numbering and are permuted
 * inside the library; preconditioner data (l_val, ut_val, dinv, every array
 * of lpcg_export_pattern) is in the INTERNAL numbering; lpcg_export_perm
 * gives perm[internal row] = original row.  The timing aids work in the
 * internal numbering.
 *
 * COLOR takes at most LPCG_COLOR_MAX_ROWS rows (all systems of a batch
 * together): the largest colour analysis that has been run and verified.  A
 * larger one is refused with EINVAL until it has been. */
#define LPCG_ORDER_NATURAL 0
#define LPCG_ORDER_COLOR   1
#define LPCG_COLOR_MAX_ROWS 262144

/* Pattern analysis (graph/matrix duality of the Method section; levels of
 * the substitution DAG): copies A, builds tril(A) (lrowptr/lcol), U = L^T
 * (urowptr/ucol and the map from U entries to L entries), the reverse-edge map
 * rev[k] = position of (j,i) for entry k = (i,j), the forward and backward
 * levels (longest-path depth) and the level sets (rows ascending inside a
 * level).  A->val must be set.  sys_rowptr (HOST, nsys+1 entries, first 0, last
 * n) splits a block-diagonal batch into independent systems; NULL or nsys <= 1
 * means one system.  ordering: LPCG_ORDER_NATURAL or LPCG_ORDER_COLOR (rows
 * of one system stay inside that system's row range).  Synchronous.  *out is
 * owned by the caller until lpcg_destroy.  Errors: EINVAL (n <= 0,
 * unsorted/duplicate columns, missing diagonal, unsymmetric pattern, a row
 * crossing a system boundary, unknown ordering, COLOR with more than
 * LPCG_COLOR_MAX_ROWS rows), ENOMEM, EHIP. */
int lpcg_analyze(const lpcg_csr *A, const int32_t *sys_rowptr, int32_t nsys,
                 int32_t ordering, lpcg_system **out, hipStream_t stream);

/* perm[internal row] = original row, device int32 [n] (the identity for the
 * natural ordering). */
int lpcg_export_perm(const lpcg_system *sys, int32_t *perm, hipStream_t stream);

/* Replace A's values (same pattern), FP64 device array of length nnz, in the
 * caller's CSR entry order. */
int lpcg_update_values(lpcg_system *sys, const double *val, hipStream_t stream);

/* Sizes and level counts (host struct). */
int lpcg_get_info(const lpcg_system *sys, lpcg_info *info);

/* Copies of the derived integer structure for inspection; every pointer is a
 * device array of the documented length or NULL to skip.  lsrc[nnz_l]: A
 * position of each L entry; u2l[nnz_l]: L position of each U entry;
 * levels[n]; lev_ptr[nlev+1]; lev_rows[n]. */
int lpcg_export_pattern(const lpcg_system *sys,
                        int32_t *lrowptr, int32_t *lcol, int32_t *lsrc,
                        int32_t *urowptr, int32_t *ucol, int32_t *u2l,
                        int32_t *rev,
                        int32_t *flevel, int32_t *flev_ptr, int32_t *flev_rows,
                        int32_t *blevel, int32_t *blev_ptr, int32_t *blev_rows,
                        hipStream_t stream);

void lpcg_destroy(lpcg_system *sys);

/* ----------------------------------------------------- building blocks */
/* y = A x (Appendix PCG, "w = A p"; Method: one round of message passing).
 * prec = 32: x, y FP32 with FP32 values; prec = 64: FP64 throughout. */
int lpcg_spmv(const lpcg_system *sys, int32_t prec, const void *x, void *y,
              hipStream_t stream);

/* Triangular solve with the factor of P = L L^T (Appendix PCG, "Solve P z =
 * r"): transpose = 0 solves L y = rhs (forward), transpose = 1 solves
 * L^T y = rhs (backward) using ut_val.  FP32.  rhs and y must not alias. */
int lpcg_sptrsv(const lpcg_system *sys, int32_t transpose, const float *l_val,
                const float *ut_val, const float *rhs, float *y, hipStream_t stream);

/* Ut values from L values (gather through the U->L map). */
int lpcg_l_to_ut(const lpcg_system *sys, const float *l_val, float *ut_val,
                 hipStream_t stream);

/* Validation of a factor before it is used as a preconditioner (the host
 * policy around a learned factor: fall back to IC(0) or Jacobi when it
 * fails): every diagonal entry of L must be a positive finite number and
 * every other entry finite.  l_val: device FP32 [nnz_l], L order.  *bad_row
 * (HOST, may be NULL): the first offending row in the internal numbering, or
 * -1.  Synchronous.  Errors: ENONFINITE (a row fails), EINVAL.
 * lpcg_gnn_predict_L itself is asynchronous and does not check. */
int lpcg_check_factor(const lpcg_system *sys, const float *l_val, int32_t *bad_row,
                      hipStream_t stream);

/* Symmetric Gauss-Seidel (Experiments, baseline methods; the triangles
 * come from A itself, taken in the symmetric form CG needs):
 * P = (D + A_<) D^-1 (D + A_<)^T = L L^T with L_ij = A_ij / sqrt(A_jj) on
 * tril(A) (sqrt(A_ii) on the diagonal), computed in FP64 and stored FP32 to
 * l_val and/or ut_val (either may be NULL, not both).  Asynchronous on
 * stream.  Errors: EINVAL. */
int lpcg_sgs(const lpcg_system *sys, float *l_val, float *ut_val, hipStream_t stream);

/* IC(0) (Experiments, incomplete Cholesky baseline): L on tril(A) with
 * (L L^T)_ij = A_ij on the pattern, computed in FP64 and stored FP32 to l_val
 * and ut_val.  On a pivot <= 0 the factorisation is retried on
 * A + shift * diag(A) with shift = shift0 (or 1e-3 if shift0 == 0), doubling,
 * at most max_retries times; *shift_used (host, may be NULL) receives the
 * shift of the returned factor.  Synchronous.  Errors: EBREAKDOWN after the
 * last retry. */
int lpcg_ic0(const lpcg_system *sys, double shift0, int32_t max_retries,
             float *l_val, float *ut_val, double *shift_used, hipStream_t stream);

/* No-allocation variant of lpcg_ic0, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): same arguments, same results bit
 * for bit, same errors, but the FP64 working copy of the factor lives in a
 * library-owned device array of LPCG_IC0_NOALLOC_MAX_NNZ_L doubles (16 MiB)
 * instead of a per-call hipMallocAsync.  Every device the library runs on
 * holds its own array until the process ends.  Calls that overlap on one
 * device (several streams or threads) share that array and race; serialise
 * them.  The array keeps the last call's contents; each call presets the
 * entries it uses.  The system itself (lpcg_analyze) is allocated at set-up
 * as for every other entry point.  Synchronous.  Errors: as lpcg_ic0, plus
 * EINVAL when nnz_l exceeds LPCG_IC0_NOALLOC_MAX_NNZ_L. */
#define LPCG_IC0_NOALLOC_MAX_NNZ_L 2097152
int lpcg_ic0_noalloc(const lpcg_system *sys, double shift0, int32_t max_retries,
                     float *l_val, float *ut_val, double *shift_used, hipStream_t stream);

/* Jacobi (Experiments baseline): dinv = 1 / diag(A), FP32 [n]. */
int lpcg_jacobi(const lpcg_system *sys, float *dinv, hipStream_t stream);

/* Timing aids for roofline measurements.  lpcg_time_sptrsv launches the
 * forward (transpose = 0) or backward substitution kernel reps times on
 * `stream`, presetting y before each launch outside the timed interval, and
 * writes to *ms_out (host) the mean duration of one substitution launch
 * measured with HIP events recorded around each launch on the same stream.
 * lpcg_time_spmv does the same for the FP32 SpMV y = A x.  Synchronous. */
int lpcg_time_sptrsv(const lpcg_system *sys, int32_t transpose, const float *l_val,
                     const float *ut_val, const float *rhs, float *y, int32_t reps,
                     double *ms_out, hipStream_t stream);
int lpcg_time_spmv(const lpcg_system *sys, const float *x, float *y, int32_t reps,
                   double *ms_out, hipStream_t stream);

/* ------------------------------------------------------------ tuning */
/* Configuration of one substitution direction.  mode 0: dependency driven
 * (one launch; rows handed to `waves` waves in level order, each row polls
 * its dependencies' ready flags, sleeping `backoff` rounds between polls);
 * mode 1: level synchronous (one launch per level, a few lanes per row, no
 * polling); mode 2: single workgroup (one block of 1024 threads walks every
 * level with block barriers, on a level-ordered copy of the factor that is
 * prepared once per factor; only for systems whose widest level has at most
 * 3072 rows); mode 3: blocked (one wave per block of rows, its in-block
 * dependencies in LDS; block_rows, block_runs).  A new system uses mode 1
 * when the direction has at most 16 levels, mode 0 with 4096 waves and
 * backoff 1 otherwise. */
typedef struct {
    int32_t direction;     /* 0: forward (L y = r), 1: backward (L^T z = y); 2: the SpMV,
                              mode = lanes per row (1: ELL form), waves = blocks */
    int32_t mode;          /* 0 dependency driven, 1 level synchronous, 2 single workgroup,
                              3 blocked (one wave per block of block_rows rows, consecutive
                              or banded (block_runs); dependencies inside a block through
                              LDS, on earlier blocks polled; rows with at most 7
                              dependencies) */
    int32_t waves;         /* mode 0: waves launched (0 = default) */
    int32_t backoff;       /* modes 0 and 3: sleep rounds between polls (0..64) */
    int32_t block_stride;  /* mode 0: only blocks whose index is a multiple of this
                              (1, 2, 4 or 8) work; with the hardware's round-robin
                              dispatch over the 8 XCDs, 8 keeps every working wave
                              on one XCD (one L2).  mode 3: 8 runs only the waves that
                              the hardware reports on XCD 0 (its XCC_ID register), so
                              all exchanges stay in one L2; other values: every wave.
                              0 means 1. */
    int32_t block_rows;    /* mode 3: rows per block (64 .. 65536; 0 = 1024); the
                              schedule is built on the host when the configuration is set
                              (synchronous).  Direction 2 (the SpMV): 0 = the gather form;
                              R >= 64 = the LDS-staged form, one block of 256 threads per
                              R consecutive rows, each block copying the input over its
                              rows' off-diagonal column window into LDS (windows computed
                              on the device when set, synchronous; EINVAL when a window
                              exceeds 16384 inputs or n / R exceeds 2048 blocks).  Both
                              forms sum a row's entries in the same order: same result bit
                              for bit */
    double us;             /* lpcg_autotune: mean duration of one solve */
    int32_t block_runs;    /* mode 3: 1 (or 0): a block is block_rows consecutive rows.
                              K > 1: banded, K runs of block_rows / K consecutive rows
                              (a power of two), one stride D apart, D = the pattern's
                              longest dependency offset (one plane of a natural-order
                              grid); the rows must tile into such blocks (n a multiple of
                              K D, D a multiple of the run) and every dependency on
                              another block must point to an earlier block in solve
                              order, else EINVAL */
} lpcg_trsv_cfg;

/* Schedule of the blocked substitution (mode 3), computed on the host from
 * a triangular CSR pattern, exactly as the library builds it for a system:
 * for inspection and tests.  rowptr/col: HOST, n rows, the pattern of L
 * (upper = 0: columns ascending, diagonal last, rows solved ascending) or of
 * U = L^T (upper = 1: diagonal first, rows solved descending).  Rows are cut
 * into blocks of block_rows rows in solve order: consecutive rows
 * (block_runs <= 1), or banded in block_runs runs as lpcg_trsv_cfg
 * describes.  A block's positions 0 .. nr-1 map to its rows ascending
 * (run_shift, run_stride below).  Inside a block the rows are ordered by
 * their level over in-block dependencies and cut into chunks of at most 64
 * rows of one level.  Call once with the five arrays NULL to get the sizes,
 * then with caller-owned HOST arrays of
 *   brow[2 nblocks]      first (smallest) row, row count of each block
 *   bch[nblocks + 1]     chunk range of each block
 *   chunks[2 nchunks]    first record (schedule position in the block) and
 *                        row count of each chunk
 *   rec[n (2 deps + 2)]  record p of block b at row position map(b, p): deps
 *                        dependency codes in CSR order (>= 0 row of an
 *                        earlier block, -1 none, <= -2 in-block row at
 *                        position -2 - code), the row's position, then
 *                        deps + 1 value words (filled on the device per
 *                        factor; 0 here)
 *   vsrc[n (deps + 1)]   position in the CSR value array of each value and,
 *                        last, of the diagonal (-1: none).
 * deps is 3 or 7.  Errors: EINVAL (block_rows outside [64, 65536], a row with
 * more than 7 dependencies, the LDS bound of the device kernel exceeded,
 * banded blocks that do not tile the rows or are not in dependency order,
 * arrays sized for another schedule). */
typedef struct {
    int32_t deps, nblocks, nchunks, max_chunks;
    int32_t *brow, *bch, *chunks, *rec, *vsrc;
    int32_t run_shift, run_stride;  /* out: position x of block b is the row
                                       brow[2b] + (x >> run_shift) * run_stride
                                       + (x & ((1 << run_shift) - 1)) */
} lpcg_blk_schedule;

int lpcg_blocked_schedule(int32_t n, const int32_t *rowptr, const int32_t *col, int32_t upper,
                          int32_t block_rows, int32_t block_runs, lpcg_blk_schedule *out);

/* Autotuner: times every candidate configuration of both substitution
 * directions on this system with the given factor (reps timed runs after
 * one warm-up, HIP events on `stream`): levels (few levels only), single
 * workgroup (narrow levels only), blocked with 512, 1024, 2048 consecutive
 * rows and banded with 1024, 2048 rows in 2, 4, 8 runs (where the rows
 * tile), and dependency driven with 64 .. 4096 waves.  It keeps the fastest
 * per direction for every later call on the system (on a two-level system,
 * a red-black grid in colour order, it keeps the level mode in both
 * directions, which lets the PCG apply L L^T in two fused launches; where
 * the rows of both halves hold at most 8 entries that pair runs in an ELL
 * form that also performs the iteration's x, r update).  It then times the
 * PCG's product kernel (p = z + beta p_prev, w = A p, p.w; median of three
 * batches of reps back-to-back launches)
 * for G = 4, 8, 16, 32, 64 lanes per row (64 / G rows per wavefront) on
 * grids of up to 512, 1024 and 2048 blocks, the LDS-staged form with 256,
 * 512 and 1024 rows per block at G = 4 and 8 (where the windows fit), and
 * the ELL form (G = 1: one row per lane, for single systems whose rows hold
 * at most 8 entries), and keeps the fastest for the PCG's product and the
 * FP32 lpcg_spmv (the ELL form unless another is at least 10% faster; the
 * FP64 product keeps the fastest gather form); those
 * table entries have direction 2, mode = G, waves = blocks and block_rows
 * (0 for the gather and ELL forms).  It writes up to table_len measured
 * candidates to table (HOST, may be NULL) and their number to *n_table
 * (HOST, may be NULL).  Uses the system's work vectors: not concurrent with
 * a solve on the same system.  Synchronous. */
int lpcg_autotune(lpcg_system *sys, const float *l_val, const float *ut_val, int32_t reps,
                  lpcg_trsv_cfg *table, int32_t table_len, int32_t *n_table, hipStream_t stream);

/* Read / force the configuration of one direction (HOST struct; `us` is
 * ignored).  Direction 2 is the SpMV: mode = lanes per row (4, 8, 16, 32 or
 * 64), waves = blocks of 256 threads (1 .. 2048) of the gather form, or
 * block_rows = R > 0 for the LDS-staged form (waves then reads back as its
 * block count; a refused R leaves the previous form in force), or mode 1 for
 * the ELL form (single systems whose rows hold at most 8 entries, else
 * EINVAL; waves and block_rows ignored, the gather form's settings kept for
 * the FP64 product).  Errors: EINVAL for an
 * unknown direction, mode, a backoff outside
 * 0..64, a block_stride other than 0, 1, 2, 4, 8, mode 2 on a system with
 * a level wider than 3072 rows, or a mode-3 block shape the pattern does not
 * allow (the previous configuration then stays in force). */
int lpcg_get_trsv_cfg(const lpcg_system *sys, int32_t direction, lpcg_trsv_cfg *out);
int lpcg_set_trsv_cfg(lpcg_system *sys, const lpcg_trsv_cfg *cfg);

/* ------------------------------------------------------------------ PCG */
#define LPCG_PC_NONE   0
#define LPCG_PC_JACOBI 1
#define LPCG_PC_LLT    2

typedef struct {
    int32_t kind;          /* LPCG_PC_* */
    const float *l_val;    /* LLT: [nnz_l] lower CSR order */
    const float *ut_val;   /* LLT: [nnz_l] U CSR order */
    const float *dinv;     /* JACOBI: [n] (NULL: computed internally) */
} lpcg_precond;

typedef struct {
    double tol;            /* stop when ||r_k||_2 <= tol * ||b||_2 */
    int32_t maxit;         /* iteration cap (<= 0: n) */
    int32_t check_every;   /* iterations per host check of the done flag; <= 0:
                              lpcg_pcg_solve without a graph sizes each chunk
                              from the recorded residual's decay, extrapolated
                              to tol (8 for the first chunk, for graphs and for
                              the batched solver) */
    int32_t max_restarts;  /* restarts from the FP64 true residual when the
                              recursive residual converged but the true one
                              did not (<= 0: none) */
    int32_t use_graph;     /* capture the iteration chunk in a hipGraph */
} lpcg_solve_opts;

typedef struct {
    int32_t iters;         /* products A p (k of the algorithm), all restarts */
    int32_t status;        /* LPCG_OK / ENOTCONV / EBREAKDOWN */
    int32_t restarts;
    int32_t reserved;
    double relres_rec;     /* recursive ||r_k|| / ||b|| at exit */
    double relres_true;    /* FP64 ||b - A x|| / ||b|| at exit */
} lpcg_result;

/* PCG (Appendix algorithm) on A x = b.  b: FP64 [n]; x: FP64 [n], holds x0 on
 * entry and the solution on return.  Vectors r, p, w, z live in FP32, the
 * products r.z and p.w and the norms are accumulated in FP64, the true
 * residual is FP64.  res (HOST) receives the outcome.  hist (device FP64
 * [maxit+1] or NULL) receives ||r_k||/||b|| for k = 0..iters of the last
 * restart.  coef (device FP64 [2 (maxit+1)] or NULL) receives alpha_k at
 * coef[2k] and beta_k at coef[2k+1] of the last restart (for
 * lpcg_lanczos_extremes).  Synchronous.  Returns res->status. */
int lpcg_pcg_solve(lpcg_system *sys, const lpcg_precond *P, const double *b,
                   double *x, const lpcg_solve_opts *opts, lpcg_result *res,
                   double *hist, double *coef, hipStream_t stream);

/* The rule lpcg_pcg_solve (check_every <= 0, no graph) uses to size its next
 * chunk of iterations, for callers that drive their own loop and for tests.
 * it, res: the last recorded iteration and its ||r||^2 / ||b||^2; prev_it,
 * prev_res: the same at the previous look (0 and ||r0||^2 / ||b||^2 at the
 * first).  The decay rate of log(res) between the two looks is extrapolated
 * to tol^2, shortened by 15%, capped at four times (it - prev_it) and at
 * maxit - it + 1, at least 1; without a decay (it <= prev_it, res or
 * prev_res not positive and finite, no decrease) the answer is 8; tol = 0
 * gives the cap.
 * *predicted_final (may be NULL): 1 when the chunk is expected to reach tol
 * (the solver then appends the FP64 true residual).  Host-only, no GPU. */
int32_t lpcg_next_chunk(int32_t it, float res, int32_t prev_it, float prev_res, double tol, int32_t maxit,
                        int32_t *predicted_final);

/* Timing aid for the PCG iteration's own kernels: from x = 0 and right-hand
 * side b (device FP64 [n], caller's numbering) with preconditioner P, the
 * iteration runs `reps` times after one warm-up, launched eagerly in its
 * three parts with HIP events between them on `stream`: out_us (HOST, 3)
 * receives the mean duration in microseconds of [0] the application
 * z = (L L^T)^-1 r (LLT only; 0 otherwise), [1] the SpMV w = A p with
 * p = z + beta p_prev and the p.w reduction, [2] the x, r update with
 * ||r||^2 (0 where the application performs it: the ELL form of the
 * two-level pair, whose launches then also carry that update from the second
 * round on).  The iteration never converges (tolerance 0).  Synchronous; uses
 * the system's work vectors (not concurrent with a solve on the system).
 * Errors: EINVAL. */
int lpcg_time_pcg_kernels(lpcg_system *sys, const lpcg_precond *P, const double *b, int32_t reps,
                          double *out_us, hipStream_t stream);

/* Condition-number estimate of the preconditioned operator (appendix
 * "Condition Number Comparison"): extreme eigenvalues of the CG-Lanczos
 * tridiagonal built from k iterations' coefficients (HOST coef as written by
 * lpcg_pcg_solve: coef[2i] = alpha_i, coef[2i+1] = beta_i), by Sturm-count
 * bisection.  kappa ~ lmax / lmin.  Errors: EINVAL (k < 1, alpha <= 0). */
int lpcg_lanczos_extremes(const double *coef, int32_t k, double *lmin, double *lmax);

/* Batched PCG: one PCG (Appendix algorithm) per system of a block-diagonal
 * batch (lpcg_analyze with sys_rowptr), each with its own alpha, beta,
 * residual test (||r_s|| <= tol ||b_s||), iteration count and status; all
 * systems advance in the same launches and a finished system stops updating.
 * b, x: FP64 [n] for the whole batch (x holds x0 on entry).  res: HOST array
 * of nsys results, in system order (restarts from the FP64 true residual as
 * in lpcg_pcg_solve, per system).  hist is not recorded.  Synchronous.
 * Returns LPCG_OK when every system converged, else the first failing
 * system's status. */
int lpcg_pcg_solve_batched(lpcg_system *sys, const lpcg_precond *P, const double *b,
                           double *x, const lpcg_solve_opts *opts, lpcg_result *res,
                           hipStream_t stream);

/* FP64 iterative refinement around the FP32 batched PCG, for every system of
 * the batch (a single system is a batch of one): r = b - A x in FP64; systems
 * with ||r|| <= tol ||b|| are done; the others solve A d = r with the inner
 * PCG to tol_inner (inner->tol is ignored) and take x += d; at most max_outer
 * refinement steps.  res (HOST, nsys): iters = inner iterations summed,
 * restarts = refinement steps taken, relres_true = final FP64 relative
 * residual, status LPCG_OK when it is <= tol (else ENOTCONV, or EBREAKDOWN
 * from an inner solve).  Synchronous. */
int lpcg_pcg_solve_ir(lpcg_system *sys, const lpcg_precond *P, const double *b, double *x,
                      double tol, double tol_inner, int32_t max_outer,
                      const lpcg_solve_opts *inner, lpcg_result *res, hipStream_t stream);

/* ------------------------------------------------------------------ GNN */
/* Encoder-processor-decoder GNN (Method "Architecture"; technical-details
 * appendix), latent and hidden width h (multiple of 16, at most 64), n_mp
 * message-passing layers.  params: FP32 master weights, device, in this order
 * (each Linear maps x -> x W + b, W stored [fan_in][fan_out] row-major):
 *   node_enc: W0[1][h] b0[h] W1[h][h] b1[h]
 *   edge_enc: W0[1][h] b0[h] W1[h][h] b1[h]
 *   for t in 0..n_mp-1:
 *     mp{t}.node: W0[2h][h] b0[h] W1[h][h] b1[h]     (input [v_i, m_i])
 *     mp{t}.edge: W0[3h][h] b0[h] W1[h][h] b1[h]     (input [e_ij, v_i, v_j])
 *   dec: W0[h][h] b0[h] W1[h][1] b1[1]
 *   xdec: W0[h][h] b0[h] W1[h][1] b1[1]              (only when x_head = 1)
 * The GEMMs run on BF16 MFMA with FP32 accumulation. */
typedef struct {
    int32_t h;
    int32_t n_mp;
    const float *params;
    int32_t diag_mode;  /* 0: L_ii = sqrt(s) max(softplus(d_ii), 1e-6), L_ij = sqrt(s) (d_ij+d_ji)/2;
                           1: L' D L'^T with D = diag(A) (technical-details appendix),
                              L' unit lower triangular:
                              L_ii = sqrt(A_ii), L_ij = sqrt(A_jj) (d_ij + d_ji)/2;
                           2: the same form with a learned positive diagonal of L':
                              L_ii = sqrt(A_ii) max(softplus(d_ii + ln(e-1)), 1e-6),
                              L_ij = sqrt(A_jj) (d_ij + d_ji)/2;
                           3: L_ij as in 1, the diagonal completed so that
                              diag(L L^T) = diag(A):
                              L_ii = sqrt(max(A_ii - sum_{j<i} L_ij^2, 1e-3 A_ii)) */
    int32_t x_head;     /* 1: the network also carries the initial-guess head xdec (appendix
                           comparing with a predicted starting guess x^0), an MLP on the
                           final node latents; 0: no head */
} lpcg_gnn;

/* Number of FP32 parameters of the layout above (-1 for invalid sizes). */
int64_t lpcg_gnn_param_count(int32_t h, int32_t n_mp, int32_t x_head);

/* Workspace bytes for gnn_predict_L (train = 0) or for the training forward
 * and backward (train = 1, activations kept). */
int64_t lpcg_gnn_workspace_bytes(const lpcg_system *sys, int32_t h, int32_t n_mp,
                                 int32_t train);

/* gnn_predict_L(graph, weights) -> L.  Node input b_i / rms(b), edge input
 * A_ij / s with s = mean(diag A) (per system of a batch); d_ij = decoder
 * output per directed edge, assembled on the lower triangle as documented
 * for lpcg_gnn.diag_mode.  b: FP64 [n].  ws: device
 * workspace of lpcg_gnn_workspace_bytes(.., 0) bytes.  Writes l_val and
 * ut_val (either may be NULL).  Errors: EINVAL (h, n_mp), ENOMEM (ws too
 * small). */
int lpcg_gnn_predict_L(const lpcg_system *sys, const lpcg_gnn *net, const double *b,
                       void *ws, int64_t ws_bytes, float *l_val, float *ut_val,
                       hipStream_t stream);

/* Training forward: as lpcg_gnn_predict_L, keeping activations in ws
 * (lpcg_gnn_workspace_bytes(.., 1) bytes) for lpcg_gnn_backward. */
int lpcg_gnn_forward_train(const lpcg_system *sys, const lpcg_gnn *net, const double *b,
                           void *ws, int64_t ws_bytes, float *l_val, hipStream_t stream);

/* Initial-guess head (appendix comparing with a predicted starting guess
 * x^0): the node decoder xdec regresses, per node, the solution of the
 * normalised system (A/s) x' = b/rms(b), that is x' = x s / rms(b), and
 * x0 = x^ rms(b) / s per system of the batch.  Runs the network (as
 * lpcg_gnn_predict_L, same workspace; l_val and ut_val may be NULL) and
 * writes x0 (FP64 [n], device, original numbering) for use as the PCG
 * starting point.  Errors: EINVAL (net->x_head = 0, x0 NULL), ENOMEM. */
int lpcg_gnn_predict_x0(const lpcg_system *sys, const lpcg_gnn *net, const double *b,
                        void *ws, int64_t ws_bytes, float *l_val, float *ut_val, double *x0,
                        hipStream_t stream);

/* Loss of the initial-guess head, per system of the batch:
 *   loss[s] = sum_i (x^_i - x_i s / rms(b))^2   over the rows of system s
 * (FP64 [nsys], device, overwritten), from the head output of the last
 * forward (lpcg_gnn_forward_train, lpcg_gnn_predict_L or _x0) run on ws; x
 * (FP64 [n], original numbering) is the target solution.  When weight != 0
 * the gradient weight * d(sum_s loss[s]) / d x^ is stored in ws for the next
 * lpcg_gnn_backward (lpcg_gnn_forward_train resets it to zero, so a backward
 * without this call leaves xdec with zero gradient).  Errors: EINVAL
 * (net->x_head = 0), ENOMEM (ws too small). */
int lpcg_x0_loss(const lpcg_system *sys, const lpcg_gnn *net, void *ws, int64_t ws_bytes,
                 const double *x, double weight, double *loss, hipStream_t stream);

/* Reverse mode of the network: given dl_val = d loss / d L (FP32 [nnz_l]),
 * writes d loss / d params (FP32, same layout as params, overwritten).
 * With x_head = 1 the head's loss gradient left in ws by lpcg_x0_loss is
 * included.  ws must hold the activations of the matching
 * lpcg_gnn_forward_train. */
int lpcg_gnn_backward(const lpcg_system *sys, const lpcg_gnn *net, void *ws,
                      int64_t ws_bytes, const float *dl_val, float *dparams,
                      hipStream_t stream);

/* Data loss of the Method section per system s of the batch:
 *   loss[s] = ||L L^T x - b||^2 / rms(b)^2   over the rows of system s
 * (FP64 [nsys], overwritten) and dl_val = d(sum_s loss[s]) / d L (FP32
 * [nnz_l], overwritten, may be NULL):  2 (r_i u_j + x_i w_j) / rms(b)^2 with
 * u = L^T x, r = L u - b, w = L^T r.  x, b: FP64 [n]. */
int lpcg_llt_loss(const lpcg_system *sys, const float *l_val, const double *x,
                  const double *b, double *loss, float *dl_val, hipStream_t stream);

/* Frobenius loss of equation loss_A (the ablation of the loss-function
 * section): per system ||L L^T - A||_F^2 / s^2 over every entry of
 * L L^T - A (fill included), s = mean(diag A) of the system, into loss[nsys]
 * (device FP64), and when dl_val is given the gradient
 * 4 (L L^T - A) L / s^2 on L's entries (FP32 [nnz_l], L order).  The pattern
 * of L L^T - A is built at the first call on a system (synchronous; it
 * allocates); later calls only enqueue.  Errors: EINVAL when a row of
 * L L^T - A has more than 256 entries, ENOMEM. */
int lpcg_frob_loss(lpcg_system *sys, const float *l_val, double *loss, float *dl_val,
                   hipStream_t stream);

/* Adam step on FP32 master weights (in place): m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
 * with t = step (>= 1). */
int lpcg_adam_step(float *params, const float *grads, float *m, float *v, int64_t count,
                   float lr, float beta1, float beta2, float eps, int32_t step,
                   hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LPCG_H */
