/*
 * amg.h -- C ABI of the MI355X (gfx950) solve path for K u = F, K sparse SPD:
 * conjugate gradients preconditioned by a matching-based aggregation AMG
 * V-cycle (D'Ambra, Durastante, Filippone, arXiv 2511.21268).
 *
 * Two-phase use, as in the paper's preconditioner-build-then-Krylov split
 * (Sec. 4, the hierarchy build followed by the Krylov call with initial guess in,
 * solution out, iteration count and error estimate out):
 *   amg_setup()  builds the hierarchy on the host (compatible weighted matching,
 *                Sec. 3.1) and uploads it to the device, factoring the coarsest
 *                matrix there;
 *   pcg_solve()  runs the whole solve phase in HIP kernels on the device.
 *
 * Conventions common to every call:
 *  - all functions return amg_status; AMG_OK == 0; negative values are errors,
 *    positive values are warnings (the output is valid);
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *    memory of the device that was current when amg_setup ran;
 *  - the caller owns every array it passes; the library copies what it keeps and
 *    holds no caller pointer after a call returns;
 *  - a context is not thread-safe: calls on one context must not overlap;
 *  - on error, amg_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).
 */
#ifndef AMG_H
#define AMG_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_NOT_CONVERGED = 1,  /* itmax reached; u holds the last iterate          */
    AMG_ERR_ARG = -1,       /* invalid argument or matrix                       */
    AMG_ERR_NOT_SPD = -2,   /* non-positive pivot in the coarsest factorization */
    AMG_ERR_HIP = -3,       /* HIP runtime error                                */
    AMG_ERR_OOM = -4,       /* device or host allocation failed                 */
    AMG_ERR_BREAKDOWN = -5, /* (p, K p) <= 0 or non-finite, or (r, B r) <= 0    */
    AMG_ERR_STATE = -6      /* coarsening stalled above 2000 unknowns           */
} amg_status;

typedef struct amg_ctx amg_ctx;   /* opaque: the hierarchy on host and device */

typedef struct {
    int sweeps_per_level;   /* m pairwise matching sweeps composed per level
                               (aggregates of at most 2^m; Sec. 3.1 m-step);
                               default 2, range 1..3                            */
    int max_coarse;         /* stop coarsening at <= this many rows; that level
                               is solved by the coarse solver (coarse_solver);
                               default 200, range 1..2000                       */
    int max_levels;         /* default 40                                       */
    int nu_pre, nu_post;    /* smoother sweeps before / after the coarse
                               correction (Sec. 3 steps 1 and 5); default 1, 1;
                               nu_pre must be >= 1                              */
    int vcycle_fp32;        /* 0: V-cycle in FP64; 1: V-cycle in FP32 (outer
                               residual, dots, coarse Cholesky stay FP64)       */
    int smoother;           /* 0: l1-Jacobi (Sec. 3.2); 1: degree-4 polynomial
                               in D^{-1}K (coefficients by amg_set_poly_coeffs);
                               2: Chebyshev acceleration of l1-Jacobi (Sec. 3.2,
                               Sec. 5.1), fourth kind, degree cheb_degree      */
    int krylov;             /* 0: CG; 1: flexible CG, FCG(1) (Sec. 3.1 end);
                               2: in pcg_solve_batched, block flexible CG (one
                               block Krylov space shared by the columns, 16 x 16
                               Gram matrices; a converged column leaves the
                               block), FCG(1) in pcg_solve                      */
    int match_positive_only;/* 0: every edge eligible (default);
                               1: only edges with c_ij > 1 (log c_ij > 0)       */
    int itmax;              /* default 1000                                     */
    int nrhs;               /* 1 (default): single-vector layout only; 2..16:
                               also build the layout of the block kernels used by
                               pcg_solve_batched and autotune it (lanes per row
                               and block size, timed on the level-0 matrix)     */
    int slice_offsets;      /* 1 (default): a 64-row slice whose rows share one
                               list of column offsets (column - row) no longer
                               than its longest row stores that list once
                               instead of per-entry indices (stencil matrices);
                               0: per-entry indices in every slice              */
    /* The paper's default preconditioner (Sec. 3.1 "Variants and efficiency",
     * Sec. 5.1) is sweeps_per_level = 3, smooth_prolong = 1, smoother = 2 with
     * cheb_degree 8 / 12 / 14 / 16 for p = 3 / 4 / 5 / 6, coarse_solver = 1 and
     * krylov = 1.  Any of smoother 2, smooth_prolong 1 or coarse_solver 1 takes
     * the FP64 single-vector V-cycle: vcycle_fp32 = 0, nrhs = 1, and with
     * smoother 2 nu_pre = nu_post = 1.                                         */
    int smooth_prolong;     /* 0 (default): tentative prolongator P;
                               1: P' = (I - omega D^{-1} K) P, D the l1 diagonal,
                               coarse matrix (P'^T K) P'                        */
    int cheb_degree;        /* smoother 2: matrix products per smoothing step,
                               1..64; default 8                                 */
    int coarse_solver;      /* 0 (default): dense Cholesky of the coarsest level;
                               1: CG preconditioned by one Jacobi sweep, to
                               coarse_tol or coarse_itmax iterations (Sec. 5.1;
                               a variable preconditioner: use krylov = 1)       */
    int coarse_itmax;       /* coarse_solver 1: 1..1000; default 30            */
    double omega;           /* smooth_prolong: damping, (0, 2]; default 4/3     */
    double coarse_tol;      /* coarse_solver 1: relative residual, >= 0;
                               default 1e-4                                     */
    int setup_device;       /* 0 (default): matching and Galerkin products on
                               the host; 1: on the device (rounds of locally
                               dominant edges, sort-based Galerkin), the same
                               hierarchy bit for bit; needs a structurally
                               symmetric K with fewer than 2^31 entries and
                               smooth_prolong = 0 (not with amg_setup_host)     */
    int bootstrap_sweeps;   /* 0 (default): the test vector is w (ones if NULL);
                               s > 0: w is the random start of s l1-Jacobi
                               sweeps on K w = 0 (Sec. 3.1) and must be given;
                               at most 1000                                     */
} amg_params;

/* Fill p with the defaults above.  p must not be NULL. */
amg_status amg_params_default(amg_params *p);

/*
 * Build the hierarchy for the n x n matrix K given in CSR on the host.
 *  row_ptr[n+1] int64, col[nnz] int32 (sorted ascending within each row),
 *  val[nnz] FP64; K must be symmetric in pattern and values, with a positive
 *  diagonal entry stored in every row, and all values finite.
 *  w: host test vector of length n (Sec. 3.1 eq. (cij)); NULL means all ones;
 *  with prm->bootstrap_sweeps > 0 it is the random start of the relaxation that
 *  produces the test vector (required then).
 *  prm: NULL means defaults.  hip_stream: the hipStream_t every later call of
 *  this context is ordered on (NULL = the null stream).
 * Per level: edge weights c_ij = 1 - 2 k_ij w_i w_j / (k_ii w_i^2 + k_jj w_j^2)
 * (eq. (cij)), greedy matching in the order (c desc, min index, max index),
 * pairwise prolongator of eq. (prolongation), Galerkin K_c = P^T K P
 * (eq. (galerkin_matrix_projection)), composed m times; with smooth_prolong the
 * composed prolongator is smoothed and K_c = (P'^T K) P'.  On the host, or on
 * the device with setup_device (the same hierarchy bit for bit).
 * Errors: AMG_ERR_ARG (n <= 0 or n >= 2^29, malformed or non-symmetric K,
 * non-finite values, missing or non-positive diagonal), AMG_ERR_NOT_SPD, AMG_ERR_STATE,
 * AMG_ERR_OOM, AMG_ERR_HIP.  On error *out is NULL.
 */
amg_status amg_setup(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *w, const amg_params *prm, void *hip_stream, amg_ctx **out);

/*
 * Solve K u = F (Sec. 4: CG or FCG preconditioned by one V-cycle per iteration).
 *  F: device, length n, FP64.  u: device, length n, FP64; in: initial guess,
 *  out: solution (last iterate on AMG_NOT_CONVERGED).  F and u must not alias.
 *  Stops when ||r_k||_2 <= tol ||F||_2 on the recursive residual.
 *  iters (host, may be NULL): completed updates of u.
 *  relres (host, may be NULL): ||r_k||_2 / ||F||_2 of the recursion at exit.
 *  relres_true (host, may be NULL): ||F - K u||_2 / ||F||_2, computed at exit.
 * F == 0 gives u = 0, iters = 0, AMG_OK.  The call is ordered on the context's
 * stream and returns after the solve has finished on the device.
 * Errors: AMG_ERR_ARG (NULL pointers, tol < 0, non-finite F), AMG_ERR_BREAKDOWN,
 * AMG_ERR_HIP; warning AMG_NOT_CONVERGED.
 */
amg_status pcg_solve(amg_ctx *c, const double *F, double *u, double tol,
                     int *iters, double *relres, double *relres_true);

/*
 * Residual history of the last pcg_solve on this context (the Krylov call's
 * trace output of Sec. 4): ||r_k||_2 / ||F||_2 of the recursion for
 * k = 0 .. iterations (iterations + 1 values; empty before the first solve and
 * for F = 0).  hist: host, the first min(cap, count) values are written (may
 * be NULL when cap is 0); count (host, may be NULL): the number available.
 */
amg_status amg_get_residual_history(const amg_ctx *c, double *hist, int cap, int *count);

/*
 * Solve nrhs independent systems K U[:,k] = F[:,k] sharing every matrix pass:
 * one block SpMV and one block V-cycle per iteration, each column with its own
 * FCG(1) scalars, converged columns frozen.
 *  F, U: device, n x nrhs column-major FP64 (U in: guesses, out: solutions).
 *  iters, relres: host arrays of length nrhs (may be NULL).
 *  1 <= nrhs <= 16.  The V-cycle precision follows prm.vcycle_fp32.
 * Errors as pcg_solve; AMG_NOT_CONVERGED if any column did not converge.
 */
amg_status pcg_solve_batched(amg_ctx *c, int nrhs, const double *F, double *U, double tol,
                             int *iters, double *relres);

/*
 * Apply the preconditioner once: z = B r, one V-cycle from the finest level
 * with a zero initial guess (Sec. 3, the five steps of the two-level
 * correction applied recursively).  r, z: device, length n, FP64, no aliasing.
 * The V-cycle precision follows prm.vcycle_fp32.
 */
amg_status amg_vcycle(amg_ctx *c, const double *r, double *z);

/*
 * y = K_l x with the device copy of level l's matrix (FP64; level 0 is the
 * caller's K).  x, y: device, length n_l, FP64, no aliasing.
 * level in 0 .. levels-2, or 0 for a single-level hierarchy.
 */
amg_status amg_spmv(amg_ctx *c, int level, const double *x, double *y);

/*
 * Variant of the block kernels used by pcg_solve_batched on the images without
 * staged windows (coarse levels, the K P images of the fused post-smoothing,
 * and every image when AMG_OPT_BLOCK_WINDOW is 0): lpr lanes per matrix row
 * (1: the single-vector SELL-64 image, one lane per row and 16 columns per
 * lane; 4, 8 or 16: SELL-(64/lpr) block images, 16/lpr columns per lane) and
 * threads per block (256 or 512).  amg_setup with prm.nrhs > 1 sets the
 * fastest by timing; amg_set_batched_variant overrides it (lpr 4/8/16 only when
 * those images were built, i.e. the autotuner's choice).
 */
amg_status amg_get_batched_variant(const amg_ctx *c, int *lpr, int *threads);
amg_status amg_set_batched_variant(amg_ctx *c, int lpr, int threads);

/*
 * Set the degree-4 polynomial smoother of one level (used when prm.smoother
 * == 1): correction sum_{k=0..3} coeffs[k] (D^{-1}K)^k D^{-1} r (Sec. 3.2,
 * polynomial acceleration of l1-Jacobi).  Accepted iff the error polynomial
 * e(t) = 1 - sum coeffs[k] t^{k+1} has |e| <= 1 on [0,1] and e < 1 on (0,1]
 * (checked on 10^4 steps): then the V-cycle stays SPD.  Rejected coefficients
 * leave the level on l1-Jacobi and return AMG_NOT_CONVERGED (a warning).
 * level in 0 .. levels-2.
 */
amg_status amg_set_poly_coeffs(amg_ctx *c, int level, const double coeffs[4]);

/* Levels and sizes.  level = -1: *n receives the number of levels and *nnz the
 * total stored entries (operator complexity = total / nnz of level 0). */
amg_status amg_get_level_info(const amg_ctx *c, int level, int64_t *n, int64_t *nnz);

/* Host copies of level `level`'s aggregate map (agg[i] = coarse index of row i)
 * and prolongator coefficients (pc[i]); level in 0 .. levels-2.  Either output
 * may be NULL. */
amg_status amg_get_aggregates(const amg_ctx *c, int level, int32_t *agg, double *pc);

/* Host CSR copy of the Galerkin matrix of `level` (sizes from
 * amg_get_level_info).  Any output may be NULL. */
amg_status amg_get_coarse_matrix(const amg_ctx *c, int level, int64_t *row_ptr, int32_t *col,
                                 double *val);

/* Rounds of the device matching (setup_device = 1): matching sweeps run, rounds
 * of locally dominant edges summed over them, and the most in one sweep; zeros
 * for a host set-up.  Any output may be NULL. */
amg_status amg_get_setup_rounds(const amg_ctx *c, int *sweeps, int *rounds_total, int *rounds_max);

/* Host CSR copy of the smoothed prolongator (I - omega D^{-1} K) P of level
 * `level` (0 .. levels-2; rows n_level, columns n_{level+1}; Sec. 3.1
 * "Variants and efficiency").  *nnz receives its stored entries (0 when the
 * context was built without smooth_prolong); row_ptr (n_level + 1), col and val
 * may each be NULL, e.g. to query the size first. */
amg_status amg_get_prolongator(const amg_ctx *c, int level, int64_t *nnz, int64_t *row_ptr, int32_t *col,
                               double *val);

/* Host-only build of the same hierarchy (no device memory, no HIP call): for
 * inspecting aggregates, coarse matrices and operator complexity on a machine
 * without a GPU.  The level accessors work on the result; the solve calls
 * return AMG_ERR_STATE.  Arguments and errors as amg_setup, except that the
 * coarsest level is not factored (AMG_ERR_NOT_SPD cannot occur). */
amg_status amg_setup_host(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *w, const amg_params *prm, amg_ctx **out);

/* One pairwise matching sweep on its own (Sec. 3.1): mate[i] = the row matched
 * with row i, or -1.  Same edge weights, eligibility and order as amg_setup;
 * host arrays; K as in amg_setup (symmetric CSR), w NULL means ones. */
amg_status amg_match(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                     const double *w, int positive_only, int32_t *mate);

/* Host check of the device matrix layout (no GPU needed): builds the SELL-C
 * image (C in {4, 8, 16, 32, 64}) of the n x ncols CSR matrix K the way the
 * library does -- layout 0: row order and per-entry indices; 1: shared column
 * offsets where they fit (square matrices only); 2: rows sorted by length
 * within windows of 4 slices; 3: as 1, with the shared-offset slices walked
 * the way the block kernels stage x windows (runs of consecutive offsets, the
 * rows each run reads copied once; C = 64 only); 4: as 3, with the windows
 * shared by blocks of four slices through the stage tables of the batched
 * set-up (AMG_OPT_WINDOW_SHARE; C = 64 only) -- and computes y = K x (host arrays, x of length
 * ncols, y of length n) by walking that image as the matrix-pass kernels do:
 * groups of 8 entries, columns rebuilt from shared offsets (clamped where the
 * slice needs it), 16-bit deltas or int32 columns, the slot -> row map.  Every
 * column the walk would read is checked against [0, ncols): AMG_ERR_STATE if
 * one is not.  shared_slices, stored (may be NULL): slices with shared offsets,
 * stored entries with padding.  For tests and inspection. */
amg_status amg_sell_spmv_host(int64_t n, int64_t ncols, const int64_t *row_ptr, const int32_t *col,
                              const double *val, int C, int layout, const double *x, double *y,
                              int64_t *shared_slices, int64_t *stored);

/* Free everything the context holds (host and device).  NULL is a no-op. */
void amg_destroy(amg_ctx *c);

/* Message of the last error on this thread ("" if none). */
const char *amg_last_error(void);

/* Solve-phase options (value 0 = off, 1 = on):
 * AMG_OPT_GRAPH (default off): replay the iteration body of pcg_solve /
 *   pcg_solve_batched from HIP graphs, captured on the library's own stream at
 *   the first solve of each kind (the caller's stream is joined by events) and
 *   replayed every iteration; re-captured after amg_set_poly_coeffs,
 *   amg_set_learned_poly or amg_set_batched_variant; not used while profiling.
 *   Results are bitwise those of the eager launches.
 * AMG_OPT_FUSE_POST (default on): with l1-Jacobi, fuse the prolongation into
 *   the first post-smoothing sweep, using f - K (u + P e) = r - (K P) e with the
 *   residual r of the pre-smoothed iterate and a stored K P (about 40% of K's
 *   entries): one full matrix pass per level becomes a K P pass.  Equal to the
 *   unfused V-cycle up to rounding.
 * AMG_OPT_BLOCK_WINDOW (default 4; autotuned between 2 and 4 by amg_setup
 *   with prm.nrhs > 1): the block kernels of pcg_solve_batched on a matrix
 *   image whose slices share column offsets (stencil matrices) copy, for each
 *   run of consecutive offsets of a slice, the rows of X the run reads into an
 *   LDS window once instead of gathering a 16-column row of X per entry, with
 *   `value` rows (and 16 / value columns) per lane; 0 turns this off (those
 *   images then take the lanes-per-row variant of amg_set_batched_variant).
 *   Bitwise the same results in every setting.
 * AMG_OPT_TAIL (default off): the coarsest levels of the V-cycle -- from the
 *   first level down whose every level has at most 2048 rows and 60,000
 *   entries -- run in one persistent single-workgroup kernel per V-cycle
 *   (residual, restriction, Cholesky solve, fused post-smoothing, level after
 *   level) instead of one launch per step; single-vector and batched solves,
 *   l1-Jacobi with one pre- and one post-sweep and the fused post-smoothing
 *   only (else the per-level kernels run).  Bitwise the same results.  Off by
 *   default: on the 2.1M-unknown cube the single workgroup takes longer than
 *   the per-level launches it replaces (0.3% of a single-vector solve, 2% of
 *   a 16-column one), whose launch gaps the stream already hides.
 *   amg_get_option returns the first tail level, or 0 when the tail is off or
 *   not available.
 * AMG_OPT_WINDOW_SHARE (a mask, default 3; autotuned by amg_setup with
 *   prm.nrhs > 1): with AMG_OPT_BLOCK_WINDOW on, the four slices of a
 *   256-thread block share their windows in the passes over FP64 values (bit
 *   0) and over FP32 values (bit 1): amg_setup groups the slices of every
 *   stencil image in fours one grid line apart (slice stride 1..4, the one
 *   that copies the fewest rows) and lists, per block, the windows of X rows
 *   the block copies once for all four waves and which run of which wave each
 *   serves, in each wave's run order.  amg_get_option returns the mask, 0 for
 *   an image without such lists.  Bitwise the same results.
 * AMG_OPT_X_WINDOW (autotuned by amg_setup): the single-vector matrix passes over FP64
 *   values (SpMV, residual, smoother sweep) walk the slices of stencil images
 *   that have run tables through x windows: per run of consecutive offsets, the
 *   1 KB of x the slice's 64 rows read is copied once into LDS and every lane
 *   reads its entries there, instead of one gather per entry; runs whose 1 KB
 *   would leave x take the gathers.  amg_setup times both walks on the level-0
 *   residual and keeps the faster (the gathers gain more from a faster memory;
 *   the two differ by a few percent either way).  Bitwise the same results.
 * amg_get_option returns the current value of an option. */
typedef enum {
    AMG_OPT_GRAPH = 1,
    AMG_OPT_FUSE_POST = 2,
    AMG_OPT_BLOCK_WINDOW = 3,
    AMG_OPT_TAIL = 4,
    AMG_OPT_WINDOW_SHARE = 5,
    AMG_OPT_X_WINDOW = 6
} amg_option;
amg_status amg_set_option(amg_ctx *c, int option, int value);
amg_status amg_get_option(const amg_ctx *c, int option, int *value);

/* ------------------------------------------------------------------------
 * Measurement.  While enabled, every launch of the level-0 sparse
 * matrix-pass kernel (SpMV, residual, smoother sweep) inside the solve calls
 * is bracketed by HIP events on the context's stream; amg_get_profile returns
 * the number of launches, their summed device time and their summed
 * algorithmic HBM bytes (each launch: matrix values and index bytes without
 * padding, plus the vectors it must read and write once).
 */
amg_status amg_set_profiling(amg_ctx *c, int enable);
amg_status amg_get_profile(amg_ctx *c, int64_t *launches, double *ms, double *bytes);
/* The same figures for one kind of level-0 pass (any output may be NULL):
 * SpMV with its dots (the Krylov product), residual, smoother sweep,
 * polynomial-smoother step, the fused K P prolongation + post-smoothing pass,
 * other passes (Chebyshev steps, prolongation with a smoothed prolongator).
 * amg_set_profiling(c, 1) clears them with the totals. */
typedef enum { AMG_PASS_SPMV = 0, AMG_PASS_RESID = 1, AMG_PASS_SMOOTH = 2, AMG_PASS_POLY = 3, AMG_PASS_KP = 4,
               AMG_PASS_OTHER = 5, AMG_PASS_KINDS = 6 } amg_pass_kind;
amg_status amg_get_profile_pass(const amg_ctx *c, int kind, int64_t *launches, double *ms, double *bytes);
/* Streaming-read reference for the rooflines (no step of the solve): reads
 * `bytes` of device memory at buf (16-byte aligned, bytes a multiple of 16)
 * once, with the 16-byte nontemporal loads of the matrix passes (each wave
 * 4 KB contiguous chunks, four loads in flight), on `stream` (a hipStream_t,
 * NULL = default), in min(sink_len / 256, 65536) blocks of 256 threads (2048:
 * eight per compute unit, the fastest grid measured); thread t writes the sum
 * of the doubles it read to sink[t] (device array of sink_len >= 256 doubles,
 * caller-owned).  Asynchronous: time it with events on the same stream.
 * AMG_ERR_ARG for a bad pointer, size or sink. */
amg_status amg_stream_read(const void *buf, int64_t bytes, double *sink, int64_t sink_len, void *stream);
/* Description of a level's single-vector layout: slice height, stored
 * entries with padding, index bytes per entry in slices with per-entry
 * indices (2 or 4), and the number of slices (of ceil(n / slice)) that store
 * shared column offsets instead.  A coarse level of the Chebyshev form held as
 * CSR with L lanes per row (long or few rows) reports slice = -L and 4 index
 * bytes.  Any output may be NULL. */
amg_status amg_get_format(const amg_ctx *c, int level, int *slice, int64_t *stored,
                          int *index_bytes, int64_t *shared_slices);

/* ------------------------------------------------------------------------
 * Workload generator (Sec. 2): the Dirichlet-reduced stiffness matrix of the
 * Poisson problem on the unit square (d = 2) or cube (d = 3), tensor-product
 * B-splines of degree p with n equal elements per direction, open uniform knots
 * (maximum regularity), homogeneous Dirichlet on every face, lexicographic
 * order with x fastest, constant coefficient: the Kronecker sum of the 1D
 * stiffness and mass matrices, each by (p+1)-point Gauss quadrature.
 * amg_iga_poisson_size gives N = (n+p-2)^d and nnz; amg_iga_poisson fills
 * caller-allocated host CSR arrays and F for f = 1 (F may be NULL).
 */
amg_status amg_iga_poisson_size(int d, int p, int n, int64_t *N, int64_t *nnz);
amg_status amg_iga_poisson(int d, int p, int n, int64_t *row_ptr, int32_t *col, double *val,
                           double *F);

/*
 * The paper's cube benchmark (Sec. 5.1, "Cube"): -Lap u = f on [0,1]^3 with
 * u = exp(x+z) sin(y), f = -exp(x+z) sin(y), Dirichlet data g_D = u on sides
 * 1-3 (x = 0, x = 1, y = 0) and Neumann data g_N = du/dn on sides 4-6 (y = 1,
 * z = 0, z = 1), tensor B-splines of degree p with n elements per direction.
 * The Dirichlet functions (first and last in x, first in y) are removed; F is
 * the interior load vector: source and Neumann integrals (Sec. 2.2, f_i) minus
 * K times the lifting, whose coefficients are those of the L2 projection of
 * g_D onto the spline space.  N = (n+p-2)(n+p-1)(n+p) (Table 1(b)); ordering
 * lexicographic, x fastest.  Host arrays sized by amg_iga_cube_size; F may be
 * NULL.  1 <= p <= 10.
 */
amg_status amg_iga_cube_size(int p, int n, int64_t *N, int64_t *nnz);
amg_status amg_iga_cube(int p, int n, int64_t *row_ptr, int32_t *col, double *val, double *F);

/* ------------------------------------------------------------------------
 * Learned polynomial smoother: a small MLP (8 -> 64 -> 64 -> 4, tanh) maps the
 * features of a level to the coefficients of its degree-4 polynomial smoother
 * (Sec. 3.2 polynomial acceleration; coefficients as in amg_set_poly_coeffs).
 * Parameters: a vector of AMG_MLP_NPARAM entries
 *   W1[64][8] b1[64] W2[64][64] b2[64] W3[4][64] b3[4],
 * held as BF16 bit patterns (uint16) for the kernels and as an FP32 master copy
 * for training; accumulation is FP32.  All MLP arrays below are device arrays
 * of the caller, ordered on hip_stream; B samples, row-major.
 */
#define AMG_MLP_NPARAM 4996
#define AMG_MLP_NFEAT 8
#define AMG_MLP_NACT 128     /* stored activations per sample (h1, h2)        */
#define AMG_MLP_NDEL 132     /* stored deltas per sample (dy, dh2, dh1)        */

/* Features of level `level` (host output, AMG_MLP_NFEAT floats), all
 * independent of the problem size: log10(nnz/n)/3, (longest row)/(nnz/n) - 1,
 * mean and min over rows of k_ii/d_i (d = l1 diagonal), mean of
 * sum_{j!=i} k_ij / d_i, fraction of positive off-diagonal entries,
 * log10((nnz/n) / (nnz_0/n_0))/2 (row density against the finest level),
 * n_{level+1}/n_level (0 on the coarsest). */
amg_status amg_level_features(const amg_ctx *c, int level, float *feat);

/* Y[B][4] = MLP(X[B][8]) with BF16 weights w; act (may be NULL) receives the
 * hidden activations, AMG_MLP_NACT floats per sample, for the backward pass. */
amg_status amg_mlp_forward(const uint16_t *w, const float *X, int B, float *Y, float *act, void *hip_stream);

/* Gradient of L = mean_{s,i} (Y - T)^2 with respect to the parameters (grad,
 * AMG_MLP_NPARAM floats) and the loss (1 float), from a forward pass's Y and
 * act; del is a workspace of B * AMG_MLP_NDEL floats. */
amg_status amg_mlp_backward(const uint16_t *w, const float *X, const float *act, const float *Y, const float *T,
                            int B, float *del, float *grad, float *loss, void *hip_stream);

/* amg_mlp_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight training or serving loops, harnesses that forbid
 * hipMalloc): the per-sample deltas live in a static device array of the
 * library, AMG_MLP_NOALLOC_MAX_B * AMG_MLP_NDEL floats (8.7 MB) per device,
 * held until the process ends, so no workspace argument and no allocation of
 * any kind.  Arguments, results and bits as amg_mlp_backward; B above
 * AMG_MLP_NOALLOC_MAX_B returns AMG_ERR_ARG.  The array is shared by every
 * call on a device: calls that overlap on one GPU (other streams, other
 * threads) race on it and must be serialized by the caller; a call leaves its
 * deltas there, and the next call overwrites what it reads before reading it. */
#define AMG_MLP_NOALLOC_MAX_B 16384
amg_status amg_mlp_backward_noalloc(const uint16_t *w, const float *X, const float *act, const float *Y,
                                    const float *T, int B, float *grad, float *loss, void *hip_stream);

/* One Adam step (b1 = 0.9, b2 = 0.999, eps = 1e-8) on the FP32 master weights
 * with bias correction for step >= 1, then w = BF16(master) (round to nearest
 * even).  step = 0 only rounds master into w. */
amg_status amg_mlp_adam(float *master, uint16_t *w, const float *grad, float *m, float *v, int step, float lr,
                        void *hip_stream);

/* Predict every level's smoother with the MLP (weights: host BF16 array) on the
 * device and set each level through the acceptance test of amg_set_poly_coeffs;
 * a rejected level keeps l1-Jacobi.  The network's four outputs are the values
 * of g(t) = 1 - e(t) = sum_k a_k t^{k+1} at the Chebyshev-Lobatto nodes
 * t_j = (1 - cos(j pi / 4)) / 2, j = 1..4 (g(0) = 0): the degree-4 interpolant
 * gives the coefficients a_0..a_3, and an output error of size eps moves e(t) by
 * at most about 2 eps on [0, 1].  accepted (host, may be NULL): levels-1 flags;
 * coeffs (host, may be NULL): (levels-1) x 4 predicted coefficients.  Needs
 * prm.smoother == 1. */
amg_status amg_set_learned_poly(amg_ctx *c, const uint16_t *w_host, int *accepted, double *coeffs);

/*
 * Variable-coefficient workload: -div(kappa grad u) = 1 on the unit cube with
 * kappa(x) = exp(0.5 sum_{k<nk} a[k] cos(2 pi m_k . x)), m_k = mk[3k..3k+2],
 * the same space, boundary conditions, pattern and order as amg_iga_poisson
 * (d = 3), assembled by (p+1)^3-point Gauss quadrature with sum factorization
 * (Sec. 2.2).  Sizes from amg_iga_poisson_size(3, p, n, ...); F (may be NULL)
 * receives the load vector of f = 1.  1 <= p <= 7.
 */
amg_status amg_iga_diffusion(int p, int n, int nk, const double *a, const int32_t *mk, int64_t *row_ptr,
                             int32_t *col, double *val, double *F);

#ifdef __cplusplus
}
#endif
#endif
