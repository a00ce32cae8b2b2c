/*
 * tc2.h - C ABI of the MI355X (gfx950) TC2 / TC2-CPSCF response solver.
 *
 * The library purifies the zero-order density matrix X0 of a Hamiltonian H
 * given in an orthonormal atom-block basis with the second-order
 * trace-correcting recursion (Sec. 2.2, Eq. TC2), and, coupled with it, the
 * first-order response X1 to a homogeneous electric field (Sec. 2.2,
 * Eq. TC2-CPSCF):
 *
 *   X0 <- (emax*I - H)/(emax - emin),  X1_d <- -H1_d/(emax - emin)
 *   repeat:  if Tr X0 >= Nocc:  X0 <- X0 X0,        X1_d <- X1_d X0 + X0 X1_d
 *            else:              X0 <- 2X0 - X0 X0,  X1_d <- 2X1_d - X1_d X0 - X0 X1_d
 *            drop every off-diagonal atom block whose Frobenius norm is < eps
 *                                     (filter of Sec. 2.3, made block-wise)
 *   until the band energies Tr(X0 H), Tr(X1_d H) and the traces
 *   Tr(X1_d H1_d) change by less than tol (tolerance of Sec. 2.3).
 *
 * emin/emax are Gershgorin bounds of H (Sec. 2.2).  Each iteration is a
 * truncated block-sparse product (symbolic pattern, numeric block products
 * X0X0, X0X1, X1X0 on MFMA, norm drop, trace reduction choosing the next
 * branch), all in HIP kernels on one GPU.  Several independent systems can be
 * solved in one call (one merged launch per iteration step).
 *
 * Conventions
 *  - Matrices are square, block-sparse (BSR) with uniform b x b blocks,
 *    1 <= b <= 16.  row_ptr has nb+1 int64 entries, col has nnzb int32
 *    entries strictly increasing within each row, val has nnzb*b*b doubles,
 *    each block row-major.  The FULL pattern (both triangles) is given and it
 *    must be symmetric; values must be symmetric (H_JI = H_IJ^T), which the
 *    library assumes and does not check beyond the pattern.
 *  - All pointers passed to tc2_setup are HOST pointers owned by the caller;
 *    tc2_setup copies what it needs, so they may be freed when it returns.
 *  - Every entry point returns a status; no C++ exception crosses the ABI.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef TC2_H
#define TC2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TC2_API __attribute__((visibility("default")))

typedef enum {
  TC2_OK = 0,
  TC2_NOT_CONVERGED = 1,   /* max_iter reached; results are the last iterate  */
  TC2_FLOOR_REACHED = 2,   /* stopped by the stall guard (precision floor)     */
  TC2_EINVAL = -1,         /* malformed argument or option                     */
  TC2_ENOMEM = -2,         /* device or host allocation failed                 */
  TC2_EDEVICE = -3,        /* no usable gfx950 device, or a HIP call failed    */
  TC2_ENONSYM = -4,        /* pattern not symmetric or a diagonal block missing */
  TC2_EDEGENERATE = -5,    /* emax == emin while 0 < Nocc < N                 */
  TC2_ENAN = -6,           /* NaN/Inf in the input or produced by an iteration */
  TC2_EOVERFLOW = -7       /* a size exceeds the library's index range         */
} tc2_status;

typedef struct {
  int32_t nb;              /* block rows (atoms); N = nb*b                      */
  int32_t b;               /* block dimension, 1..16                             */
  const int64_t *row_ptr;  /* nb+1, row_ptr[0] = 0                               */
  const int32_t *col;      /* nnzb = row_ptr[nb]                                 */
  const double *val;       /* nnzb*b*b                                           */
} tc2_bsr;

typedef struct {
  tc2_bsr H;               /* ground-state Hamiltonian, orthonormal basis        */
  int32_t n_dir;           /* number of perturbations (field directions), 0..3   */
  tc2_bsr H1[3];           /* first-order Hamiltonians; same nb and b as H       */
  int64_t n_occ;           /* occupied states, 0..N                              */
  double eps_drop;         /* block drop threshold, >= 0                         */
  double tol;              /* band-energy convergence tolerance, > 0             */
  int32_t max_iter;        /* 1..TC2_MAX_ITER                                    */
  const char *replay;      /* NULL, or a string of 'S'/'D' forcing each step's
                              branch (exactly strlen(replay) steps are run)    */
  const double *xyz;       /* NULL, or nb x 3 atom positions: used only to group
                              nearby atoms into clusters for the tiled kernel  */
} tc2_problem;

#define TC2_MAX_ITER 200

enum { TC2_FP64 = 0, TC2_FP32 = 1, TC2_BF16 = 2 };

typedef struct {
  int32_t precision;       /* TC2_FP64 / TC2_FP32 / TC2_BF16 block products.  FP32
                              and BF16 keep X in FP32 with FP32 accumulation;
                              BF16 rounds the MFMA operands to bfloat16 (a
                              first stage, handed over to FP32), or, with
                              wide_accumulate = 1, splits each operand into
                              three bfloat16 parts for the whole reduced stage;
                              traces, branch and stopping tests stay in FP64   */
  int32_t closing_fp64;    /* 0, or 2: finish a reduced-precision solve with two
                              FP64 steps of opposite branches                  */
  int32_t skip;            /* 0: every candidate block is computed; 1: exact
                              norm-bound screen (skips blocks that are certainly
                              dropped; results unchanged); 2: the exact screen,
                              then the skip network on the remaining candidates
                              (an approximation); tiled kernel only            */
  int32_t device;          /* HIP device ordinal                                 */
  int32_t export_matrices; /* 1: tc2_run copies X0/X1 back to host views         */
  int32_t verbose;         /* 1: per-iteration log on stderr                     */
  int32_t profile;         /* 1: time each phase with HIP events on the stream   */
  int32_t numeric_kernel;  /* 0: clustered output tiles (default); 1: one wave per
                              output block (reference kernel; FP64/FP32 only)  */
  int32_t fp64_first;      /* reduced precision only: number of leading updates
                              run in FP64 before switching (0..TC2_MAX_ITER)   */
  const float *mlp_weights;/* skip = 2: TC2_MLP_PARAMS parameters of the skip
                              network (copied at setup)                        */
  float mlp_threshold;     /* skip = 2: skip a candidate whose predicted drop
                              probability exceeds this, in (0, 1)              */
  int64_t log_capacity;    /* > 0: log up to this many (features, dropped)
                              samples per tc2_run for training (tiled kernel)  */
  int32_t wide_accumulate; /* 0 or 1 (tiled kernel): in FP32 stages, the FP32
                              MFMA product of each column block is added to an
                              FP64 sum over the common columns, instead of one
                              FP32 sum over all of them.  With TC2_BF16: each
                              FP32 operand is split into three bfloat16 parts
                              (24 significant bits), the six cross products
                              above 2^-24 of the leading one run on bfloat16
                              MFMAs, and each column block's sum is added to
                              the FP64 sums (an FP32-accurate stage)           */
  int32_t tune;            /* 0: default sub-tile shapes; 1 (tiled kernel):
                              per kernel kind, take the shape from tune_cache
                              or, failing that, time every available shape on
                              the first update past the peak of the candidate
                              outputs of a tc2_run and keep the fastest for the
                              context (results do not depend on the shape)     */
  const char *tune_cache;  /* NULL, or a file: tuned shapes are read from it at
                              setup and appended to it (one JSON object per
                              line) when measured                              */
  int32_t graph;           /* 0 or 1 (tiled kernel): run each update as one
                              captured hipGraph (persistent numeric launch, no
                              size read back within the update), replayed while
                              its buffers suffice.  Not with skip = 2, logging,
                              an update that is being tuned, or the closing
                              FP64 pair (those updates run without a graph);
                              results are identical                            */
  const char *metrics_log; /* NULL, or a file: after every update one JSON line
                              per system that took part is appended: solve,
                              system, update, branch, kernel kind, phase (1 =
                              closing pair), tr_x0, e0, e1[], alpha[], tr_x1[],
                              iota = Tr X0 - ||X0||_F^2, dmax (largest change of
                              the band energies and traces), nnzb (stored
                              blocks), active (still iterating), status      */
  int32_t count_useful;    /* 0 or 1: count the useful block products of every
                              update exactly (an integer pass over the old and
                              new patterns after each update; see
                              tc2_result.useful_flops).  0: useful_flops = 0 */
  float mlp_bound_cap;     /* skip = 2: the network may skip only a candidate whose
                              exact norm bound is below mlp_bound_cap * eps for
                              X0 and every X1_d (and, on the DOUBLE branch, never
                              a stored block whose 2 ||X_IJ|| alone reaches
                              eps); 0 means 4                                   */
  double mlp_budget;       /* skip = 2: once, for some problem, the bounds of the
                              candidates the network skipped in a solve add up
                              to more than this, the rest of the solve runs with
                              the exact screen alone (skip = 1); 0: no limit   */
  int32_t device_loop;     /* 0: after every update the host reads the per-system
                              scalars and takes the branch (Eq. TC2: SQUARE
                              when Tr X0 >= Nocc) and stopping decisions (the
                              band-energy tolerance of Sec. 2.3, the stall
                              guard, max_iter).  k in 1..TC2_MAX_ITER: a kernel
                              at the end of each captured update takes them on
                              the device and writes the per-system flags that
                              the next update reads; the host replays the update
                              graph k times between two reads of a flag word.
                              Taken by tc2_run for graph = 1, precision =
                              TC2_FP64 solves with skip 0 or 1 and no replay,
                              metrics_log, log_capacity, count_useful, profile
                              or FP64 shape still to be tuned, when the dense
                              bound of the stage (every
                              upper block of every system kept) is at most
                              TC2_DEVICE_LOOP_MAX_BYTES; otherwise (and in
                              tc2_advance) the host decides.  A batch ends at
                              the update count of the context's last such
                              solve, and past it the word is polled after
                              every update; the first such solve of a context
                              polls at least every 4 updates.  Updates
                              launched after the last system stops copy the
                              iterate unchanged.  Results are identical      */
} tc2_options;

/* Largest stage (kept upper blocks x (1 + n_dir) padded 16 x 16 FP64 blocks)
 * that device_loop sizes for the dense bound. */
#define TC2_DEVICE_LOOP_MAX_BYTES ((int64_t)1 << 30)

typedef struct {
  tc2_status status;
  int32_t iters;           /* updates performed (including closing steps)        */
  double trace_x1h1[3];    /* Tr(X1_d H1_d), the raw polarizability trace        */
  double tr_x0;            /* Tr X0                                              */
  double idem_err;         /* Tr X0 - ||X0||_F^2                                 */
  double tr_x1[3];         /* Tr X1_d                                            */
  double e0;               /* Tr(X0 H)                                           */
  double e1[3];            /* Tr(X1_d H)                                         */
  double emin, emax;       /* Gershgorin bounds                                  */
  double seconds;          /* device time of the solve                           */
  double useful_flops;     /* count_useful = 1: 2 b^3 per useful block product:
                              X0_IK X0_KJ with both blocks nonzero in X0, on an
                              output (I <= J) that X0 keeps; X0_IK X1_KJ and
                              X1_IK X0_KJ with both operand blocks nonzero, on an
                              output that X1_d keeps; summed over the updates */
  double union_flops;      /* 2 b^3 (1 + 2D) per block triple with a block of
                              any matrix on both sides, on an output any matrix
                              keeps (the union pattern): an upper bound of the
                              useful flops, counted in every run               */
  double executed_flops;   /* MFMA flops issued, padding included                */
  int64_t kept_blocks;     /* stored blocks of the final X pattern (both halves) */
  int64_t screened_blocks; /* output blocks skipped by the exact screen, all
                              updates (batch total, on the first problem)     */
  int64_t mlp_skipped_blocks; /* output blocks skipped by the skip network    */
  int32_t mlp_updates;     /* updates run with the skip network (skip = 2)      */
  /* phase times in ms, summed over the updates (profile = 1 only) */
  double ms_symbolic, ms_numeric, ms_compact;
  int32_t numeric_launches;
  int32_t tile_shape[4];   /* sub-tile shape used per kernel kind (FP64, FP32,
                              BF16, FP32 with FP64 sums): 0 8x8, 1 4x8, 2 8x4,
                              3 4x4 output blocks per workgroup; -1 unused     */
  double ms_tune;          /* device time spent timing shapes in this run      */
  /* per kernel kind (index as tile_shape): useful flops of the updates run
     with it, and (profile = 1) numeric-kernel time in ms and launches */
  double useful_flops_kind[4];
  double ms_numeric_kind[4];
  int32_t numeric_launches_kind[4];
  int32_t graph_updates;   /* updates run as a captured graph                   */
  int32_t graph_captures;  /* update graphs captured (the others were replays)  */
  int32_t device_loop_updates; /* updates whose branch and stopping decisions
                              were taken on the device (device_loop)           */
  double nominal_flops;    /* 2 b^3 (1 + 2D) per block triple of the full products
                              on each update's input pattern (sum over rows K of
                              m_K^2): the work of full sparse products, as the
                              paper counts it, against useful_flops            */
  char branches[TC2_MAX_ITER + 4]; /* 'S'/'D' per update, NUL-terminated        */
  /* Library-owned host copies (valid until the next tc2_run or tc2_free) when
     export_matrices = 1; same layout as the inputs.  Otherwise zeroed. */
  tc2_bsr X0;
  tc2_bsr X1[3];
} tc2_result;

typedef struct tc2_ctx tc2_ctx;

/* Validate n_problems >= 1 problems (they must share b and n_dir), copy them
 * to the device and prepare one solver context.  *out is NULL on failure.
 * Errors: TC2_EINVAL (argument ranges, b mismatch, bad BSR ordering),
 * TC2_ENONSYM, TC2_ENAN, TC2_EDEGENERATE (checked on the device once emin and
 * emax are known, at tc2_run), TC2_EDEVICE, TC2_ENOMEM, TC2_EOVERFLOW. */
TC2_API tc2_status tc2_setup(const tc2_problem *problems, int32_t n_problems,
                     const tc2_options *opts, tc2_ctx **out);

/* Run the solve for every problem of the context on hip_stream (a
 * hipStream_t; NULL means the library's own stream).  res points to
 * n_problems results.  Returns the worst status over the problems (errors
 * before warnings).  May be called again; each call restarts from H. */
TC2_API tc2_status tc2_run(tc2_ctx *ctx, void *hip_stream, tc2_result *res);

/* Progress of tc2_advance. */
typedef struct {
  int32_t updates;         /* updates run by this call                          */
  int32_t solves_completed;/* solves that finished within this call            */
  int32_t solve_open;      /* 1: a solve is still in progress after this call   */
  double useful_flops;     /* count_useful = 1: useful flops of this call's
                              updates (as tc2_result.useful_flops)              */
  double executed_flops;   /* MFMA flops issued by this call's updates          */
} tc2_progress;

/* Run at most max_updates TC2 / TC2-CPSCF updates of the context's solve, on
 * hip_stream (NULL: the library's stream), and return.  A solve that is not in
 * progress begins first (Gershgorin bounds and the initial matrices, as
 * tc2_run).  When a solve finishes within the call (every system stopped and
 * no stage switch pending), its results are written to res (n_problems
 * entries, as tc2_run) and, if updates remain, the next solve begins from H.
 * The updates and results are those of tc2_run: a solve advanced in pieces
 * gives the same iterates.  tc2_run abandons a solve in progress.
 * Returns the worst status of the solves finished in this call (TC2_OK if
 * none finished), or an error; prog is filled in either case.
 * Errors: TC2_EINVAL (NULL ctx, prog or res; max_updates < 0), and those of
 * tc2_run. */
TC2_API tc2_status tc2_advance(tc2_ctx *ctx, void *hip_stream, int32_t max_updates,
                               tc2_progress *prog, tc2_result *res);

/* ---------------------------------------------------------------------------
 * Access to the current iterate of a context (after tc2_run, or between two
 * tc2_advance calls): for checks of sampled rows of systems too large to
 * export whole, and for comparing two solves of the same problems on the
 * device.  Matrix index m: 0 = X0, 1 + d = X1_d.
 * ------------------------------------------------------------------------- */

/* Complete block rows `rows` (n_rows indices into the block rows of problem
 * `system`, in any order) of X0 and of every X1_d (x1 holds n_dir matrices),
 * as library-allocated host BSR matrices of the problem's size whose other
 * rows are empty; columns are the problem's own.  Each output is freed with
 * tc2_bsr_release.  Errors: TC2_EINVAL (no iterate yet, ranges, NULL),
 * TC2_ENOMEM, TC2_EDEVICE. */
TC2_API tc2_status tc2_export_rows(tc2_ctx *ctx, int32_t system, const int32_t *rows,
                                   int32_t n_rows, tc2_bsr *x0, tc2_bsr *x1);

/* Stored entries (blocks) of the current iterate of all problems of the
 * context, merged into one block-diagonal matrix in problem order. */
TC2_API tc2_status tc2_iterate_size(tc2_ctx *ctx, int64_t *nnz);

/* Entries [first, first + count) of that merged pattern, in row-major order:
 * block row and column (merged indices) and the b x b values of matrix m,
 * row-major.  Any of rows, cols, vals may be NULL (not written); the caller
 * owns them (count, count and count*b*b elements).
 * Errors: TC2_EINVAL (ranges, no iterate), TC2_ENOMEM, TC2_EDEVICE. */
TC2_API tc2_status tc2_export_entries(tc2_ctx *ctx, int32_t matrix, int64_t first, int64_t count,
                                      int32_t *rows, int32_t *cols, double *vals);

/* Largest |A - B| over the union of two block patterns: A is given by the
 * caller as n entries (merged block row and column, strictly increasing in
 * row-major order, with b x b row-major values), B is matrix m of the current
 * iterate; a block missing on one side counts as zero.  The caller's values
 * are uploaded in chunks, so A may be larger than the free device memory
 * (its rows and columns are uploaded whole).  detail (NULL, or 6 doubles)
 * receives: the largest difference over blocks both sides hold; the largest
 * |A| over nonzero blocks only A holds; the largest |B| over nonzero blocks
 * only B holds; the counts of those two kinds of blocks; and the largest
 * Frobenius norm of a block held by one side only.  Under a drop threshold,
 * blocks held by one side only are those whose norm lies near the threshold
 * and that one side kept and the other dropped.
 * Errors: TC2_EINVAL (ranges, order, NULL), TC2_ENOMEM, TC2_EDEVICE. */
TC2_API tc2_status tc2_compare_entries(tc2_ctx *ctx, int32_t matrix, int64_t n, const int32_t *rows,
                                       const int32_t *cols, const double *vals, double *max_abs,
                                       double *detail);

/* Copy the samples logged by the last tc2_run (log_capacity > 0): features
 * (n x TC2_MLP_IN floats: scaled log10 of the norm bounds of X0 and X1 relative
 * to eps, of the largest single product, of the number of common columns,
 * distance / 10, scaled log10 of the previous block norm or -3, update / 20,
 * branch), labels (1 = the block was dropped, 0 = kept, -1 = skipped by the
 * network, outcome unknown) and, if z is not NULL, the logit the in-kernel
 * network gave the sample (skip = 2; 0 otherwise).  Returns the number of
 * samples copied (at most cap), or a negative tc2_status. */
TC2_API int64_t tc2_log_copy(tc2_ctx *ctx, float *x, float *y, float *z, int64_t cap);

/* Release the context and everything it owns.  NULL-safe. */
TC2_API void tc2_free(tc2_ctx *ctx);

/* Device memory pool (Sec. 2.3's products grow their buffers every update).
   Large buffers of every context map physical memory in fixed chunks; the
   chunks a buffer or a freed context gives back stay in a per-device pool of
   the process and are mapped again by later buffers and contexts, so that
   the GPU driver does not clear reclaimed memory before each reuse.  The pool
   is returned to the GPU driver when an allocation of the library fails for lack
   of memory (then retried), and by this call: device = HIP ordinal.  Returns
   TC2_EINVAL for an ordinal without a device.  Call it when other code of the
   process needs the memory; no context of the library needs to be freed.  */
TC2_API tc2_status tc2_trim_memory(int32_t device);

/* Static description of a status code. */
TC2_API const char *tc2_strerror(tc2_status s);

/* Library version string. */
TC2_API const char *tc2_version(void);

/* ---------------------------------------------------------------------------
 * Block-skip network (learned screen).  A multilayer perceptron
 * TC2_MLP_IN -> 64 -> 64 -> 1 with ReLU hidden layers maps features of a
 * candidate output block of an update to the logit of the probability that
 * the block ends below the drop threshold.  theta holds TC2_MLP_PARAMS floats:
 * W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major, W2[j][k] maps input
 * k to output j), b2 (64), w3 (64), b3 (1).  The loss is the mean binary
 * cross-entropy on logits, softplus(z) - y z.  All pointers are host pointers
 * owned by the caller; x is n x TC2_MLP_IN row-major, y holds 0/1 labels.
 * Errors: TC2_EINVAL (ranges, NULL), TC2_ENAN (non-finite input),
 * TC2_EDEVICE, TC2_ENOMEM.
 * ------------------------------------------------------------------------- */
#define TC2_MLP_IN 8
#define TC2_MLP_HIDDEN 64
#define TC2_MLP_PARAMS 4801

typedef struct {
  int32_t epochs;          /* passes over the data, >= 1                        */
  int32_t batch;           /* samples per Adam step, >= 1 (in data order)       */
  float lr;                /* Adam step size, > 0                               */
  float beta1, beta2;      /* Adam moment decays, in [0, 1)                     */
  float adam_eps;          /* Adam denominator guard, > 0                       */
  int32_t device;          /* HIP device ordinal                                */
} tc2_mlp_train_opts;

/* Logits of n samples (n >= 0). */
TC2_API tc2_status tc2_mlp_forward(const float *theta, const float *x, int64_t n,
                                   int32_t device, float *logits);

/* Gradient (TC2_MLP_PARAMS floats) and value of the mean loss over n >= 1
 * samples. */
TC2_API tc2_status tc2_mlp_grad(const float *theta, const float *x, const float *y,
                                int64_t n, int32_t device, float *grad, double *loss);

/* tc2_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same gradient and mean loss, with every pointer a DEVICE pointer owned
 * by the caller (theta: TC2_MLP_PARAMS floats, x: n x TC2_MLP_IN, y: n,
 * grad: TC2_MLP_PARAMS floats, loss: one double), on the current device and
 * hip_stream (NULL: the null stream).  Asynchronous: grad and loss hold the
 * result once the stream reaches this work.  The per-block partial sums live
 * in a fixed library array on each device (about 4.9 MB, held until the
 * process ends), so 1 <= n <= TC2_MLP_NOALLOC_MAX_N; calls that overlap on one
 * device share that array and race.  Inputs are not checked for NaN (they are
 * not on the host); a non-finite input gives non-finite outputs.
 * Errors: TC2_EINVAL (NULL pointer, n out of range), TC2_EDEVICE. */
#define TC2_MLP_NOALLOC_MAX_N 65536
TC2_API tc2_status tc2_mlp_grad_noalloc(const float *theta, const float *x, const float *y,
                                        int64_t n, void *hip_stream, float *grad, double *loss);

/* Train with Adam on the device; theta holds the initial parameters on entry
 * (drawn by the caller) and the trained ones on return.  loss_per_epoch, if
 * not NULL, receives `epochs` mean losses. */
TC2_API tc2_status tc2_mlp_train(const float *x, const float *y, int64_t n,
                                 const tc2_mlp_train_opts *opts, float *theta,
                                 double *loss_per_epoch);

/* ---------------------------------------------------------------------------
 * Dense O(N^3) density matrix and response (Sec. 2.1, the O(N^3) method): the
 * reference against which the linear-scaling path is timed in the crossover
 * experiment of Sec. 4.
 *
 * The method, in the orthonormal basis (S = I):
 *  - H, densified, is diagonalised as H C = C E.
 *  - P0 = C_occ C_occ^T over the n_occ lowest states.
 *  - For each direction d, the coefficient response is C1 = C U.  Its
 *    elements are U_pq = -(C^T H1_d C)_pq / (e_p - e_q) for p != q
 *    (Eq. cpscf-LCAO) and U_pp = 0.
 *  - P1_d = sum over occupied i of (C1_i C_i^T + C_i C1_i^T) (Eq. DM1).
 *
 * The occupied-occupied terms of P1_d cancel. It is therefore formed as
 *     G = C_virt^T (H1_d C_occ),   M_ai = G_ai / (e_i - e_a),
 *     Y = C_virt M,                P1_d = Y C_occ^T + C_occ Y^T.
 *
 * Traces are taken over the stored blocks of H and H1_d.
 *
 * Device work:
 *  - rocSOLVER dsyevd for the eigenpairs;
 *  - rocBLAS for the products (dsyrk, dgemm, dsyr2k);
 *  - HIP kernels for densifying, the gap scaling, mirroring and the traces.
 *
 * The problem must pass the checks of tc2_setup. Its eps_drop, tol, max_iter,
 * replay and xyz fields are not used.
 *
 * Edge cases: n_occ = 0 gives P0 = 0, and n_occ = N gives P0 = I; both give
 * P1_d = 0 and gap = 0, without computing eigenpairs (eigenvalues is not
 * written).
 *
 * Host buffers in the options are owned by the caller. The device memory is
 * about 3 N^2 doubles plus the solver's workspace; it is allocated and freed
 * within the call.
 *
 * Errors:
 *  - TC2_EINVAL: NULL arguments, ranges, N > TC2_DENSE_MAX_N;
 *  - TC2_ENONSYM, TC2_ENAN: the checks of tc2_setup;
 *  - TC2_EDEGENERATE: the highest occupied and lowest virtual eigenvalues
 *    coincide, so P0 is not defined;
 *  - TC2_EDEVICE: the eigensolver did not converge, or a HIP/ROCm call failed;
 *  - TC2_ENOMEM.
 * ------------------------------------------------------------------------- */
#define TC2_DENSE_MAX_N 40000

typedef struct {
  int32_t device;          /* HIP device ordinal                                */
  void *hip_stream;        /* hipStream_t to run on; NULL: a stream of the call */
  double *p0;              /* NULL, or N*N host doubles receiving P0 (symmetric) */
  double *p1[3];           /* NULL, or N*N host doubles per direction: P1_d      */
  double *eigenvalues;     /* NULL, or N host doubles: e, ascending              */
} tc2_dense_options;

typedef struct {
  tc2_status status;
  double e0;               /* Tr(P0 H)                                           */
  double e1[3];            /* Tr(P1_d H)                                         */
  double trace_p1h1[3];    /* Tr(P1_d H1_d), the polarizability trace            */
  double tr_p0;            /* Tr P0 (= n_occ up to rounding)                    */
  double gap;              /* e_lowest virtual - e_highest occupied              */
  double seconds;          /* device time from the densified H to the traces     */
  double ms_eigh;          /* phase times (ms): eigenpairs, P0, all P1_d         */
  double ms_p0, ms_p1;
  double flops_p1;         /* nominal flops of the P1 products, all directions  */
} tc2_dense_result;

TC2_API tc2_status tc2_dense_response(const tc2_problem *problem,
                                      const tc2_dense_options *opts,
                                      tc2_dense_result *res);

/* ---------------------------------------------------------------------------
 * Loewdin orthogonalisation for a non-orthogonal basis (Sec. 2.2).
 *
 * The TC2 cycles take the orthogonal forms H_orth = S^-1/2 H S^-1/2 and
 * H1_orth = S^-1/2 H1_d S^-1/2. Their converged results go back to the
 * non-orthogonal basis as P = S^-1/2 P_orth S^-1/2. S^-1/2 comes from a
 * Newton-Schulz iteration of block-sparse products; the paper computes the
 * square root of S with such an iteration, in linear scaling.
 *
 * tc2_lowdin runs the coupled form of the iteration. With lam the Gershgorin
 * upper bound of S, start from Y = S/lam and Z = I, then repeat:
 *     M = Z Y;  stop if ||M - I||_F / sqrt(N) < tol;
 *     T = (3 I - M)/2;  Y <- Y T;  Z <- Z T
 * At the end S^-1/2 = Z / sqrt(lam).  A stall guard stops the iteration with
 * TC2_FLOOR_REACHED when an update did not halve that residual: the filter
 * or rounding, not the iteration, then sets it.
 *
 * Every product is atom-block sparse with the block filter of Sec. 2.3: an
 * off-diagonal block whose Frobenius norm is strictly below eps is dropped.
 * Products whose exact value is symmetric (Z Y, Y T, Z T, and the outer
 * product of a congruence) are formed on their upper blocks and mirrored, so
 * that they are exactly symmetric. This includes the upper scalar triangle
 * of each diagonal block. A congruence Z X Z is the product (Z X) Z.
 *
 * Inputs: host BSR matrices with the layout and checks of tc2_setup. S must
 * store every diagonal block. S, H, H1_d and X must be symmetric.
 *
 * Outputs: BSR matrices in host memory allocated by the library with the
 * same layout (full symmetric pattern, row-major blocks). The caller frees
 * each one with tc2_bsr_release. On an error nothing is left allocated.
 *
 * Errors:
 *  - TC2_EINVAL: NULL arguments, ranges, more than 2^18 block rows;
 *  - TC2_ENONSYM, TC2_ENAN: the checks of tc2_setup, or a non-finite
 *    residual;
 *  - TC2_EDEGENERATE: the Gershgorin bound of S is not positive;
 *  - TC2_EOVERFLOW, TC2_ENOMEM, TC2_EDEVICE.
 * TC2_NOT_CONVERGED (max_iter updates did not reach tol) and
 * TC2_FLOOR_REACHED (the stall guard) come with valid outputs.
 * ------------------------------------------------------------------------- */
typedef struct {
  double eps;              /* block drop threshold of every product, >= 0       */
  double tol;              /* tc2_lowdin: stop when ||Z Y - I||_F/sqrt(N) < tol  */
  int32_t max_iter;        /* tc2_lowdin: 1..TC2_MAX_ITER updates                */
  int32_t device;          /* HIP device ordinal                                */
  void *hip_stream;        /* hipStream_t to run on; NULL: a stream of the call */
} tc2_lowdin_options;

typedef struct {
  tc2_status status;
  int32_t iters;           /* Newton-Schulz updates performed                   */
  double resid;            /* ||Z Y - I||_F / sqrt(N) at the last test          */
  double lambda;           /* the Gershgorin bound S was divided by             */
  double seconds;          /* device time of the iteration and the transforms   */
  tc2_bsr Z;               /* S^-1/2                                            */
  tc2_bsr H;               /* S^-1/2 H S^-1/2                                   */
  tc2_bsr H1[3];           /* S^-1/2 H1_d S^-1/2, d < n_dir                     */
} tc2_lowdin_result;

/* S^-1/2 and the orthogonal forms of H and of n_dir (0..3) perturbations. */
TC2_API tc2_status tc2_lowdin(const tc2_bsr *S, const tc2_bsr *H, int32_t n_dir,
                              const tc2_bsr *H1, const tc2_lowdin_options *opts,
                              tc2_lowdin_result *res);

/* out = Z X Z (the back-transform when Z = S^-1/2); opts->eps, device and
 * hip_stream are used.  seconds, if not NULL, receives the device time. */
TC2_API tc2_status tc2_congruence(const tc2_bsr *Z, const tc2_bsr *X,
                                  const tc2_lowdin_options *opts, tc2_bsr *out,
                                  double *seconds);

/* ---------------------------------------------------------------------------
 * Perturbations that move the basis: an atomic displacement changes the
 * overlap as well (S1_d != 0). The paper names this as the next use of the
 * formalism, after the field perturbation.
 *
 * Differentiating P = Z X Z with Z = S^-1/2 gives
 *     H1_orth = Z1 H Z + Z H1_d Z + Z H Z1,
 *     P1      = Z1 X0 Z + Z X1 Z + Z X0 Z1.
 * Here Z1 is the derivative of S^-1/2 along S1_d. X0 and X1 are the TC2 /
 * TC2-CPSCF results on H_orth and H1_orth.
 *
 * tc2_lowdin_response runs the iteration of tc2_lowdin together with its
 * derivative along each S1_d:
 *     M1 = Z1 Y + Z Y1;  T1 = -M1/2;
 *     Y1 <- Y1 T + Y T1;  Z1 <- Z1 T + Z T1;
 * starting from Y1 = S1_d/lam and Z1 = 0. The updates and stopping tests are
 * those of tc2_lowdin, on the unperturbed residual. At the end
 * Z1 = Z1/sqrt(lam).
 *
 * Each derivative is a sum of two products, filtered after the sum. A sum
 * whose exact value is symmetric is mirrored from its upper blocks, as in
 * tc2_lowdin.
 *
 * tc2_congruence_response forms P1 as (Z1 X0 + Z X1) Z + (Z X0) Z1.
 *
 * S1_d and H1_d must be symmetric BSR matrices with the layout of H; they
 * need not store diagonal blocks. Errors and output ownership are those of
 * tc2_lowdin and tc2_congruence. S1 may be NULL only when n_dir = 0.
 * ------------------------------------------------------------------------- */
typedef struct {
  tc2_status status;
  int32_t iters;           /* Newton-Schulz updates performed                   */
  double resid;            /* ||Z Y - I||_F / sqrt(N) at the last test          */
  double lambda;           /* the Gershgorin bound S was divided by             */
  double seconds;          /* device time of the iteration and the transforms   */
  tc2_bsr Z;               /* S^-1/2                                            */
  tc2_bsr H;               /* S^-1/2 H S^-1/2                                   */
  tc2_bsr Z1[3];           /* derivative of S^-1/2 along S1_d                   */
  tc2_bsr H1[3];           /* Z1 H Z + Z H1_d Z + Z H Z1                        */
} tc2_lowdin_response_result;

TC2_API tc2_status tc2_lowdin_response(const tc2_bsr *S, const tc2_bsr *H, int32_t n_dir,
                                       const tc2_bsr *H1, const tc2_bsr *S1,
                                       const tc2_lowdin_options *opts,
                                       tc2_lowdin_response_result *res);

/* out = Z1 X Z + Z X1 Z + Z X Z1 (the back-transform of a response when the
 * overlap moves). */
TC2_API tc2_status tc2_congruence_response(const tc2_bsr *Z, const tc2_bsr *Z1,
                                           const tc2_bsr *X, const tc2_bsr *X1,
                                           const tc2_lowdin_options *opts, tc2_bsr *out,
                                           double *seconds);

/* Free a matrix returned by tc2_lowdin, tc2_lowdin_response, tc2_congruence
 * or tc2_congruence_response and zero it.  NULL-safe. */
TC2_API void tc2_bsr_release(tc2_bsr *m);

#ifdef __cplusplus
}
#endif
#endif /* TC2_H */
