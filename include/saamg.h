/*
 * saamg.h -- C ABI of the MI355X smoothed-aggregation AMG + CG solver for 3D
 * elasticity systems kept in 3x3 block CSR (BSR3) form.
 *
 * Method: D. E. Demidov, "Efficient solution of 3D elasticity problems with
 * smoothed aggregation algebraic multigrid and block arithmetics" (2022).
 *   - The system A u = f (Section 2, eq. (1)) has a natural 3x3 block per pair
 *     of mesh nodes; every level of the hierarchy is stored with 3x3 blocks
 *     (Section 2, discussion of Fig. 1: coarse levels have 6x6 blocks, i.e.
 *     2x2 groups of 3x3 blocks).
 *   - Setup follows Algorithm 1 with the "NS Block" structure of Section 3:
 *     the tentative prolongation is built from the six rigid body modes in
 *     scalar space, everything else (prolongation smoothing, Galerkin
 *     product, smoother) in block arithmetic.  It runs on the host in FP64.
 *   - The solve (Algorithm 2 V-cycle as the preconditioner of CG, Section 4:
 *     relative residual 1e-8) runs on the GPU in hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   - Return value: amg_status.  AMG_OK (0) on success, AMG_NOT_CONVERGED (1)
 *     is a warning (outputs are valid), negative values are errors.  On error
 *     amg_last_error() returns a message for the calling thread.
 *   - The library never aborts and never prints.
 *   - Host pointers are read during the call only and never retained.
 *   - Device pointers are HIP device allocations (e.g. PyTorch CUDA tensors on
 *     ROCm); the library does not free them.
 *   - A context is bound to one HIP stream and one device; it is not
 *     thread-safe.  Calls on different contexts may run concurrently.
 *   - Unknowns are node-major: u_x, u_y, u_z of node 0, then node 1, ...
 *   - Environment (read at upload): SAAMG_TUNE_CACHE names a file of recorded
 *     operator layouts (read if present, appended with new choices);
 *     SAAMG_TUNE_LOG a file that receives every timed layout candidate;
 *     SAAMG_SORT_WINDOW the window (in slices, 1..4096, default 256) inside
 *     which sorted sliced-ELL layouts order their rows by length.
 */
#ifndef SAAMG_H
#define SAAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_NOT_CONVERGED = 1,       /* maxiter or max_restarts reached; x holds the last iterate */
    AMG_ERR_ARG = -1,            /* invalid argument (null, size, pattern, non-finite) */
    AMG_ERR_SINGULAR_BLOCK = -2, /* a 3x3 diagonal block is not invertible */
    AMG_ERR_NOT_SPD = -3,        /* coarsest Cholesky failed / non-positive diagonal */
    AMG_ERR_OOM = -4,            /* host or device allocation failed */
    AMG_ERR_HIP = -5,            /* a HIP runtime call failed */
    AMG_ERR_BREAKDOWN = -6,      /* CG breakdown: p^T A p <= 0 (matrix or preconditioner not SPD) */
    AMG_ERR_UNSUPPORTED = -7     /* input the requested option does not support */
} amg_status;

typedef enum { AMG_FP64 = 0, AMG_FP32 = 1, AMG_BF16 = 2 } amg_precision;
/* Outer iteration.  CG / FCG: conjugate gradients (flexible: Polak-Ribiere
 * beta) in FP64, preconditioned by the V-cycle of the chosen precision.  IR
 * (FP32/BF16 forms only): FP64 iterative refinement around an inner FP32 CG. */
typedef enum { AMG_KRYLOV_CG = 0, AMG_KRYLOV_FCG = 1, AMG_KRYLOV_IR = 2 } amg_krylov;
/* Smoother (Section 3 names Jacobi and SPAI-0 as the smoothers whose cost is
 * the SpMV).  JACOBI: damped block Jacobi with the inverted 3x3 diagonal
 * blocks on every level.  SPAI0: damped block SPAI-0 on every level,
 * M_I = omega A_II (sum_J A_IJ A_IJ^T)^{-1} (the block-diagonal minimiser of
 * ||I - M A||_F, damped like Jacobi); the post-sweep applies M_I^T so the
 * V-cycle stays symmetric.  LEARNED: learned blocks on level 1, Jacobi below;
 * the setup also keeps the per-node inputs of the learned smoother blocks
 * (amg_smoother_set_weights); until weights are set level 1 is block Jacobi. */
typedef enum {
    AMG_SMOOTHER_JACOBI = 0,
    AMG_SMOOTHER_LEARNED = 1,
    AMG_SMOOTHER_SPAI0 = 2,
    /* Block ILU(0), the smoother of the paper's experiments (Section 3: ILU(0)
     * with block-valued entries; Section 4 and Tables 1-2 use it in every run):
     * incomplete factors L (unit block lower) and U (block upper) on A's own
     * 3x3 block pattern, computed in a greedy multicolour order of the block
     * rows (in increasing row order, the smallest colour no coupled row has
     * taken), so each triangular solve is one dependent pass per colour;
     * undamped, x <- x + (L U)^{-1} (f - A x) before and after the coarse
     * correction.  Applies to the first smoother_levels levels (0: every
     * level); levels below use block Jacobi.  FP64 and FP32 V-cycles only;
     * not for amg_solve_multi or batches. */
    AMG_SMOOTHER_ILU0 = 3
} amg_smoother;

/* Setup and solve parameters.  Fill with amg_default_params() first. */
typedef struct {
    double eps_strong;    /* strength threshold on level 1 (0.08) */
    double eps_decay;     /* threshold factor per level (0.5) */
    double omega_p;       /* prolongation smoothing damping (2/3) */
    double omega_j;       /* block-Jacobi damping; <= 0: 4/(3 lambda_max(D^-1 A)) per level */
    int32_t npre;         /* pre-smoothing sweeps (1) */
    int32_t npost;        /* post-smoothing sweeps (1) */
    int32_t coarse_enough;/* a level with at most this many unknowns is solved directly (3000) */
    int32_t max_levels;   /* hierarchy depth limit (10) */
    int32_t use_nullspace;/* 1: rigid body modes from coords; 0: constant modes per component */
    int32_t precision;    /* amg_precision of the V-cycle (AMG_FP64) */
    int32_t krylov;       /* amg_krylov outer iteration (AMG_KRYLOV_CG) */
    int32_t maxiter;      /* CG iteration limit (1000) */
    int32_t check_every;  /* CG iterations between host convergence checks (8) */
    int32_t max_restarts; /* true-residual restarts after a false convergence (2) */
    int32_t use_graphs;   /* 1: replay iteration chunks as HIP graphs (1) */
    int32_t nthreads;     /* host setup threads; 0: hardware concurrency */
    int32_t autotune;     /* 1: time the candidate device layouts of every operator at upload
                             and keep the fastest (1); 0: fixed rule by row length */
    int32_t smoother;     /* amg_smoother (AMG_SMOOTHER_JACOBI) */
    int32_t accept_recurrence; /* 1: stop when the CG recurrence residual meets tol and report
                             the recomputed FP64 true residual without restarting (for systems
                             whose true residual cannot reach tol in FP64); 0: the FP64 true
                             residual must meet tol (0) */
    int32_t smoother_levels; /* AMG_SMOOTHER_ILU0: levels that use it, from the finest (0: every
                             level; default 1); the others use block Jacobi */
    int32_t setup_path;   /* amg_setup_path: how the host builds the transfer operators and the
                             Galerkin products (AMG_SETUP_BLOCK) */
    int32_t setup_device; /* amg_setup only: 1 = form the values of the Galerkin products A P and
                             R (A P) on the GPU (block path; patterns on the host) (0) */
} amg_params;

/* Host setup construction (Section 3).  BLOCK ("NS Block"): the matrix stays
 * in 3x3 blocks, only the tentative prolongation is formed in scalar space
 * (per aggregate); prolongation smoothing, R = P^T and R A P are block
 * products.  SCALAR (the hybrid construction of the "NS Hybrid" solvers):
 * strength, prolongation smoothing, transpose and the Galerkin products in
 * scalar CSR, every matrix converted to 3x3 blocks afterwards.  Both give
 * the same hierarchy up to rounding; the smoothers are built from the block
 * matrices either way. */
typedef enum { AMG_SETUP_BLOCK = 0, AMG_SETUP_SCALAR = 1 } amg_setup_path;

/* A square matrix in 3x3 block CSR, all arrays on the host.  Block columns are
 * sorted within each block row, every block row holds its diagonal block, and
 * val holds nnzb row-major 3x3 blocks (9 doubles each). */
typedef struct {
    int32_t nb;              /* block rows (= mesh nodes) */
    int64_t nnzb;            /* stored blocks */
    const int32_t *row_ptr;  /* [nb+1] */
    const int32_t *col;      /* [nnzb] */
    const double *val;       /* [nnzb*9] */
} amg_bsr3;

typedef struct {
    int32_t iters;            /* CG iterations (products A p) */
    int32_t restarts;         /* true-residual restarts */
    int32_t converged;        /* 1 if ||b - A x|| <= tol ||b|| (FP64); 2 if only the CG recurrence
                                 residual met tol (accept_recurrence = 1, the FP64 true residual
                                 above tol); 0 otherwise */
    int32_t fell_back;        /* 1 if a learned smoother was replaced by block Jacobi */
    double rel_true_residual; /* ||b - A x|| / ||b||, recomputed in FP64 */
    double solve_ms;          /* device time of the solve (HIP events) */
} amg_solve_info;

#define AMG_MAX_LEVELS 16

typedef struct {
    int32_t levels;
    int32_t nb[AMG_MAX_LEVELS];        /* block rows per level */
    int64_t nnzb_A[AMG_MAX_LEVELS];
    int64_t nnzb_P[AMG_MAX_LEVELS];    /* P_l: nb[l] x nb[l+1] blocks (0 on the coarsest) */
    int32_t n_agg[AMG_MAX_LEVELS];
    double omega_j[AMG_MAX_LEVELS];
    int32_t n_coarse;                  /* unknowns of the coarsest (dense) level */
    double operator_complexity;        /* sum nnzb(A_l) / nnzb(A_1) */
    double setup_ms;                   /* host setup wall time */
    double device_bytes;               /* hierarchy bytes resident on the GPU */
    double vcycle_bytes;               /* algorithmic HBM bytes of one V-cycle */
    double iter_bytes;                 /* algorithmic HBM bytes of one CG iteration */
    int32_t layout_A[AMG_MAX_LEVELS];  /* device layout: rows per slice of sliced ELL (4..64), or
                                          1 = one wavefront per row, 2 = one workgroup per row
                                          (both with contiguous blocks); negative = rows sorted
                                          by length within slice windows */
    int32_t layout_P[AMG_MAX_LEVELS];
    int32_t layout_R[AMG_MAX_LEVELS];
    int32_t layout_AM[AMG_MAX_LEVELS]; /* layouts of the fused-sweep operators (0: none) */
    int32_t layout_G[AMG_MAX_LEVELS];
    /* host setup wall time by phase, summed over the levels (ms): 0 strength graph and
     * aggregation, 1 tentative prolongation (QR), 2 prolongation smoothing, 3 transpose,
     * 4 Galerkin products, 5 smoother blocks and damping, 6 fused-sweep operators,
     * 7 ILU(0) factors, 8 coarsest inverse, 9 other (checks, near-nullspace, learned
     * inputs), 10 scalar/block conversions (AMG_SETUP_SCALAR) */
    double setup_phase_ms[11];
} amg_stats_t;

typedef struct amg_hierarchy amg_hierarchy;
typedef struct amg_ctx amg_ctx;

/* Defaults listed in the field comments above. */
void amg_default_params(amg_params *prm);

/* Thread-local message for the last error of the calling thread ("" if none). */
const char *amg_last_error(void);

/* ---- host setup (Algorithm 1), no GPU involved ------------------------- */

/* Build the FP64 hierarchy on the host from A (BSR3, host) and the node
 * coordinates coords[nb*3] (host; used for the six rigid body modes,
 * Section 2).  *out is owned by the caller and released with
 * amg_hierarchy_free.
 * Errors: AMG_ERR_ARG (null pointers, nb <= 0, unsorted / out-of-range
 * columns, missing diagonal block, non-finite values),
 * AMG_ERR_SINGULAR_BLOCK, AMG_ERR_NOT_SPD, AMG_ERR_OOM. */
amg_status amg_hierarchy_build(const amg_bsr3 *A, const double *coords,
                               const amg_params *prm, amg_hierarchy **out);
/* amg_hierarchy_build with the numeric phase of every level's Galerkin
 * products (A P and A_{l+1} = R (A P), Algorithm 1) on the GPU: the
 * patterns are formed on the host, the values by device kernels on
 * hip_stream (NULL: the null stream), and copied back for the rest of the
 * host setup.  Block construction only (setup_path is ignored).  Device
 * memory is allocated and freed within the call.  Errors as
 * amg_hierarchy_build, plus AMG_ERR_HIP. */
amg_status amg_hierarchy_build_device(const amg_bsr3 *A, const double *coords, const amg_params *prm,
                                      void *hip_stream, amg_hierarchy **out);
void amg_hierarchy_free(amg_hierarchy *h);
amg_status amg_hierarchy_stats(const amg_hierarchy *h, amg_stats_t *st);

/* Host copies of one level for inspection.  which: 0 = A_l, 1 = P_l,
 * 2 = R_l (all BSR3: the caller passes row_ptr[rows+1], col[nnzb],
 * val[nnzb*9] sized from amg_hierarchy_level_shape); 3 = smoother blocks
 * M_l (val[nb*9], row_ptr and col unused); 4 = aggregate id per node
 * (written as doubles into val[nodes]; -1 for isolated nodes); 5 = the dense
 * inverse of the coarsest matrix (val[n_coarse^2], row-major; level ignored);
 * 6 = the learned smoother's per-node features (val[nb*90], stored in FP32,
 * written as doubles; empty unless smoother = AMG_SMOOTHER_LEARNED); 7 = the
 * Cholesky factors of the level-1 smoother blocks that go with them
 * (val[nb*6]: L00 L10 L11 L20 L21 L22); 8 = the post-sweep smoother blocks
 * (val[nb*9]; the transposes of kind 3 for SPAI-0, equal to kind 3 otherwise);
 * 9 = AM_l and 10 = G_l, the BSR3 operators of the fused sweeps (AM = A M with
 * blocks A_IJ M_J, levels below the first; G = (I - Mt A) P with Mt the
 * post-sweep blocks, every level but the coarsest, on level 1 of the learned
 * smoother formed with the block-Jacobi blocks until weights are set; both
 * empty unless npre = npost = 1); on levels with the ILU(0) smoother:
 * 11 = the colour of each block row (written as doubles into val[nb]),
 * 12 = the strictly lower factor L without its unit diagonal and 13 = the
 * upper factor U with its diagonal blocks (both BSR3 in the level's own row
 * numbering; L U = A on A's pattern in the colour order). */
amg_status amg_hierarchy_level_shape(const amg_hierarchy *h, int32_t level, int32_t which,
                                     int32_t *rows, int32_t *cols, int64_t *nnzb);
amg_status amg_hierarchy_export(const amg_hierarchy *h, int32_t level, int32_t which,
                                int32_t *row_ptr, int32_t *col, double *val);

/* ---- device context (upload + solve) ----------------------------------- */

/* amg_setup = amg_hierarchy_build (amg_hierarchy_build_device if
 * prm->setup_device) + amg_upload.  hip_stream is a hipStream_t
 * (e.g. torch.cuda.current_stream().cuda_stream) or NULL for the null stream;
 * the context uses it for every later call.  The context owns all device
 * memory it allocates (freed by amg_destroy). */
amg_status amg_setup(const amg_bsr3 *A, const double *coords, const amg_params *prm,
                     void *hip_stream, amg_ctx **out);
/* Upload an existing host hierarchy (not consumed; may be freed afterwards). */
amg_status amg_upload(const amg_hierarchy *h, const amg_params *prm, void *hip_stream,
                      amg_ctx **out);
void amg_destroy(amg_ctx *ctx);
amg_status amg_stats(const amg_ctx *ctx, amg_stats_t *st);

/* Solve A x = b by CG preconditioned with one V-cycle per iteration
 * (Algorithm 2; Section 4).  b and x are device arrays of 3*nb doubles; x is
 * the initial guess on entry and the solution on exit.  tol bounds the FP64
 * relative true residual ||b - A x|| / ||b||.  Allocates nothing.  If info is
 * NULL the call is asynchronous on the context stream and returns AMG_OK once
 * the iteration loop has finished (the loop itself synchronises to test
 * convergence); if info is non-NULL it is filled.
 * ||b|| = 0 gives x = 0.  Errors: AMG_ERR_ARG (null, non-finite b),
 * AMG_ERR_BREAKDOWN, AMG_ERR_HIP; AMG_NOT_CONVERGED after maxiter, or when the
 * FP64 true residual is still above tol after max_restarts restarts (a
 * recurrence residual below tol whose true residual stalls at the rounding
 * floor of an ill-conditioned operator). */
amg_status amg_solve(amg_ctx *ctx, const double *b, double *x, double tol,
                     amg_solve_info *info);

/* Solve A X = B for k <= 32 right-hand sides at once.  B and X are device
 * arrays of 3*nb*k doubles stored row-major (column index fastest:
 * B[i*k + j] is unknown i of right-hand side j); X holds the initial guesses.
 * Every operator is read once per product for all k columns (block SpMM);
 * each column runs its own FP64 CG (its own alpha, beta and convergence test,
 * frozen once converged) preconditioned by the V-cycle of the context's
 * precision.  info_k, if not NULL, is a host array of k entries.  The first
 * call allocates the context's multi-column buffers (sized for 32 columns);
 * later calls allocate nothing.  Needs a hierarchy of at least two levels
 * (AMG_ERR_UNSUPPORTED otherwise).  A column counts as converged when its
 * FP64 true residual meets tol (or, with accept_recurrence, its CG recurrence
 * residual); there are no restarts.  Errors as amg_solve. */
amg_status amg_solve_multi(amg_ctx *ctx, int32_t k, const double *B, double *X, double tol,
                           amg_solve_info *info_k);

/* One V-cycle for k <= 32 columns at once (Algorithm 2 with every operator
 * read once per product for all columns, block SpMM; on a single-level
 * hierarchy the coarsest dense solve alone, an FP64 MFMA GEMM).  R and Z are
 * device arrays of 3*nb*k doubles, row-major like amg_solve_multi's B and X,
 * Z != R; the V-cycle runs in the context's precision (FP64 in and out).
 * The first multi-column call allocates the context's multi-column buffers.
 * Errors: AMG_ERR_ARG, AMG_ERR_UNSUPPORTED (ILU(0) smoother), AMG_ERR_HIP. */
amg_status amg_vcycle_multi(amg_ctx *ctx, int32_t k, const double *R, double *Z);

/* ---- batch of independent problems ----------------------------------- */

typedef struct amg_batch amg_batch;

/* Set up np independent problems (A[p] host BSR3, coords[p] host [nb_p*3]) for
 * one batched solve.  Every problem gets its own hierarchy (same parameters);
 * on the device the operators of each level are concatenated so that every
 * V-cycle step is one launch for the whole batch, and the coarsest solves of
 * the problems that stop at a level run as one batched dense product.
 * precision AMG_FP64 keeps an FP64 V-cycle; any other value gives the FP32
 * V-cycle.  The outer iteration is FP64 CG with one set of CG scalars per
 * problem.  Errors as amg_setup. */
amg_status amg_setup_batch(int32_t np, const amg_bsr3 *A, const double *const *coords,
                           const amg_params *prm, void *hip_stream, amg_batch **out);
/* b[p], x[p]: device arrays of 3*nb_p doubles (x holds the initial guesses).
 * info (host array of np entries) may be NULL.  Allocates nothing. */
amg_status amg_solve_batch(amg_batch *batch, const double *const *b, double *const *x, double tol,
                           amg_solve_info *info);
/* One batched V-cycle (Algorithm 2 for every problem, the level operators of
 * all problems concatenated so each step is one launch, the coarsest solves
 * one batched dense product): z[p] = V_p(r[p]) with r[p], z[p] device arrays
 * of 3*nb_p doubles (z[p] != r[p]), in the batch's precision (FP64 in and
 * out).  Allocates nothing.  Errors: AMG_ERR_ARG, AMG_ERR_HIP. */
amg_status amg_vcycle_batch(amg_batch *batch, const double *const *r, double *const *z);
void amg_batch_destroy(amg_batch *batch);

/* Apply one V-cycle z = V(r) (Algorithm 2, zero initial guess on every
 * level).  r and z are device arrays of 3*nb doubles, z != r. */
amg_status amg_vcycle(amg_ctx *ctx, const double *r, double *z);

/* Debug/test access to single kernels on level l (device arrays, FP64):
 * op 0: out = A_l in           (in, out: 3*nb_l)
 * op 1: out = R_l in           (in: 3*nb_l, out: 3*nb_{l+1})
 * op 2: out = P_l in           (in: 3*nb_{l+1}, out: 3*nb_l)
 * op 3: out = M_l in           (zero-guess smoothing step)
 * op 4: out = in2 + M_l (in - A_l in2)  (one smoothing sweep from in2)
 * op 5: out = A_L^{-1} in      (coarsest dense solve; l ignored)
 * op 6: out = in - A_l in2     (residual)
 * op 11: out = in - AM_l in    (fused pre-sweep residual t = f - A M f)
 * op 12: out = G_l in + M_l (in2 + out)  (fused post-sweep: in = e on level
 *        l+1, in2 = f, out holds t on entry and z on return)
 * Ops 11 and 12 exist on levels with fused sweeps (export kinds 9 and 10);
 * elsewhere they fail with AMG_ERR_ARG.
 * in2 may be NULL for ops that do not use it. */
amg_status amg_debug_apply(amg_ctx *ctx, int32_t level, int32_t op, const double *in,
                           const double *in2, double *out);

/* Time one kernel of the solve on the context's internal buffers: `reps`
 * back-to-back launches between two HIP events on the context stream.
 * op as in amg_debug_apply (0: A_l x, 1: R_l x, 2: x += P_l x_c, 3: x = M_l f,
 * 4: smoothing sweep, 5: coarsest solve, 6: residual) plus 7: smoothing sweep
 * fused with a dot product and 8: product fused with a dot product (the two
 * level-1 kernels of a CG iteration), 9: one whole V-cycle, 10: one CG
 * iteration, 11 and 12: the fused pre- and post-sweep kernels, 14: the
 * post-sweep operator G as a plain product (its stream without the
 * epilogue), 15: A with the post-sweep's epilogue z = A x + M (f + y),
 * 16: the coarsest solve with the last restriction folded in (W = A_L^{-1}
 * R applied to the residual of the level above; level ignored; AMG_ERR_ARG
 * if the V-cycle does not fold it).  *avg_ms receives the mean duration of one launch and *bytes the
 * algorithmic HBM bytes it must move (each stored block, index and vector
 * entry counted once; padding and cache re-reads excluded).
 * Errors: AMG_ERR_ARG (level/op out of range, reps < 1), AMG_ERR_HIP. */
amg_status amg_time_op(amg_ctx *ctx, int32_t level, int32_t op, int32_t reps, double *avg_ms,
                       double *bytes);

/* FP64 true residual norm ||b - A x|| / ||b|| with A the finest matrix. */
amg_status amg_true_residual(amg_ctx *ctx, const double *b, const double *x, double *rel);

/* Bytes of the static device array behind amg_true_residual_noalloc (one
 * copy per GPU the library runs on, held until the process ends). */
#define AMG_NOALLOC_SCRATCH_BYTES (1 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the computation
 * of amg_true_residual with its scratch -- the per-workgroup partial sums of
 * the two norms and the reduction state -- in a static device array of
 * AMG_NOALLOC_SCRATCH_BYTES instead of context memory.  Calls no allocating
 * routine.
 *   b, x:  device inputs, 3*nb doubles each.
 *   r:     device output, 3*nb doubles: r = b - A x (A the finest matrix);
 *          must not alias b or x.
 *   norms: device output, 2 doubles: ||b||^2 and ||b - A x||^2.
 *   rel:   host output or NULL.  Non-NULL: the call waits for the context
 *          stream and writes ||b - A x|| / ||b|| (||b - A x|| if b = 0), the
 *          value amg_true_residual returns.  NULL: the call only enqueues its
 *          kernels on the context stream (no host synchronisation).
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (any contexts, any streams) race and must be ordered by the
 * caller.  Errors: AMG_ERR_ARG (null or aliased pointers; a finest operator
 * whose product launch needs more partial sums than the array holds, i.e.
 * more than (AMG_NOALLOC_SCRATCH_BYTES - 256) / 16 workgroups), AMG_ERR_HIP. */
amg_status amg_true_residual_noalloc(amg_ctx *ctx, const double *b, const double *x, double *r,
                                     double *norms, double *rel);

/* ---- learned level-1 smoother blocks --------------------------------- */
/*
 * The level-1 block-Jacobi blocks M_i = omega_J A_ii^{-1} (Section 3) are
 * replaced by S_i = L_i (I + X_i) L_i^T, M_i = L_i L_i^T, X_i = sym(c .*
 * tanh(g_i)) with c = (.25,.25,.25,.05,.05,.05) and g_i the 6 outputs of a
 * per-node network 90 -> 64 -> 64 -> 6 (ReLU) on scale-free features of the
 * node's row of A: D_i/||D_i||_F (9) and diag(A_ij)/||D_i||_F at the 27
 * neighbour slots given by the sign pattern of the coordinate differences
 * (81).  sym(u) = [[u0,u3,u4],[u3,u1,u5],[u4,u5,u2]].  Every eigenvalue of
 * I + X_i lies in (0.65, 1.35), so the relaxation contracts the error in the
 * energy norm for any weights and the V-cycle stays symmetric positive
 * definite (plain CG applies).  Zero output weights give block Jacobi.
 * Parameters: AMG_MLP_PARAMS floats, W1[90][64] b1[64] W2[64][64] b2[64]
 * W3[64][6] b3[6] (row-major, input index first).
 */
#define AMG_MLP_PARAMS 10374

/* Compute S from theta (device, AMG_MLP_PARAMS parameters of type dtype:
 * AMG_FP32, or AMG_BF16 as 16-bit patterns widened to FP32 for the forward
 * pass; bytes must be AMG_MLP_PARAMS times 4 or 2) on the GPU and use it
 * for every level-1 relaxation of later solves (every precision; the
 * multi-right-hand-side solve too).  theta = NULL restores block Jacobi
 * (bytes and dtype ignored).
 * check = 1: a node whose S_i is not finite keeps M_i (count in *n_fallback,
 * may be NULL); check = 0 stores S as computed (lets a caller force the solve
 * path's fallback: a solve that meets a non-finite value with learned blocks
 * restores block Jacobi, restarts from the caller's x and sets fell_back).
 * Requires a context set up with smoother = AMG_SMOOTHER_LEARNED and at least
 * two levels (AMG_ERR_UNSUPPORTED otherwise).  Allocates nothing. */
amg_status amg_smoother_set_weights(amg_ctx *ctx, const void *theta, size_t bytes, int32_t dtype, int32_t check,
                                    int32_t *n_fallback);

/* Training step pieces (FP64 contexts with smoother = AMG_SMOOTHER_LEARNED).
 * Loss of theta over k error vectors E (device, column j at E + j*3*nb):
 *   l = mean_j  y_j^T A y_j / (e_j^T A e_j),  y_j = (I - P V_2(R A .)) (e_j - S A e_j),
 * the energy left after one learned relaxation and the coarse-grid
 * correction (V_2: the V-cycle from level 2).  grad (device, AMG_MLP_PARAMS
 * floats) receives scale * dl/dtheta (added to its contents if accumulate).
 * *loss (host) receives l.  Leaves S(theta) installed as the level-1
 * smoother.  The first call allocates the training buffers. */
amg_status amg_mlp_loss_grad(amg_ctx *ctx, const float *theta, const double *E, int32_t k, float scale,
                             int32_t accumulate, double *loss, float *grad);

/* Adam (Kingma and Ba) with bias correction on n device floats; step >= 1. */
amg_status amg_mlp_adam(amg_ctx *ctx, float *theta, const float *grad, float *m, float *v, int32_t n,
                        int32_t step, float lr, float beta1, float beta2, float eps);

/* Training errors from the method's own iteration: each of the k columns of
 * E (device, column j at E + j*3*nb) becomes e - V(A e), `cycles` times
 * (the context's current smoother and precision). */
amg_status amg_training_errors(amg_ctx *ctx, double *E, int32_t k, int32_t cycles);

#ifdef __cplusplus
}
#endif
#endif /* SAAMG_H */
