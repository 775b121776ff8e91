/*
 * sym.h -- C ABI of an MI355X (gfx950) library for the numeric phase of
 * decoupled sparse Cholesky: supernodal A = L L^T and sparse triangular
 * solve L x = b with a dense or reach-set-pruned sparse right-hand side.
 *
 * Problem statement (Cheshmi et al., "Sympiler", 2017): A is symmetric
 * positive definite (Section 3.2), stored as its lower triangle in
 * compressed sparse column form (Section 1.1, CSC {n, Lp, Li, Lx}); its
 * pattern stays fixed while its values change (Section 1.2), so the
 * symbolic analysis runs once and the numeric phase many times (Section
 * 4.3); the right-hand side's pattern drives the reach-set inspector of the
 * triangular solve (Section 3, the inspection-set table).
 *
 * Conventions for every call:
 *   - Indices are 0-based.  Orderings map new to old: perm[new] = old.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - Device pointers are caller-owned buffers on the GPU that is current
 *     when the call is made; the library never allocates device memory.
 *     All of its device state lives in one caller-allocated workspace.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Device work is asynchronous on that stream; no call except
 *     sym_status and sym_export_factor synchronizes with the host.
 *   - Return value 0 is success, negative values are the SYM_E* codes.
 *     No exception crosses the ABI.
 *   - A handle is not thread-safe: issue its calls on one stream at a time.
 */
#ifndef SYM_H
#define SYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SYM_OK 0
#define SYM_EINVAL (-1)     /* null pointer, n < 0, bad option value */
#define SYM_EPATTERN (-2)   /* entry above the diagonal, row out of range, duplicate (i, j) */
#define SYM_ENOMEM (-3)     /* host allocation failed */
#define SYM_EHIP (-4)       /* a HIP runtime call failed */
#define SYM_ESTATE (-5)     /* call out of order: e.g. factor before bind, solve before factor */
#define SYM_EWORKSPACE (-6) /* workspace too small or misaligned */
#define SYM_ESCHED (-7)     /* a device scheduler gave up waiting (internal error) */
#define SYM_ENUMERIC (-8)   /* refinement on a failed factor (a non-positive pivot), or its
                               backward error is not finite (NaN or infinity) */

/* orderings */
#define SYM_ORDER_ND 0      /* the library's own graph nested dissection */
#define SYM_ORDER_NATURAL 1 /* identity */
#define SYM_ORDER_USER 2    /* opts.perm, used exactly as given */

/* factor precision.
 *   SYM_F64: FP64 panels and arithmetic.
 *   SYM_F32: FP32 panels and arithmetic; the factorization of every diagonal
 *     block runs in FP64 (its result rounded once to FP32).
 *   SYM_BF16, SYM_F16: FP32 panels, the matrix scaled per device supernode
 *     (D P A P^T D, D a power of two constant on each device supernode, from
 *     the supernode's largest diagonal entry), and the Schur-complement
 *     update products -- the supernodal update of Section 3.2, external and
 *     internal -- on the bfloat16 / IEEE-half matrix cores: operands rounded
 *     to 16 bits, products accumulated in FP32.  Diagonal factorization in
 *     FP64 as for SYM_F32, off-diagonal triangular solves in FP32.  A pivot
 *     below tau times its column's diagonal entry of the scaled matrix is
 *     replaced by that value (tau = 2^pivot_floor_exp; see sym_opts and
 *     sym_pivots_perturbed).  The solves undo the scaling, so every call
 *     keeps its meaning (sym_export_factor returns the factor of P A P^T).
 * Factors below FP64 are for iterative refinement (sym_refine,
 * sym_refine_pcg). */
#define SYM_F64 0
#define SYM_F32 1
#define SYM_BF16 2
#define SYM_F16 3
/* default pivot-floor exponents of the 16-bit update precisions */
#define SYM_PIVOT_FLOOR_DEFAULT_BF16 (-20)
#define SYM_PIVOT_FLOOR_DEFAULT_F16 (-24)

typedef struct sym_opts {
    int32_t ordering;        /* SYM_ORDER_* (default SYM_ORDER_ND) */
    const int32_t *perm;     /* host int32[n], perm[new] = old, for SYM_ORDER_USER */
    int32_t block_width;     /* widest column block a device task handles (default 64; 16..64, multiple of 16) */
    int32_t precision;       /* SYM_F64 (default), SYM_F32, SYM_BF16 or SYM_F16 (see above) */
    int32_t nd_leaf;         /* SYM_ORDER_ND: subgraphs up to this size are not split further (default 24) */
    int32_t amalgamate;      /* 1 (default): merge small supernodes into device panels with explicit
                                zeros; 0: device panels are the fundamental supernodes.  Reported
                                symbolic outputs are the fundamental ones either way. */
    int32_t pivot_floor_exp; /* SYM_BF16 / SYM_F16: tau = 2^pivot_floor_exp (-60..0); 0 = the
                                format's default; 1 = no floor.  Ignored otherwise. */
    int32_t max_super_width; /* widest device supernode, 1..16384 (0 = 16384); wider ones, and
                                ones whose w x r panel reaches 4 GiB, are cut into pieces of
                                consecutive columns (device panels only; the reported
                                supernodes stay the fundamental ones) */
    int32_t split_share;     /* an external-update tile costing more than max(64, level cost /
                                split_share) units (16-wide inner batches) is cut into parts of
                                about that size, run by separate workgroups (0 = 12288;
                                1..2^24) */
    int32_t chain_launch;    /* 0 (default): the steps inside the supernodes of a level (off-diagonal
                                solves of their first blocks, then for every later block its update
                                by the previous one, its factorization and its solves) run as one
                                launch per step and kind; 1: as one persistent launch per level
                                whose tasks wait for the tiles they read (same results, bit for
                                bit; measured slower on this chip, kept for comparison) */
    int32_t update_depth;    /* step launches (chain_launch 0): the updates of a supernode's later
                                blocks by its column blocks are applied in groups of this many
                                consecutive blocks, as one product per target tile with an inner
                                dimension of up to update_depth x block_width; inside a group each
                                block updates only the group's later blocks (0 = 4; 1 = one block
                                at a time; at most 16).  Same factor up to rounding order. */
    int32_t reserved[2];
} sym_opts;

typedef struct sym_plan *sym_handle;
typedef struct sym_rhs_plan *sym_rhs;

/* Fill *opts with the defaults listed above. */
void sym_opts_default(sym_opts *opts);

/*
 * Symbolic analysis, host only (Section 3.2, Eq. (1) and the supernode rule
 * after it; Section 3.1 for the solve).  Input: the lower triangle of A in
 * CSC, Ap int64[n+1], Ai int32[Ap[n]] with Ai[p] >= j for p in column j;
 * rows may be unsorted; a missing diagonal is accepted structurally.
 * Computes the fill-reducing ordering, the elimination tree
 * parent[j] = min{i > j : L_ij != 0}, column counts, fundamental
 * supernodes, their row patterns, the device task blocks, level sets and
 * descendant lists, and the map from A's entries to L's storage.
 * opts may be NULL for defaults.  On success *out owns a new handle.
 * Errors: SYM_EINVAL, SYM_EPATTERN, SYM_ENOMEM.
 */
int sym_analyze(int64_t n, const int64_t *Ap, const int32_t *Ai, const sym_opts *opts,
                sym_handle *out);

/* Bytes of device workspace the handle needs (factor, solve and plan). */
int sym_workspace(sym_handle h, size_t *bytes);

/*
 * Attach a caller-allocated device workspace of at least sym_workspace
 * bytes, 256-byte aligned, and upload the plan into it asynchronously on
 * `stream`.  The workspace must stay allocated until sym_destroy or the next
 * sym_bind.  Errors: SYM_EINVAL, SYM_EWORKSPACE, SYM_EHIP.
 */
int sym_bind(sym_handle h, void *dev_ws, size_t bytes, void *stream);

/*
 * Numeric factorization P A P^T = L L^T (Section 3.2: supernodal
 * left-looking Cholesky with dense factorization of each diagonal block and
 * dense triangular solves for the rows below it).  Ax_dev: device
 * double[nnz(A)] in the order of the Ai given to sym_analyze.  Asynchronous.
 * The factorization ends by storing, for the triangular solves, the inverse
 * of each diagonal block in the block's otherwise unused upper triangle.
 * A non-positive pivot is not an error return: it is recorded on the device
 * and reported by sym_status.  Errors: SYM_EINVAL, SYM_ESTATE (not bound),
 * SYM_EHIP.
 */
int sym_factor(sym_handle h, const double *Ax_dev, void *stream);

/*
 * Full solve A x = b, in place: bx_dev (device double[n], original
 * ordering) holds b on entry and x = P^T L^-T L^-1 P b on exit (Section 3.1:
 * the diagonal block of each column block is solved first, then its result
 * is applied to the rows below it).  Errors: SYM_EINVAL, SYM_ESTATE (no
 * factor), SYM_EHIP.
 */
int sym_solve(sym_handle h, double *bx_dev, void *stream);

/*
 * For callers that cannot allocate device memory or must not touch the
 * handle's scratch (code under graph capture, serving loops): the full
 * solve of sym_solve, with the sweeps' scratch -- the accumulator and
 * forward-result vectors, per-block counters, done flags and ticket word --
 * taken from a fixed static device array of the library instead of the
 * bound workspace (which still supplies the plan and the factor).  The
 * array holds n and block counts up to SYM_STATIC_MAX_N (about 12.6 MB per
 * GPU, resident from the first call on that GPU until the process ends).
 * The call allocates nothing.  All calls on one GPU share the array: calls
 * that overlap in time on one GPU (other streams, other threads, other
 * handles) race and give wrong results; serialize them.  Every value it
 * needs cleared is reset by a kernel at the start of each sweep.  Errors:
 * SYM_EINVAL, SYM_EWORKSPACE (n or the number of device blocks exceeds
 * SYM_STATIC_MAX_N), SYM_ESTATE (no factor), SYM_EHIP.
 */
#define SYM_STATIC_MAX_N 524288
int sym_solve_static(sym_handle h, double *bx_dev, void *stream);

/*
 * Forward sweep only: y = L^-1 P b.  b_dev: device double[n] in the
 * original ordering (read only); y_dev: device double[n] in the permuted
 * ordering of L (written).  Errors as sym_solve.
 */
int sym_solve_lower(sym_handle h, const double *b_dev, double *y_dev, void *stream);

/*
 * Backward sweep only, in place: x = L^-T y for y_dev in the permuted
 * ordering of L.  Errors as sym_solve.
 */
int sym_solve_upper(sym_handle h, double *y_dev, void *stream);

/*
 * Solve A x = b with the current factor (FP64, or FP32 for mixed precision)
 * and FP64 iterative refinement on the device: x0 = P^T L^-T L^-1 P b, then
 * repeatedly r = b - A x in FP64 (Ax_dev: the values the factor was computed
 * from, in sym_analyze's order), eta = ||r||_inf / (||A||_inf ||x||_inf +
 * ||b||_inf) (normwise backward error), stopping when eta <= tol or after
 * maxit corrections, else x += solve(r).  b_dev, x_dev: device double[n],
 * original ordering, distinct.  Synchronizes the stream once per iteration
 * to read eta.  *iters (may be NULL): corrections applied; *eta (may be
 * NULL): final backward error.  A NaN anywhere in r or x makes eta NaN.
 * Errors: SYM_EINVAL, SYM_ESTATE (no factor), SYM_EHIP, SYM_ENUMERIC (the
 * factor recorded a non-positive pivot, or eta is not finite; *iters and
 * *eta still hold what was reached).
 */
int sym_refine(sym_handle h, const double *Ax_dev, const double *b_dev, double *x_dev, double tol,
               int32_t maxit, void *stream, int32_t *iters, double *eta);

/*
 * The same solve with the refinement accelerated by conjugate gradients:
 * preconditioned CG in FP64 on A x = b, the preconditioner being the
 * current factor (M = P^T L^-T L^-1 P, symmetric positive definite like A,
 * so CG applies), started from x0 = M b.  Every step computes the true FP64
 * residual r = b - A x (used in place of the recurrence) and its eta as
 * sym_refine; the stopping rule and outputs are those of sym_refine, with
 * *iters counting applications of M after the first.  Dot products are
 * reduced in a fixed order (bitwise reproducible).  Synchronizes the
 * stream three times per step.  Errors as sym_refine.
 */
int sym_refine_pcg(sym_handle h, const double *Ax_dev, const double *b_dev, double *x_dev,
                   double tol, int32_t maxit, void *stream, int32_t *iters, double *eta);

/*
 * Reach-set inspector for one right-hand-side pattern, host only (Section
 * 1.1, Gilbert-Peierls: Reach_L(beta) is the set of columns reachable in the
 * dependence graph of L from beta = {i : b_i != 0}; numerical cancellation
 * is neglected).  bi: host int32[nb], distinct positions in the original
 * ordering.  The result is reused for every numeric solve with that
 * pattern.  Errors: SYM_EINVAL, SYM_ENOMEM.
 */
int sym_rhs_analyze(sym_handle h, int64_t nb, const int32_t *bi, sym_rhs *out);

/* Device workspace bytes for an RHS plan, and its asynchronous upload into
 * a caller buffer (256-byte aligned).  Errors as sym_workspace / sym_bind. */
int sym_rhs_workspace(sym_rhs r, size_t *bytes);
int sym_rhs_bind(sym_rhs r, void *dev_ws, size_t bytes, void *stream);

/*
 * Reach-pruned forward solve y = L^-1 P b for a sparse b (Section 1.1, the
 * decoupled code: only columns in the reach set are visited).  bv_dev:
 * device double[nb], the values at the positions given to sym_rhs_analyze.
 * y_dev: device double[n], permuted ordering; every entry outside the reach
 * set is written as exactly 0.  Errors: SYM_EINVAL, SYM_ESTATE, SYM_EHIP.
 */
int sym_solve_lower_sparse(sym_handle h, sym_rhs r, const double *bv_dev, double *y_dev,
                           void *stream);

/*
 * Full solve A x = b for a sparse b: the reach-pruned forward sweep of
 * sym_solve_lower_sparse (Section 1.1), then the backward sweep over every
 * block (the transposed sweep's reach from a root path covers nearly all
 * of L), then the permutation back.  bv_dev: device double[nb], values at
 * the positions given to sym_rhs_analyze; x_dev: device double[n], original
 * ordering (written).  Errors as sym_solve_lower_sparse.
 */
int sym_solve_sparse(sym_handle h, sym_rhs r, const double *bv_dev, double *x_dev, void *stream);

/* Synchronize the bound stream and return the factorization status:
 * *info = 0, or 1 + the original index of the first column whose pivot was
 * not positive (first in elimination order).  Errors: SYM_ESTATE, SYM_EHIP. */
int sym_status(sym_handle h, int64_t *info);

/* The number of pivots the last factorization replaced by their floor
 * (SYM_BF16 / SYM_F16 factors; 0 otherwise).  Synchronizes the bound
 * stream.  Errors: SYM_EINVAL, SYM_ESTATE, SYM_EHIP. */
int sym_pivots_perturbed(sym_handle h, int64_t *count);

/* Copy the factor into compressed sparse column form on the host, in the
 * pattern returned by SYM_GET_LP / SYM_GET_LI (diagonal first, rows
 * increasing).  Lx_host: double[nnz(L)].  Synchronizes the stream. */
int sym_export_factor(sym_handle h, double *Lx_host, void *stream);

/* Symbolic outputs for inspection and tests.  sym_get_size gives the element
 * count of an array; sym_get copies it into a host buffer of that many
 * elements of the listed type. */
#define SYM_GET_PERM 1        /* int32[n]   perm[new] = old */
#define SYM_GET_PARENT 2      /* int32[n]   elimination tree, permuted numbering, -1 = root */
#define SYM_GET_COLCOUNT 3    /* int64[n]   |L_j| including the diagonal */
#define SYM_GET_LP 4          /* int64[n+1] column pointers of L */
#define SYM_GET_LI 5          /* int32[nnz(L)] row indices of L, diagonal first */
#define SYM_GET_SUPER 6       /* int32[ns+1] first column of each fundamental supernode, then n */
#define SYM_GET_SPARENT 7     /* int32[ns]  supernodal elimination tree */
#define SYM_GET_BLOCKS 8      /* int32[nb+1] first column of each device block, then n */
#define SYM_GET_BLEVEL 9      /* int32[nb]  level of each block (leaves 0) */
#define SYM_GET_SUPER_FEAT 10 /* double[nds*12] features of each device supernode (see below) */
#define SYM_GET_TASK_SUPER 11 /* int32[ntasks] device supernode an external-update task
                                 updates, -1 for the factor's other tasks */
#define SYM_GET_VARIANT 12    /* uint8[nds] kernel variant of each device supernode */
int sym_get_size(sym_handle h, int what, int64_t *count);
int sym_get(sym_handle h, int what, void *out);

/* Reach set of an RHS plan: int32 columns (permuted numbering), increasing. */
int sym_rhs_get(sym_rhs r, int64_t *count, int32_t *cols_or_null);

/* Scalar statistics. */
#define SYM_STAT_N 1
#define SYM_STAT_NNZA 2
#define SYM_STAT_NNZL 3
#define SYM_STAT_FLOPS 4          /* sum_j |L_j|^2: multiplies, adds, divides and square roots */
#define SYM_STAT_NSUPER 5
#define SYM_STAT_NBLOCKS 6
#define SYM_STAT_NLEVELS 7
#define SYM_STAT_NPAIRS 8         /* (descendant block, target block) update pairs */
#define SYM_STAT_PANEL_ENTRIES 9  /* stored panel entries, incl. each diagonal block's upper part */
#define SYM_STAT_ANALYZE_MS 10
#define SYM_STAT_SUM_ROWS 11      /* sum over blocks of their row counts */
#define SYM_STAT_NPHASES 12       /* kernel launches of one factorization (excluding scatter) */
#define SYM_STAT_NINCIDENCES 13   /* (row tile, descendant block) incidences of the factor */
#define SYM_STAT_NSLEVELS 14      /* levels of the device supernodal elimination tree */
#define SYM_STAT_NDSUPER 15       /* device supernodes (after amalgamation) */
#define SYM_STAT_STORED_LOWER 16  /* lower-trapezoid entries stored (nnz(L) plus explicit zeros) */
#define SYM_STAT_WALKERS 18        /* backward-sweep walkers: the (at most 64) device supernodes of
                                     three or more blocks with the most blocks, whose diagonal chain
                                     one workgroup walks; used while value sets x walkers <= 128 */
#define SYM_STAT_EXT_OPERAND_ENTRIES 17 /* panel entries the external-update products read, without
                                           cache reuse: sum of (rows + columns) x inner dimension */
int sym_stat(sym_handle h, int what, double *value);

/* Per-launch timing of the factorization for measurement.  With enable != 0,
 * every later sym_factor brackets each of its kernel launches with HIP
 * events on its stream (a small overhead).  sym_profile_read synchronizes
 * the stream and returns, for the most recent sym_factor, the summed event
 * time in ms and the launch count of each kernel kind:
 *   [0] A scatter (zero fill + placement), [1] external (descendant)
 *   updates, [2] off-diagonal triangular solves and the diagonal-block
 *   inverses, [3] internal updates and the factorizations of leaf blocks
 *   (single narrow tiles that no update reaches).
 * algorithmic_flops[k] is the arithmetic each kind performs by the
 * method's count (lower-triangle products only), from the analysis.
 * Arrays hold SYM_PROFILE_KINDS entries.  Errors: SYM_EINVAL, SYM_ESTATE,
 * SYM_EHIP. */
#define SYM_PROFILE_KINDS 4
int sym_profile(sym_handle h, int enable);
int sym_profile_read(sym_handle h, double *ms, int64_t *launches, double *algorithmic_flops);

/*
 * Per-supernode kernel variants (the choices a cost model makes).  The
 * external update of device supernode s (nds = SYM_STAT_NDSUPER of them)
 * runs its incidences -- (row tile, descendant) products -- either all as
 * per-wavefront items (variant 0), or, for those with at least 64 (variant
 * 1, the default) or 32 (variant 2) rows, columns and inner indices, on
 * the whole workgroup through LDS, or all as staged chunks whose rows are
 * read once per tile into LDS (variant 3).  Results do not depend on the
 * variant beyond rounding order.  SYM_GET_SUPER_FEAT gives 12 features per
 * device supernode: width, rows, row tiles receiving updates, incidences
 * received, their product flops, the fractions of those flops in
 * incidences of >= 64 and >= 32 rows, columns and inner indices, level;
 * then the context of its level (the supernodes whose updates share its
 * launches): the level's update flops, its number of supernodes, its row
 * tiles receiving updates, and this supernode's share of the level's
 * update flops.
 *
 * sym_set_variants: variant[nds] (values 0..3) for every device supernode;
 * rebuilds the schedule on the host, so the workspace size may change and
 * the handle must be bound again (it is left unbound).  Errors:
 * SYM_EINVAL (count != nds or a value > 3).
 *
 * sym_task_times: for the most recent sym_factor run with profiling
 * enabled (sym_profile), the duration in microseconds of every factor
 * task's workgroup (us[ntasks], ntasks = SYM_GET_TASK_SUPER's count);
 * external-update tasks only, the others read 0.  Synchronizes.  Errors:
 * SYM_EINVAL, SYM_ESTATE (not bound), SYM_EHIP.
 */
int sym_set_variants(sym_handle h, const uint8_t *variant, int32_t count);
int sym_task_times(sym_handle h, double *us);

/*
 * The cost model's network (the learned part of kernel-variant selection):
 * fully connected, FP32, d_in inputs (1..32), two hidden layers of
 * SYM_MLP_HIDDEN ReLU units, one linear output.  Parameters are one flat
 * device float array of sym_mlp_param_count(d_in) entries: W1[64][d_in]
 * (row j = unit j's input weights), b1[64], W2[64][64], b2[64], w3[64], b3.
 * Samples: X_dev float[n][d_in] row-major; targets and outputs float[n].
 *
 * sym_mlp_forward: y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 per sample.
 * sym_mlp_backward: grad_dev = the gradient, with respect to every
 * parameter, of the mean squared error (1/n) sum (y - t)^2; work_dev:
 * caller scratch of sym_mlp_work_size(n, d_in) floats.  Each gradient
 * entry is a sum over samples in a fixed order -- 64 chunks of consecutive
 * samples, each summed in sample order, then the chunk sums in chunk order
 * -- so gradients are bitwise reproducible.
 * sym_mlp_work_size: *floats = n * (4 * 64 + 1) + 64 * param_count.
 * sym_mlp_adam: one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step
 * counted from 1) on params_dev with moment buffers m_dev, v_dev.
 * All run on `stream` without synchronizing.  Errors: SYM_EINVAL, SYM_EHIP.
 */
#define SYM_MLP_HIDDEN 64
int sym_mlp_param_count(int32_t d_in, int64_t *count);
int sym_mlp_work_size(int32_t n, int32_t d_in, int64_t *floats);
int sym_mlp_forward(const float *params_dev, const float *X_dev, int32_t n, int32_t d_in,
                    float *y_dev, void *stream);
int sym_mlp_backward(const float *params_dev, const float *X_dev, const float *t_dev, int32_t n,
                     int32_t d_in, float *grad_dev, float *work_dev, void *stream);
int sym_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                 int64_t count, int32_t step, float lr, void *stream);

/*
 * Batches: m value sets on the pattern of one analysis (Section 1.2: the
 * pattern is fixed while the values change), factored and solved together,
 * one launch per step of the schedule for all m (the instances occupy the
 * launches' second grid dimension).  The batch uses the analysis's bound
 * plan (h must stay bound and alive) and owns, in its own caller-allocated
 * workspace, m sets of panels, scratch vectors, status words and sweep
 * counters.  Layouts: Ax_dev is m x nnz(A) (instance-major, each in
 * sym_analyze's order); right-hand sides and solutions are m x n, original
 * ordering.  No batch call except sym_batch_eta and sym_batch_status
 * synchronizes; none allocates or records a memset, so a sequence of them
 * can be captured into a HIP graph and replayed.
 *
 * sym_batch_create: 1 <= m <= 65535.  sym_batch_bind: h must be bound
 * (SYM_ESTATE otherwise); alignment and size rules as sym_bind.  The batch
 * holds the analysis's device plan as it was at sym_batch_bind: after a
 * later sym_bind or sym_set_variants on h every batch call returns
 * SYM_ESTATE until the batch is bound again.
 * sym_batch_factor: factor all m value sets.  sym_batch_solve: in place,
 * A_i x_i = b_i for every instance.  sym_batch_refine: x_i = solve(b_i)
 * followed by exactly `steps` FP64 refinement steps r = b - A x, x +=
 * solve(r) (no stopping test, so no host synchronization).
 * sym_batch_eta: eta_host[i] = the normwise backward error of x_i (as
 * sym_refine).  sym_batch_status: info_host[i] as sym_status for instance
 * i; returns SYM_ESCHED if any instance's device scheduler gave up.
 */
typedef struct sym_batch *sym_batch_t;
int sym_batch_create(sym_handle h, int32_t m, sym_batch_t *out);
int sym_batch_workspace(sym_batch_t b, size_t *bytes);
int sym_batch_bind(sym_batch_t b, void *dev_ws, size_t bytes, void *stream);
int sym_batch_factor(sym_batch_t b, const double *Ax_dev, void *stream);
int sym_batch_solve(sym_batch_t b, double *bx_dev, void *stream);
int sym_batch_refine(sym_batch_t b, const double *Ax_dev, const double *b_dev, double *x_dev,
                     int32_t steps, void *stream);
int sym_batch_eta(sym_batch_t b, const double *Ax_dev, const double *b_dev, const double *x_dev,
                  double *eta_host, void *stream);
int sym_batch_status(sym_batch_t b, int64_t *info_host);
void sym_batch_destroy(sym_batch_t b);

void sym_destroy(sym_handle h);
void sym_rhs_destroy(sym_rhs r);

#ifdef __cplusplus
}
#endif
#endif /* SYM_H */
