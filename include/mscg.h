/*
 * mscg.h -- C ABI of the recursive multi-scale preconditioned conjugate
 * gradient solver for -div(K grad p) = f on MI355X (gfx950).
 *
 * Method: Lackner & Menikoff, "Multi-scale linear solvers for very large
 * systems derived from PDEs".  The outer solver is preconditioned CG
 * (Section 2, eq. 2.2; Templates book, Section 2.3.1, Figure 2.5).  The
 * preconditioner is eq. 2.10 of Section 2.3, evaluated as a two-grid cycle:
 * m symmetric Gauss-Seidel steps of the splitting A = P - Q (eq. 2.3,
 * Section 3), a coarse correction E A_c^-1 R whose A_c^-1 is itself the same
 * PCG on the coarse-grained operator (Section 3, coarse-grained
 * transmissivities), recursing to a coarsest grid solved exactly, and m more
 * smoothing steps.  Level k stops when |r|^2 / N_k < f^k eps^2 (Section 3).
 *
 * Discretisation (Section 3): cell-centred 5-point (2-D) or 7-point (3-D)
 * finite volumes on a regular grid, diagonal permeability tensor, face values
 * by the harmonic mean of the two cells, transmissibility = K * face area /
 * cell width.  Boundary faces: Dirichlet T = 2 K area / width with the value
 * moved to the right-hand side, Neumann T = 0.
 *
 * Layout: every cell array is row-major with x fastest,
 * idx = i + nx * (j + ny * k); n[2] = 1 in 2-D.
 *
 * Memory: all array arguments are DEVICE pointers (hipMalloc'd or torch CUDA
 * tensors) unless stated otherwise; the caller owns them and they must stay
 * valid for the duration of the call.  All GPU work is ordered on the
 * problem's HIP stream; every call returns after that work has completed.
 *
 * Errors: functions return an mscg_status code; no exception crosses the
 * ABI.  Argument and state errors are detected before any launch.
 * mscg_last_error() gives a thread-local message for the last failure.
 *
 * Threading: distinct problems may be used from distinct threads; a single
 * problem is not reentrant.
 */
#ifndef MSCG_H
#define MSCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSCG_MAX_LEVELS 8
#define MSCG_MAX_COARSE 1024 /* largest coarsest level solved by dense factorisation */

typedef enum {
  MSCG_OK = 0,
  MSCG_NOT_CONVERGED = 1, /* hit max_outer_iters; stats are filled */
  MSCG_E_ARG = -1,        /* invalid argument (sizes, K <= 0 or not finite, ...) */
  MSCG_E_NOMEM = -2,      /* workspace too small or device allocation failed */
  MSCG_E_DEVICE = -3,     /* a HIP call failed */
  MSCG_E_BREAKDOWN = -4,  /* r.z <= 0 or p.Ap <= 0 or a non-finite reduction */
  MSCG_E_STATE = -5,      /* call out of order (solve before set_permeability) */
  MSCG_E_SINGULAR = -6    /* coarsest operator not positive definite (no Dirichlet face) */
} mscg_status;

enum { MSCG_NEUMANN = 0, MSCG_DIRICHLET = 1 };
enum { MSCG_FP64 = 0, MSCG_MIXED = 1 };
/* Extension operator E (Section 3): tensor product of 1-D linear interpolation
 * with zero slope at the boundary, or piecewise-constant interpolation (the
 * alternative the paper reports to work nearly as well). R = E^T. */
enum { MSCG_INTERP_LINEAR = 0, MSCG_INTERP_CONSTANT = 1 };
/* Splittings (Section 3): symmetric Gauss-Seidel in red-black order,
 * P = (D+L) D^-1 (D+U); or modified Jacobi, P = 2D, fully parallel (every
 * inner level then runs host-driven with grid-wide kernels). */
enum { MSCG_SPLIT_SGS = 0, MSCG_SPLIT_JACOBI = 1 };
/* Coarse part of the preconditioner on the inner levels.  RECURSIVE: the
 * recursive multi-scale PCG of eq. 2.10, A_c^-1 applied by an inner PCG on
 * each coarse level.  MGCG: Tatebe's multigrid preconditioner of eq. 2.9,
 * the next level's preconditioner M_{k+1}^-1 applied once (one V-shaped pass
 * per outer iteration, no inner PCG).  Both end with the exact coarsest
 * solve.  With MGCG every inner level runs host-driven with grid-wide kernels.
 * POLY: the polynomial preconditioner of Section 2.1 (W = P^-1), 2m+1 steps
 * of the splitting from zero on the finest level; the coarse levels are
 * still planned and set up but never visited. */
enum { MSCG_CYCLE_RECURSIVE = 0, MSCG_CYCLE_MGCG = 1, MSCG_CYCLE_POLY = 2 };

typedef struct {
  int dim;            /* 2 or 3 */
  int n[3];           /* cells per axis; n[2] is ignored in 2-D */
  double length[3];   /* domain extent per axis; <= 0 means 1 */
  int bc_type[6];     /* faces -x, +x, -y, +y, -z, +z: MSCG_NEUMANN or MSCG_DIRICHLET */
  double bc_value[6]; /* Dirichlet values per face */
} mscg_grid;

typedef struct {
  int precision;          /* MSCG_FP64 (default) or MSCG_MIXED */
  int scale;              /* coarsening factor per axis between levels, default 4 (Section 3) */
  int smooth_steps;       /* m, default = scale (Section 3) */
  double level_factor;    /* f of the per-level criterion, default 0.1 (Section 3) */
  int min_coarse_side;    /* coarsen while every side / scale >= this, default 8 */
  int max_levels;         /* default MSCG_MAX_LEVELS */
  int max_outer_iters;    /* default 200 */
  int max_inner_iters;    /* per inner PCG call, default 200 */
  int interp;             /* MSCG_INTERP_LINEAR (default) or MSCG_INTERP_CONSTANT */
  int flexible;           /* beta on the host-driven levels: 0 Fletcher-Reeves (Templates CG, default),
                             1 Polak-Ribiere, robust to a preconditioner that varies between iterations */
  double inner_rel_floor; /* MIXED only: inner levels stop once |r| <= floor * |rhs| (default 1e-6) */
  int semi_coarsen;       /* 0: every axis coarsened together (default).  1: aspect-ratio-aware plan
                             (Section 5, anisotropic strip): per level, among the axes that can be
                             coarsened by `scale`, those whose effective cell size h_a / sqrt(axis_weight[a])
                             is within sqrt(scale) of the smallest are coarsened */
  double axis_weight[3];  /* permeability scale per axis for that plan (e.g. 1, 1, kz/kx), default 1 */
  int splitting;          /* operator splitting A = P - Q of the smoother (eq. 2.3, Section 3):
                             MSCG_SPLIT_SGS (default) or MSCG_SPLIT_JACOBI */
  int cycle;              /* MSCG_CYCLE_RECURSIVE (default, eq. 2.10), MSCG_CYCLE_MGCG (eq. 2.9) or
                             MSCG_CYCLE_POLY (Section 2.1) */
  double frac_scale;      /* 0 (default): integer factor `scale` with exact division.  > 1: a factor that
                             need not be an integer (Section 3): each coarsened axis goes from d to
                             round(d / frac_scale) cells while every result is >= min_coarse_side and
                             < d, and the coarse graining weights partly overlapping fine faces by the
                             fractions of the overlap.  Such hierarchies run host-driven with grid-wide
                             kernels on every level; not combined with semi_coarsen */
} mscg_options;

typedef struct {
  int status;             /* mscg_status of this solve */
  int outer_iters;        /* iterations on the finest level */
  int n_levels;
  int level_n[MSCG_MAX_LEVELS][3];
  long long level_iters[MSCG_MAX_LEVELS]; /* CG iterations summed over calls (Table 1 of the paper) */
  long long level_calls[MSCG_MAX_LEVELS]; /* solver calls per level (coarsest: direct solves) */
  double rel_residual_true; /* |b - A p| / |b| recomputed in FP64 after the solve */
  double b_norm;
  double solve_ms;        /* wall time of the solve on the host clock */
} mscg_stats;

typedef struct mscg_problem mscg_problem;

/* Fills the defaults listed above. */
void mscg_default_options(mscg_options *opt);

/* Device bytes the problem needs for its hierarchy and work vectors; 0 if the
 * grid or options are invalid (see mscg_last_error). */
size_t mscg_footprint_bytes(const mscg_grid *grid, const mscg_options *opt);

/* Plans the level hierarchy (Section 3: scale factor 4, coarsen while every
 * side / scale >= min_coarse_side with exact divisibility; the coarsest level
 * must have at most MSCG_MAX_COARSE cells) and carves it out of `workspace`
 * (device, >= mscg_footprint_bytes bytes, 256-byte aligned).  workspace ==
 * NULL makes the library allocate it and free it on destroy.  hip_stream is a
 * hipStream_t (NULL = default stream).  opt == NULL takes the defaults. */
int mscg_create_problem(const mscg_grid *grid, const mscg_options *opt, void *workspace, size_t ws_bytes,
                        void *hip_stream, mscg_problem **out);

/* Sets the cell-centred permeabilities (device, N doubles each; ky == NULL
 * means ky = kx; in 3-D kz == NULL means kz = kx) and builds the hierarchy on
 * the device: face transmissibilities (Section 3, harmonic mean), the
 * coarse-grained transmissivities of every level (Section 3: series sum over
 * the parallel sums, partial overlaps weighted by fraction), and the FP64
 * factorisation of the coarsest operator.  Returns MSCG_E_ARG if any K is not
 * finite and > 0, MSCG_E_SINGULAR if the coarsest operator is not positive
 * definite. */
int mscg_set_permeability(mscg_problem *prob, const double *kx, const double *ky, const double *kz);

/* Solves A p = b with b_c = f_c |V_c| plus T_b p_D on Dirichlet faces (device
 * f, p: N doubles).  Stops when |b - A p| <= rel_tol |b| on the recursively
 * updated residual; stats (may be NULL) report the true residual recomputed
 * afterwards.  use_x0 != 0 starts from the p passed in; otherwise from the
 * linear ramp between the two x-face Dirichlet values when only those faces
 * are Dirichlet (Section 3, lifting by a smooth boundary field), else zero.
 * Returns the stats status. */
int mscg_solve(mscg_problem *prob, const double *f, double *p, double rel_tol, int use_x0, mscg_stats *stats);

/* Solves `count` independent problems (any mix of sizes), overlapping their
 * GPU work; f[i], p[i] as in mscg_solve for probs[i].  Problems must be
 * distinct; each runs on its own stream.  stats: array of count (may be
 * NULL).  Returns the worst status (errors first, then NOT_CONVERGED). */
int mscg_solve_batch(mscg_problem *const *probs, const double *const *f, double *const *p, const double *rel_tol,
                     int count, mscg_stats *stats);

int mscg_destroy_problem(mscg_problem *prob);

/* Thread-local description of the last error, "" if none. */
const char *mscg_last_error(void);

/* ---- Operator-level entry points (same kernels the solver runs) ---- */

/* Level count and cell dims of level `level` (0 = finest). */
int mscg_level_info(const mscg_problem *prob, int level, int dims[3]);

/* Copies the FP64 face transmissibilities of a level (device outputs sized
 * (nx+1)ny nz, nx(ny+1)nz, nx ny(nz+1); tz ignored in 2-D). */
int mscg_get_transmissibility(const mscg_problem *prob, int level, double *tx, double *ty, double *tz);

/* y = A_level x (Section 3 operator; device, N_level doubles). */
int mscg_apply_operator(mscg_problem *prob, int level, const double *x, double *y);

/* steps symmetric Gauss-Seidel steps x <- x + P^-1 (r - A x) in red-black
 * order on a level, in place (eq. 2.3 splitting; device). */
int mscg_apply_smoother(mscg_problem *prob, int level, const double *r, double *x, int steps);

/* g_coarse = R (r_fine - A x_fine) between level and level + 1 (R = E^T;
 * x_fine may be NULL for zero).  MSCG_E_ARG on hierarchies with a
 * non-integer frac_scale (their restriction works on a stored residual). */
int mscg_restrict_residual(mscg_problem *prob, int level, const double *r_fine, const double *x_fine, double *g_coarse);

/* x_fine += E y_coarse between level and level + 1 (any factor). */
int mscg_prolong_add(mscg_problem *prob, int level, const double *y_coarse, double *x_fine);

/* z = M_0^-1 r, the finest-level preconditioner of eq. 2.10 with inner
 * levels stopped at |r_k|^2 / N_k < f^k eps2 (eps2 = 0 runs them to
 * max_inner_iters); with MSCG_CYCLE_MGCG eq. 2.9, with MSCG_CYCLE_POLY the
 * polynomial preconditioner (eps2 unused).  FP64 problems only. */
int mscg_apply_preconditioner(mscg_problem *prob, const double *r, double *z, double eps2);

/* ---- Measurement ---- */

enum {
  MSCG_KERNEL_SMOOTH_HALF = 0, /* one red-black Gauss-Seidel half sweep */
  MSCG_KERNEL_SPMV = 1,        /* q = A p with the partial sums of p.q */
  MSCG_KERNEL_RESTRICT = 2,    /* g = R (r - A x) */
  MSCG_KERNEL_PROLONG = 3,     /* x += E y */
  MSCG_KERNEL_CG_UPDATE = 4,   /* x += alpha p, r -= alpha q with partial |r|^2 */
  MSCG_KERNEL_SMOOTH_PRE = 5,  /* m SGS steps from zero, one tiled launch (2-D, m = 4) */
  MSCG_KERNEL_SMOOTH_POST = 6  /* prolongation + m SGS steps, one tiled launch (2-D, m = 4) */
};

/* Launches one solver kernel `reps` times back to back on the problem's
 * stream, with the launch configuration the solver uses on `level`, and
 * reports its average duration (HIP events) and its algorithmic bytes per
 * launch: every operand array read once and written once.  Operates on the
 * problem's own work vectors (their contents are overwritten).  Needs
 * mscg_set_permeability; run a solve first so the vectors hold finite values.
 * MSCG_KERNEL_RESTRICT and MSCG_KERNEL_SMOOTH_POST are not available on
 * hierarchies with a non-integer frac_scale (MSCG_E_ARG). */
int mscg_time_kernel(mscg_problem *prob, int kernel, int level, int reps, double *avg_us, double *alg_bytes);

/* Launch timing of the one-workgroup solver of the last inner level (the
 * inner PCG of the level above the coarsest grid, Section 2.3, with its
 * coarsest solve), available for 2-D hierarchies of three or more levels
 * whose last inner level runs in one workgroup (MSCG_E_ARG otherwise).
 * on = 1 clears the totals and brackets each of its launches in the following
 * solves with HIP events on the problem's stream; on = 0 stops recording. */
int mscg_enable_kernel_timing(mscg_problem *prob, int on);

/* Totals since timing was enabled: summed launch durations (ms, HIP events),
 * launches (every dispatch, including those of iterations queued past
 * convergence, which return at once), iterations of that level, and their
 * algorithmic FP64 operations: per iteration (9 (2m+1) + 45) n + 4 ny ncx +
 * 2 nc^2 for a level of n cells (ny rows) above a coarsest level of nc cells
 * (ncx columns).  Any pointer may be NULL. */
int mscg_small_level_timing(const mscg_problem *prob, double *total_ms, long long *launches, long long *iterations,
                            double *flops);

#ifdef __cplusplus
}
#endif

#endif /* MSCG_H */
