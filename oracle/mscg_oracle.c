/*
 * mscg_oracle.c -- plain, slow FP64 reference of the recursive multi-scale
 * preconditioned conjugate gradient (Lackner & Menikoff, "Multi-scale linear
 * solvers for very large systems derived from PDEs").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the GPU
 * path.
 *
 * Every routine follows one passage of the paper, cited in its comment.  Where
 * the paper is silent the reading used is stated at the routine (the same
 * readings are applied by the GPU path):
 *   - boundary faces: Dirichlet face T = 2 K_cell area / width (value held at
 *     the face, half a cell from the centre); Neumann face T = 0;
 *   - coarse graining acts on the face-centred T over staggered control
 *     volumes, parallel sums first, then series sums weighted by overlap;
 *   - scale factor 4 on every coarsened axis, exact divisibility, coarsen
 *     while every coarsened side / 4 >= min_side;
 *   - red-black ordering of the symmetric Gauss-Seidel splitting (red =
 *     (i+j+k) even, red first);
 *   - R is the unscaled transpose of E;
 *   - an entry check of the convergence criterion before the first iteration
 *     on every level; inner levels start from x = 0;
 *   - eps^2 = tol^2 |b|^2 / N_0 with b the full right-hand side;
 *   - the coarsest level is solved by a dense Cholesky factorisation;
 *   - initial guess on the finest level: the linear ramp between the two
 *     x-face Dirichlet values when only those faces are Dirichlet, else 0.
 *
 * Plain loops, no blocking, no fusion, no reordering beyond what the
 * definitions state.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAX_LEVELS 8

/* Boundary-condition codes per face: -x, +x, -y, +y, -z, +z. */
#define OR_NEUMANN 0
#define OR_DIRICHLET 1

typedef struct {
  int nx, ny, nz, n;
  double hx, hy, hz;
  double *tx; /* (nx+1)*ny*nz, face i between cells i-1 and i */
  double *ty; /* nx*(ny+1)*nz */
  double *tz; /* nx*ny*(nz+1) */
  int sx, sy, sz; /* factor to the next coarser level */
  double *chol;   /* coarsest level only: lower Cholesky factor, n*n row-major */
  /* work vectors for this level's PCG and preconditioner */
  double *x, *r, *z, *p, *q, *s, *t;
} or_level;

typedef struct {
  int dim, nlev;
  or_level lev[OR_MAX_LEVELS];
  int m;            /* smoothing steps (pre and post) */
  double flvl;      /* level factor f of the per-level criterion */
  int max_outer, max_inner;
  double eps2;      /* eps^2 of the finest level */
  long long iters[OR_MAX_LEVELS], calls[OR_MAX_LEVELS];
  int status;
} or_problem;

typedef struct {
  int status;       /* 0 ok, 1 not converged, -4 breakdown, -1 bad argument */
  int outer_iters, nlev;
  int level_n[OR_MAX_LEVELS][3];
  long long level_iters[OR_MAX_LEVELS], level_calls[OR_MAX_LEVELS];
  double rel_residual_true, b_norm;
} or_stats;

/* ------------------------------------------------------------------------ */
/* Level plan (reading of Section 3: scale factor about 4 between levels).  */
/* ------------------------------------------------------------------------ */

/* Fills dims[l][3] for l = 0..nlev-1 and returns nlev.  Every coarsened axis
 * (x, y; plus z in 3-D) is divided by `scale` while all of them stay divisible
 * and the quotient is >= min_side; at most max_levels levels. */
int oracle_level_plan(int dim, const int n[3], int scale, int min_side, int max_levels, int dims[][3]) {
  int d[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  int nl = 0;
  if (max_levels > OR_MAX_LEVELS) max_levels = OR_MAX_LEVELS;
  for (;;) {
    dims[nl][0] = d[0]; dims[nl][1] = d[1]; dims[nl][2] = d[2];
    nl++;
    if (nl >= max_levels) break;
    int ok = 1;
    for (int a = 0; a < dim; ++a)
      if (d[a] % scale != 0 || d[a] / scale < min_side) ok = 0;
    if (!ok) break;
    for (int a = 0; a < dim; ++a) d[a] /= scale;
  }
  return nl;
}

/* Plan with a factor that need not be an integer (Section 3: the scale
 * factor between grids is not limited to an integer; the effective factor
 * varies slightly so that every level has an integer dimension).  Each
 * coarsened axis goes from d to round(d / scale) cells while every result is
 * >= min_side and smaller than d.  g_frac_scale > 0 selects it for the
 * solver entry points (set by oracle_set_frac_scale; 0 restores the integer
 * plans). */
static double g_frac_scale = 0.0;
void oracle_set_frac_scale(double scale) { g_frac_scale = scale > 0.0 ? scale : 0.0; }

int oracle_level_plan_frac(int dim, const int n[3], double scale, int min_side, int max_levels, int dims[][3]) {
  int d[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  int nl = 0;
  if (max_levels > OR_MAX_LEVELS) max_levels = OR_MAX_LEVELS;
  for (;;) {
    dims[nl][0] = d[0]; dims[nl][1] = d[1]; dims[nl][2] = d[2];
    nl++;
    if (nl >= max_levels) break;
    int c[3] = {d[0], d[1], d[2]}, ok = 1;
    for (int a = 0; a < dim; ++a) {
      c[a] = (int)floor(d[a] / scale + 0.5);
      if (c[a] < min_side || c[a] >= d[a]) ok = 0;
    }
    if (!ok) break;
    for (int a = 0; a < dim; ++a) d[a] = c[a];
  }
  return nl;
}

/* Aspect-ratio-aware plan (Section 5, anisotropic strip: coarsening aims at
 * cells of aspect ratio 1, so the finer direction is coarsened first, then
 * both).  The effective size of a cell along axis a is h_a / sqrt(w_a), with
 * w_a the caller's permeability scale of that axis (e.g. kz / kx).  Per level,
 * among the axes that can be coarsened by `scale` (exact division, coarse side
 * >= min_side), those whose effective size is within a factor sqrt(scale) of
 * the smallest are coarsened; the plan stops when no axis can be. */
int oracle_level_plan_semi(int dim, const int n[3], const double Ldom[3], const double w[3], int scale, int min_side,
                           int max_levels, int dims[][3]) {
  int d[3] = {n[0], n[1], dim == 3 ? n[2] : 1};
  int nl = 0;
  if (max_levels > OR_MAX_LEVELS) max_levels = OR_MAX_LEVELS;
  for (;;) {
    dims[nl][0] = d[0]; dims[nl][1] = d[1]; dims[nl][2] = d[2];
    nl++;
    if (nl >= max_levels) break;
    int can[3] = {0, 0, 0}, any = 0;
    double e[3] = {0.0, 0.0, 0.0}, emin = 0.0;
    for (int a = 0; a < dim; ++a) {
      can[a] = d[a] % scale == 0 && d[a] / scale >= min_side;
      e[a] = (Ldom[a] / d[a]) / sqrt(w[a]);
      if (can[a] && (!any || e[a] < emin)) emin = e[a];
      any |= can[a];
    }
    if (!any) break;
    for (int a = 0; a < dim; ++a)
      if (can[a] && e[a] <= emin * sqrt((double)scale) * (1.0 + 1e-12)) d[a] /= scale;
  }
  return nl;
}

/* ------------------------------------------------------------------------ */
/* a1: face transmissibilities (Section 3: harmonic mean of the two cells,   */
/* T_xx = (dy/dx) K_xx, T_yy = (dx/dy) K_yy; boundary type changes the       */
/* boundary K).                                                              */
/* ------------------------------------------------------------------------ */

static double harmonic(double a, double b) { return 2.0 * a * b / (a + b); }

/* kx, ky, kz: cell-centred, n cells each (kz ignored in 2-D).  bc_type per
 * face -x,+x,-y,+y,-z,+z.  Interior face: (area/dist) * 2 kL kR / (kL + kR);
 * Dirichlet boundary face: 2 (area/dist) k_cell; Neumann: 0.
 * In 2-D the cell has unit thickness (hz = 1) and no z faces are used. */
void oracle_face_T(int dim, int nx, int ny, int nz, double hx, double hy, double hz, const double *kx,
                   const double *ky, const double *kz, const int bc_type[6], double *tx, double *ty, double *tz) {
  if (dim == 2) { nz = 1; hz = 1.0; }
  double ax = hy * hz / hx, ay = hx * hz / hy, az = hx * hy / hz;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        double t;
        if (i == 0) t = bc_type[0] == OR_DIRICHLET ? 2.0 * ax * kx[(size_t)nx * (j + (size_t)ny * k)] : 0.0;
        else if (i == nx) t = bc_type[1] == OR_DIRICHLET ? 2.0 * ax * kx[(nx - 1) + (size_t)nx * (j + (size_t)ny * k)] : 0.0;
        else {
          size_t c = i + (size_t)nx * (j + (size_t)ny * k);
          t = ax * harmonic(kx[c - 1], kx[c]);
        }
        tx[i + (size_t)(nx + 1) * (j + (size_t)ny * k)] = t;
      }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double t;
        if (j == 0) t = bc_type[2] == OR_DIRICHLET ? 2.0 * ay * ky[i + (size_t)nx * ny * k] : 0.0;
        else if (j == ny) t = bc_type[3] == OR_DIRICHLET ? 2.0 * ay * ky[i + (size_t)nx * ((ny - 1) + (size_t)ny * k)] : 0.0;
        else {
          size_t c = i + (size_t)nx * (j + (size_t)ny * k);
          t = ay * harmonic(ky[c - nx], ky[c]);
        }
        ty[i + (size_t)nx * (j + (size_t)(ny + 1) * k)] = t;
      }
  if (dim == 3) {
    size_t plane = (size_t)nx * ny;
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double t;
          if (k == 0) t = bc_type[4] == OR_DIRICHLET ? 2.0 * az * kz[i + (size_t)nx * j] : 0.0;
          else if (k == nz) t = bc_type[5] == OR_DIRICHLET ? 2.0 * az * kz[i + (size_t)nx * j + plane * (nz - 1)] : 0.0;
          else {
            size_t c = i + (size_t)nx * j + plane * k;
            t = az * harmonic(kz[c - plane], kz[c]);
          }
          tz[i + (size_t)nx * j + plane * k] = t;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* a2: coarse graining of transmissivities (Section 3):                      */
/*   1 / T^c = sum_i [ alpha_i / sum_j T(i, j) ]                             */
/* over the fine faces i whose control volume overlaps the coarse face's     */
/* control volume (the span between adjacent cell centres, a half cell at    */
/* the boundary), alpha_i = overlapping fraction of the fine span; j runs    */
/* over the fine faces inside the coarse face.  A fine column whose parallel */
/* sum is zero (no flow) makes the coarse face zero.                         */
/* ------------------------------------------------------------------------ */

/* Overlap, in units of the fine spacing, of fine face i's span with coarse
 * face I's span, divided by the fine span's width (the fraction of the width
 * in the overlap).  nf, nc = fine and coarse cells along the axis; the factor
 * f = nf / nc need not be an integer (Section 3). */
static double face_overlap(int i, int I, int nf, int nc) {
  double f = (double)nf / nc;
  double a0 = i - 0.5, a1 = i + 0.5;
  if (i == 0) a0 = 0.0;
  if (i == nf) a1 = nf;
  double b0 = f * I - 0.5 * f, b1 = f * I + 0.5 * f;
  if (I == 0) b0 = 0.0;
  if (I == nc) b1 = nf;
  double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  if (hi <= lo) return 0.0;
  return (hi - lo) / (a1 - a0);
}

/* Fraction of fine cell j (span [j, j+1]) inside coarse cell J (span
 * [J f, (J+1) f], f = nf / nc): the fraction of the height in the overlap. */
static double cell_overlap(int j, int J, int nf, int nc) {
  double f = (double)nf / nc;
  double b0 = f * J, b1 = J + 1 == nc ? (double)nf : f * (J + 1);
  double lo = j > b0 ? j : b0, hi = j + 1 < b1 ? j + 1 : b1;
  return hi > lo ? hi - lo : 0.0;
}

/* Generic coarsening of one face array along `axis` (0, 1, 2).  Fine face
 * array f has dims (fnx + (axis==0), fny + (axis==1), fnz + (axis==2)); the
 * coarse one c likewise with the coarse cell counts cd.  A fine face that
 * only partly overlaps the coarse face is weighted by the fraction of the
 * height in the overlap (parallel sum) and inversely by the fraction of the
 * width (series sum), Section 3. */
static void coarsen_axis(int axis, const int fd[3], const int cd[3], const double *f, double *c) {
  int fe[3] = {fd[0], fd[1], fd[2]}, ce[3] = {cd[0], cd[1], cd[2]};
  fe[axis] += 1; ce[axis] += 1;
  int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
  int C[3];
  for (C[2] = 0; C[2] < ce[2]; ++C[2])
    for (C[1] = 0; C[1] < ce[1]; ++C[1])
      for (C[0] = 0; C[0] < ce[0]; ++C[0]) {
        int I = C[axis];
        double inv = 0.0;
        int blocked = 0;
        /* fine faces along the axis that can overlap coarse face I */
        double fa = (double)fd[axis] / cd[axis];
        int ilo = (int)floor(fa * (I - 1)), ihi = (int)ceil(fa * (I + 1));
        if (ilo < 0) ilo = 0;
        if (ihi > fd[axis]) ihi = fd[axis];
        /* fine cells across the face that overlap the coarse cell */
        double f1 = (double)fd[a1] / cd[a1], f2 = (double)fd[a2] / cd[a2];
        int ulo = (int)floor(f1 * C[a1]), uhi = (int)ceil(f1 * (C[a1] + 1));
        int vlo = (int)floor(f2 * C[a2]), vhi = (int)ceil(f2 * (C[a2] + 1));
        if (uhi > fd[a1]) uhi = fd[a1];
        if (vhi > fd[a2]) vhi = fd[a2];
        for (int i = ilo; i <= ihi; ++i) {
          double alpha = face_overlap(i, I, fd[axis], cd[axis]);
          if (alpha == 0.0) continue;
          double par = 0.0; /* parallel sum over the fine faces inside the coarse face */
          for (int u = ulo; u < uhi; ++u) {
            double bu = cell_overlap(u, C[a1], fd[a1], cd[a1]);
            if (bu == 0.0) continue;
            for (int v = vlo; v < vhi; ++v) {
              double bv = cell_overlap(v, C[a2], fd[a2], cd[a2]);
              if (bv == 0.0) continue;
              int F[3];
              F[axis] = i;
              F[a1] = u;
              F[a2] = v;
              par += bu * bv * f[F[0] + (size_t)fe[0] * (F[1] + (size_t)fe[1] * F[2])];
            }
          }
          if (par == 0.0) { blocked = 1; break; }
          inv += alpha / par;
        }
        c[C[0] + (size_t)ce[0] * (C[1] + (size_t)ce[1] * C[2])] = blocked ? 0.0 : 1.0 / inv;
      }
}

/* cd: coarse cell counts (fd / integer factors, or any coarser counts) */
static void coarsen_T_dims(int dim, const int fd[3], const int cd[3], const double *tx, const double *ty,
                           const double *tz, double *ctx, double *cty, double *ctz) {
  int f3[3] = {fd[0], fd[1], dim == 3 ? fd[2] : 1};
  int c3[3] = {cd[0], cd[1], dim == 3 ? cd[2] : 1};
  coarsen_axis(0, f3, c3, tx, ctx);
  coarsen_axis(1, f3, c3, ty, cty);
  if (dim == 3) coarsen_axis(2, f3, c3, tz, ctz);
}

void oracle_coarsen_T(int dim, const int fd[3], const int s[3], const double *tx, const double *ty,
                      const double *tz, double *ctx, double *cty, double *ctz) {
  int cd[3] = {fd[0] / s[0], fd[1] / s[1], dim == 3 ? fd[2] / s[2] : 1};
  coarsen_T_dims(dim, fd, cd, tx, ty, tz, ctx, cty, ctz);
}

/* ------------------------------------------------------------------------ */
/* a5: the operator (Section 3, 5-point / 7-point support-operator form):    */
/*   (A x)_c = sum over faces of c of T_f (x_c - x_nb),                      */
/* with x_nb = 0 across a boundary face (its value is moved to the rhs).     */
/* ------------------------------------------------------------------------ */

static double cell_diag(const or_level *L, int i, int j, int k) {
  int nx = L->nx, ny = L->ny;
  double d = L->tx[i + (size_t)(nx + 1) * (j + (size_t)ny * k)] + L->tx[i + 1 + (size_t)(nx + 1) * (j + (size_t)ny * k)] +
             L->ty[i + (size_t)nx * (j + (size_t)(ny + 1) * k)] + L->ty[i + (size_t)nx * (j + 1 + (size_t)(ny + 1) * k)];
  if (L->tz) d += L->tz[i + (size_t)nx * j + (size_t)nx * ny * k] + L->tz[i + (size_t)nx * j + (size_t)nx * ny * (k + 1)];
  return d;
}

/* sum over neighbours of T_f x_nb */
static double cell_offsum(const or_level *L, const double *x, int i, int j, int k) {
  int nx = L->nx, ny = L->ny, nz = L->nz;
  size_t c = i + (size_t)nx * (j + (size_t)ny * k), plane = (size_t)nx * ny;
  double s = 0.0;
  if (i > 0) s += L->tx[i + (size_t)(nx + 1) * (j + (size_t)ny * k)] * x[c - 1];
  if (i < nx - 1) s += L->tx[i + 1 + (size_t)(nx + 1) * (j + (size_t)ny * k)] * x[c + 1];
  if (j > 0) s += L->ty[i + (size_t)nx * (j + (size_t)(ny + 1) * k)] * x[c - nx];
  if (j < ny - 1) s += L->ty[i + (size_t)nx * (j + 1 + (size_t)(ny + 1) * k)] * x[c + nx];
  if (L->tz) {
    if (k > 0) s += L->tz[i + (size_t)nx * j + plane * k] * x[c - plane];
    if (k < nz - 1) s += L->tz[i + (size_t)nx * j + plane * (k + 1)] * x[c + plane];
  }
  return s;
}

static void apply_A(const or_level *L, const double *x, double *y) {
  for (int k = 0; k < L->nz; ++k)
    for (int j = 0; j < L->ny; ++j)
      for (int i = 0; i < L->nx; ++i) {
        size_t c = i + (size_t)L->nx * (j + (size_t)L->ny * k);
        y[c] = cell_diag(L, i, j, k) * x[c] - cell_offsum(L, x, i, j, k);
      }
}

/* ------------------------------------------------------------------------ */
/* Smoother: symmetric Gauss-Seidel splitting A = P - Q with                 */
/* P = (D+L) D^-1 (D+U), Q = L D^-1 U (Section 3, eq. 2.3), in red-black    */
/* ordering.  One step x <- x + P^-1 (r - A x) is a forward Gauss-Seidel     */
/* sweep (red, then black) followed by a backward sweep (black, then red).   */
/* A Gauss-Seidel update of a cell is x_c = (r_c + sum T_f x_nb) / D_c.      */
/* ------------------------------------------------------------------------ */

static void gs_colour(const or_level *L, const double *r, double *x, int colour) {
  for (int k = 0; k < L->nz; ++k)
    for (int j = 0; j < L->ny; ++j)
      for (int i = 0; i < L->nx; ++i) {
        if (((i + j + k) & 1) != colour) continue;
        size_t c = i + (size_t)L->nx * (j + (size_t)L->ny * k);
        x[c] = (r[c] + cell_offsum(L, x, i, j, k)) / cell_diag(L, i, j, k);
      }
}

static void sgs_steps(const or_level *L, const double *r, double *x, int m) {
  for (int step = 0; step < m; ++step) {
    gs_colour(L, r, x, 0); /* forward: red */
    gs_colour(L, r, x, 1); /*          black */
    gs_colour(L, r, x, 1); /* backward: black */
    gs_colour(L, r, x, 0); /*           red */
  }
}

/* The modified Jacobi splitting (Section 3): P = 2D, Q = D - U - L.  One step
 * is x <- x + P^-1 (r - A x) = x + (r - A x) / (2 d) for every cell at once. */
static void mjac_steps(const or_level *L, const double *r, double *x, int m) {
  const size_t n = (size_t)L->nx * L->ny * L->nz;
  double *ax = malloc(sizeof(double) * n);
  for (int step = 0; step < m; ++step) {
    apply_A(L, x, ax);
    for (int k = 0; k < L->nz; ++k)
      for (int j = 0; j < L->ny; ++j)
        for (int i = 0; i < L->nx; ++i) {
          size_t c = i + (size_t)L->nx * (j + (size_t)L->ny * k);
          ax[c] = x[c] + (r[c] - ax[c]) / (2.0 * cell_diag(L, i, j, k));
        }
    memcpy(x, ax, sizeof(double) * n);
  }
  free(ax);
}

/* m steps of the chosen splitting: 0 symmetric Gauss-Seidel, 1 modified Jacobi */
static int g_split = 0;
static void smooth(const or_level *L, const double *r, double *x, int m) {
  if (g_split == 1) mjac_steps(L, r, x, m);
  else sgs_steps(L, r, x, m);
}

/* ------------------------------------------------------------------------ */
/* Grid transfers (Section 3): E = tensor product of 1-D linear              */
/* interpolation between cell centres with zero slope at the boundary;       */
/* R = E^T.                                                                  */
/* ------------------------------------------------------------------------ */

/* 1-D weights: fine cell i (of nf) takes coarse cells I0, I1 (of nc) with
 * weights w0, w1; f = nf / nc need not be an integer.  Linear (interp = 0):
 * coarse coordinate xi = (i + 1/2)/f - 1/2, clamped to [0, nc-1] (zero slope
 * at the boundary).  Piecewise constant (interp = 1, the alternative the
 * paper reports to work nearly as well): the coarse cell containing the fine
 * cell's centre. */
static int g_interp = 0;
static void interp1(int i, int nf, int nc, int *I0, double *w0, int *I1, double *w1) {
  if (nf == nc) { *I0 = i; *w0 = 1.0; *I1 = i; *w1 = 0.0; return; }
  double f = (double)nf / nc;
  if (g_interp == 1) {
    int I = (int)floor((i + 0.5) / f);
    if (I > nc - 1) I = nc - 1;
    *I0 = I; *w0 = 1.0; *I1 = I; *w1 = 0.0;
    return;
  }
  double xi = (i + 0.5) / f - 0.5;
  if (xi <= 0.0) { *I0 = 0; *w0 = 1.0; *I1 = 0; *w1 = 0.0; return; }
  if (xi >= nc - 1) { *I0 = nc - 1; *w0 = 1.0; *I1 = nc - 1; *w1 = 0.0; return; }
  int b = (int)floor(xi);
  double t = xi - b;
  *I0 = b; *w0 = 1.0 - t; *I1 = b + 1; *w1 = t;
}

/* y_fine += E y_coarse */
static void prolong_add(const or_level *F, const or_level *C, const double *yc, double *xf) {
  for (int k = 0; k < F->nz; ++k) {
    int K[2]; double wk[2];
    interp1(k, F->nz, C->nz, &K[0], &wk[0], &K[1], &wk[1]);
    for (int j = 0; j < F->ny; ++j) {
      int J[2]; double wj[2];
      interp1(j, F->ny, C->ny, &J[0], &wj[0], &J[1], &wj[1]);
      for (int i = 0; i < F->nx; ++i) {
        int I[2]; double wi[2];
        interp1(i, F->nx, C->nx, &I[0], &wi[0], &I[1], &wi[1]);
        double v = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
              v += wk[a] * wj[b] * wi[c] * yc[I[c] + (size_t)C->nx * (J[b] + (size_t)C->ny * K[a])];
        xf[i + (size_t)F->nx * (j + (size_t)F->ny * k)] += v;
      }
    }
  }
}

/* g_coarse = E^T r_fine */
static void restrict_T(const or_level *F, const or_level *C, const double *rf, double *gc) {
  memset(gc, 0, sizeof(double) * C->n);
  for (int k = 0; k < F->nz; ++k) {
    int K[2]; double wk[2];
    interp1(k, F->nz, C->nz, &K[0], &wk[0], &K[1], &wk[1]);
    for (int j = 0; j < F->ny; ++j) {
      int J[2]; double wj[2];
      interp1(j, F->ny, C->ny, &J[0], &wj[0], &J[1], &wj[1]);
      for (int i = 0; i < F->nx; ++i) {
        int I[2]; double wi[2];
        interp1(i, F->nx, C->nx, &I[0], &wi[0], &I[1], &wi[1]);
        double v = rf[i + (size_t)F->nx * (j + (size_t)F->ny * k)];
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
              gc[I[c] + (size_t)C->nx * (J[b] + (size_t)C->ny * K[a])] += wk[a] * wj[b] * wi[c] * v;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Coarsest level: "solved exactly" (Section 2.2/2.3).  Dense assembly of    */
/* the level's operator and a textbook Cholesky factorisation.               */
/* ------------------------------------------------------------------------ */

static void dense_A(const or_level *L, double *A) {
  double *e = calloc(L->n, sizeof(double)), *col = malloc(sizeof(double) * L->n);
  for (int c = 0; c < L->n; ++c) {
    e[c] = 1.0;
    apply_A(L, e, col);
    for (int i = 0; i < L->n; ++i) A[(size_t)i * L->n + c] = col[i];
    e[c] = 0.0;
  }
  free(e); free(col);
}

/* returns 0 on success, -6 if not positive definite */
int oracle_cholesky(int n, const double *A, double *Lf) {
  memset(Lf, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= Lf[(size_t)j * n + k] * Lf[(size_t)j * n + k];
    if (!(d > 0.0)) return -6;
    d = sqrt(d);
    Lf[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= Lf[(size_t)i * n + k] * Lf[(size_t)j * n + k];
      Lf[(size_t)i * n + j] = s / d;
    }
  }
  return 0;
}

void oracle_cholesky_solve(int n, const double *Lf, const double *b, double *x) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= Lf[(size_t)i * n + k] * x[k];
    x[i] = s / Lf[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int k = i + 1; k < n; ++k) s -= Lf[(size_t)k * n + i] * x[k];
    x[i] = s / Lf[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------------------ */
/* Recursive multi-scale PCG (Section 2.3, eq. 2.10; Section 3).             */
/* ------------------------------------------------------------------------ */

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

static int pcg_level(or_problem *P, int k, const double *b, double *x, int x_is_zero, int max_iter);

/* Coarse part of the preconditioner: 0 the recursive multi-scale form
 * (eq. 2.10, A_c^-1 by an inner PCG), 1 Tatebe's multigrid form (eq. 2.9,
 * M_{k+1}^-1 applied once); both end with the exact coarsest solve.  2 the
 * polynomial preconditioner (Section 2.1, W = P^-1), which has no coarse part. */
static int g_cycle = 0;

/* z = M_k^-1 r, eq. 2.10 evaluated as m smoothing steps from zero, a coarse
 * correction E A_c^-1 R of the remaining residual, and m smoothing steps
 * (eq. 2.9 when g_cycle is 1). */
static void precond(or_problem *P, int k, const double *r, double *z) {
  or_level *L = &P->lev[k], *C = &P->lev[k + 1];
  memset(z, 0, sizeof(double) * L->n);
  if (g_cycle == 2) {
    /* polynomial preconditioner (Section 2.1): W = P^-1 in eq. 2.6 makes M^-1
     * the first 2m+1 terms of the series of eq. 2.4, i.e. 2m+1 steps of the
     * splitting from zero; no coarse level is used */
    smooth(L, r, z, 2 * P->m + 1);
    return;
  }
  smooth(L, r, z, P->m);
  apply_A(L, z, L->s);
  for (int i = 0; i < L->n; ++i) L->s[i] = r[i] - L->s[i];
  restrict_T(L, C, L->s, C->t); /* coarse right-hand side */
  if (k + 1 == P->nlev - 1) {
    oracle_cholesky_solve(C->n, C->chol, C->t, C->x);
    P->calls[k + 1]++;
  } else if (g_cycle == 1) {
    /* Tatebe's multigrid preconditioner (eq. 2.9): W_k = E M_{k+1}^-1 R, one
     * application of the next level's preconditioner instead of a PCG solve */
    precond(P, k + 1, C->t, C->x);
    P->calls[k + 1]++;
  } else {
    memset(C->x, 0, sizeof(double) * C->n);
    pcg_level(P, k + 1, C->t, C->x, 1, P->max_inner);
  }
  prolong_add(L, C, C->x, z);
  smooth(L, r, z, P->m);
}

/* Conjugate gradient with preconditioner as in the Templates book, Section
 * 2.3.1, Figure 2.5; stop when |r|^2 / N_k < f^k eps^2 (Section 3).
 * Returns the number of iterations. */
static int pcg_level(or_problem *P, int k, const double *b, double *x, int x_is_zero, int max_iter) {
  or_level *L = &P->lev[k];
  int n = L->n;
  double tolk = P->eps2;
  for (int i = 0; i < k; ++i) tolk *= P->flvl;
  double *r = L->r, *z = L->z, *p = L->p, *q = L->q;
  P->calls[k]++;
  if (x_is_zero) memcpy(r, b, sizeof(double) * n);
  else {
    apply_A(L, x, q);
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
  }
  double rr = dot(n, r, r);
  if (rr / n < tolk) return 0;
  double rho_old = 0.0;
  int it;
  for (it = 1; it <= max_iter; ++it) {
    precond(P, k, r, z);
    double rho = dot(n, r, z);
    /* r.z <= 0 (or p.Ap <= 0): no further progress in finite precision.  An
     * inner level stops there (its solve is approximate by design); on the
     * finest level, or with a non-finite value, it is a breakdown. */
    if (!(rho > 0.0)) { if (k == 0 || rho != rho) P->status = -4; break; }
    if (it == 1) memcpy(p, z, sizeof(double) * n);
    else {
      double beta = rho / rho_old;
      for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    apply_A(L, p, q);
    double pq = dot(n, p, q);
    if (!(pq > 0.0)) { if (k == 0 || pq != pq) P->status = -4; break; }
    double alpha = rho / pq;
    for (int i = 0; i < n; ++i) x[i] += alpha * p[i];
    for (int i = 0; i < n; ++i) r[i] -= alpha * q[i];
    P->iters[k]++;
    rr = dot(n, r, r);
    if (rr / n < tolk) break;
    rho_old = rho;
  }
  if (it > max_iter) it = max_iter;
  return it;
}

/* ------------------------------------------------------------------------ */
/* Driver.                                                                   */
/* ------------------------------------------------------------------------ */

static void free_problem(or_problem *P) {
  for (int l = 0; l < P->nlev; ++l) {
    or_level *L = &P->lev[l];
    free(L->tx); free(L->ty); free(L->tz); free(L->chol);
    free(L->x); free(L->r); free(L->z); free(L->p); free(L->q); free(L->s); free(L->t);
  }
}

/* Builds the hierarchy: face T on level 0, coarse-grained T below, Cholesky
 * factor on the coarsest level.  Returns 0, or -1 / -6 on error. */
static int build_problem(or_problem *P, int dim, const int n[3], const double Ldom[3], const double *kx,
                         const double *ky, const double *kz, const int bc_type[6], int scale, int min_side,
                         int max_levels, int max_coarse, int factor, const double *axis_w) {
  int dims[OR_MAX_LEVELS][3];
  memset(P, 0, sizeof(*P));
  P->dim = dim;
  if (g_frac_scale > 0.0)
    P->nlev = oracle_level_plan_frac(dim, n, g_frac_scale, min_side, max_levels, dims);
  else
    P->nlev = axis_w ? oracle_level_plan_semi(dim, n, Ldom, axis_w, scale, min_side, max_levels, dims)
                     : oracle_level_plan(dim, n, scale, min_side, max_levels, dims);
  for (int l = 0; l < P->nlev; ++l) {
    or_level *L = &P->lev[l];
    L->nx = dims[l][0]; L->ny = dims[l][1]; L->nz = dims[l][2];
    L->n = L->nx * L->ny * L->nz;
    L->hx = Ldom[0] / L->nx; L->hy = Ldom[1] / L->ny; L->hz = dim == 3 ? Ldom[2] / L->nz : 1.0;
    L->tx = malloc(sizeof(double) * (size_t)(L->nx + 1) * L->ny * L->nz);
    L->ty = malloc(sizeof(double) * (size_t)L->nx * (L->ny + 1) * L->nz);
    L->tz = dim == 3 ? malloc(sizeof(double) * (size_t)L->nx * L->ny * (L->nz + 1)) : NULL;
    size_t nn = (size_t)L->n;
    L->x = calloc(nn, 8); L->r = calloc(nn, 8); L->z = calloc(nn, 8); L->p = calloc(nn, 8);
    L->q = calloc(nn, 8); L->s = calloc(nn, 8); L->t = calloc(nn, 8);
    if (l + 1 < P->nlev) {
      L->sx = dims[l][0] / dims[l + 1][0]; L->sy = dims[l][1] / dims[l + 1][1]; L->sz = dims[l][2] / dims[l + 1][2];
    } else { L->sx = L->sy = L->sz = 1; }
  }
  or_level *L0 = &P->lev[0];
  oracle_face_T(dim, L0->nx, L0->ny, L0->nz, L0->hx, L0->hy, L0->hz, kx, ky, kz, bc_type, L0->tx, L0->ty, L0->tz);
  for (int l = 1; l < P->nlev; ++l) {
    or_level *F = &P->lev[l - 1], *C = &P->lev[l];
    int fd[3] = {F->nx, F->ny, F->nz}, cd[3] = {C->nx, C->ny, C->nz};
    coarsen_T_dims(dim, fd, cd, F->tx, F->ty, F->tz, C->tx, C->ty, C->tz);
  }
  or_level *LL = &P->lev[P->nlev - 1];
  if (!factor) return 0;
  if (LL->n > max_coarse) return -1;
  double *A = malloc(sizeof(double) * (size_t)LL->n * LL->n);
  LL->chol = malloc(sizeof(double) * (size_t)LL->n * LL->n);
  dense_A(LL, A);
  int rc = oracle_cholesky(LL->n, A, LL->chol);
  free(A);
  return rc;
}

/* Full solve of -div(K grad p) = f (Section 3 with the sign flipped so the
 * matrix is SPD).  Inputs on the host: cell-centred kx, ky, kz (kz only in
 * 3-D), source f; per-face BC type and value.  rhs b_c = f_c |V_c| plus, on
 * each Dirichlet boundary face, T_b p_D.  Output p (n cells).
 * iopt: scale, min_side, m, max_outer, max_inner, max_levels, interp (0 linear,
 * 1 piecewise constant), splitting (0 symmetric Gauss-Seidel, 1 modified Jacobi),
 * cycle (0 recursive multi-scale PCG, eq. 2.10; 1 Tatebe's multigrid
 * preconditioner, eq. 2.9; 2 polynomial preconditioner, Section 2.1);
 * non-positive entries take the defaults 4, 8,
 * scale, 200, 200, 8, 0, 0, 0.
 * flvl_opt: f (default 0.1).  axis_w: NULL for the uniform level plan, else
 * the per-axis weights of the aspect-ratio-aware plan. */
int oracle_solve(int dim, const int n[3], const double Ldom_in[3], const double *kx, const double *ky,
                 const double *kz, const double *f, const int bc_type[6], const double bc_value[6], double tol,
                 const int iopt[9], const double *flvl_opt, double *p_out, or_stats *st, const double *axis_w) {
  int scale = iopt && iopt[0] > 0 ? iopt[0] : 4;
  int min_side = iopt && iopt[1] > 0 ? iopt[1] : 8;
  int m = iopt && iopt[2] > 0 ? iopt[2] : scale;
  int max_outer = iopt && iopt[3] > 0 ? iopt[3] : 200;
  int max_inner = iopt && iopt[4] > 0 ? iopt[4] : 200;
  int max_levels = iopt && iopt[5] > 0 ? iopt[5] : OR_MAX_LEVELS;
  g_interp = iopt && iopt[6] == 1 ? 1 : 0;
  g_split = iopt && iopt[7] == 1 ? 1 : 0;
  g_cycle = iopt && (iopt[8] == 1 || iopt[8] == 2) ? iopt[8] : 0;
  double flvl = flvl_opt && *flvl_opt > 0.0 ? *flvl_opt : 0.1;
  double Ldom[3] = {1.0, 1.0, 1.0};
  if (Ldom_in) for (int a = 0; a < 3; ++a) if (Ldom_in[a] > 0.0) Ldom[a] = Ldom_in[a];
  memset(st, 0, sizeof(*st));
  or_problem P;
  int rc = build_problem(&P, dim, n, Ldom, kx, ky, kz, bc_type, scale, min_side, max_levels, 1024, 1, axis_w);
  if (rc != 0) { free_problem(&P); st->status = rc; return rc; }
  P.m = m; P.flvl = flvl; P.max_outer = max_outer; P.max_inner = max_inner;
  or_level *L0 = &P.lev[0];
  int nx = L0->nx, ny = L0->ny, nz = L0->nz, N = L0->n;
  double vol = L0->hx * L0->hy * L0->hz;
  /* right-hand side */
  double *b = malloc(sizeof(double) * N);
  for (int c = 0; c < N; ++c) b[c] = f[c] * vol;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j) {
      size_t row = (size_t)nx * (j + (size_t)ny * k);
      if (bc_type[0] == OR_DIRICHLET) b[row] += L0->tx[(size_t)(nx + 1) * (j + (size_t)ny * k)] * bc_value[0];
      if (bc_type[1] == OR_DIRICHLET) b[row + nx - 1] += L0->tx[nx + (size_t)(nx + 1) * (j + (size_t)ny * k)] * bc_value[1];
    }
  for (int k = 0; k < nz; ++k)
    for (int i = 0; i < nx; ++i) {
      if (bc_type[2] == OR_DIRICHLET) b[i + (size_t)nx * ny * k] += L0->ty[i + (size_t)nx * (ny + 1) * k] * bc_value[2];
      if (bc_type[3] == OR_DIRICHLET)
        b[i + (size_t)nx * ((ny - 1) + (size_t)ny * k)] += L0->ty[i + (size_t)nx * (ny + (size_t)(ny + 1) * k)] * bc_value[3];
    }
  if (dim == 3) {
    size_t plane = (size_t)nx * ny;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        if (bc_type[4] == OR_DIRICHLET) b[i + (size_t)nx * j] += L0->tz[i + (size_t)nx * j] * bc_value[4];
        if (bc_type[5] == OR_DIRICHLET)
          b[i + (size_t)nx * j + plane * (nz - 1)] += L0->tz[i + (size_t)nx * j + plane * nz] * bc_value[5];
      }
  }
  double bb = dot(N, b, b);
  P.eps2 = tol * tol * bb / N;
  /* initial guess: lifting by a smooth field that matches the boundary values */
  int only_x_dirichlet = bc_type[0] == OR_DIRICHLET && bc_type[1] == OR_DIRICHLET;
  for (int a = 2; a < 6; ++a) if (bc_type[a] == OR_DIRICHLET) only_x_dirichlet = 0;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double xc = (i + 0.5) * L0->hx;
        p_out[i + (size_t)nx * (j + (size_t)ny * k)] =
            only_x_dirichlet ? bc_value[0] + (bc_value[1] - bc_value[0]) * xc / Ldom[0] : 0.0;
      }
  int outer;
  if (P.nlev == 1) {
    /* the finest grid is itself small enough to solve directly */
    oracle_cholesky_solve(N, L0->chol, b, p_out);
    P.calls[0]++;
    outer = 0;
  } else {
    outer = pcg_level(&P, 0, b, p_out, 0, max_outer);
  }
  /* true residual */
  double *Ax = malloc(sizeof(double) * N);
  apply_A(L0, p_out, Ax);
  double rt = 0.0;
  for (int c = 0; c < N; ++c) rt += (b[c] - Ax[c]) * (b[c] - Ax[c]);
  st->status = P.status;
  if (st->status == 0 && P.nlev > 1 && dot(N, L0->r, L0->r) / N >= P.eps2) st->status = 1;
  st->outer_iters = outer;
  st->nlev = P.nlev;
  for (int l = 0; l < P.nlev; ++l) {
    st->level_n[l][0] = P.lev[l].nx; st->level_n[l][1] = P.lev[l].ny; st->level_n[l][2] = P.lev[l].nz;
    st->level_iters[l] = P.iters[l]; st->level_calls[l] = P.calls[l];
  }
  st->b_norm = sqrt(bb);
  st->rel_residual_true = bb > 0.0 ? sqrt(rt / bb) : sqrt(rt);
  free(b); free(Ax);
  free_problem(&P);
  return st->status;
}

/* ------------------------------------------------------------------------ */
/* Operator-level entry points used by the tests to pin each piece.          */
/* A level is described by its dims and face arrays; the coarse level of a   */
/* transfer by the factor s per axis.                                        */
/* ------------------------------------------------------------------------ */

static or_level make_view(int dim, int nx, int ny, int nz, const double *tx, const double *ty, const double *tz) {
  or_level L;
  memset(&L, 0, sizeof(L));
  L.nx = nx; L.ny = ny; L.nz = dim == 3 ? nz : 1; L.n = L.nx * L.ny * L.nz;
  L.tx = (double *)tx; L.ty = (double *)ty; L.tz = dim == 3 ? (double *)tz : NULL;
  return L;
}

void oracle_apply_A(int dim, int nx, int ny, int nz, const double *tx, const double *ty, const double *tz,
                    const double *x, double *y) {
  or_level L = make_view(dim, nx, ny, nz, tx, ty, tz);
  apply_A(&L, x, y);
}

/* m symmetric Gauss-Seidel steps x <- x + P^-1 (r - A x), in place */
void oracle_sgs(int dim, int nx, int ny, int nz, const double *tx, const double *ty, const double *tz,
                const double *r, double *x, int m) {
  or_level L = make_view(dim, nx, ny, nz, tx, ty, tz);
  sgs_steps(&L, r, x, m);
}

/* m modified Jacobi steps (P = 2D) from x, in place */
void oracle_mjac(int dim, int nx, int ny, int nz, const double *tx, const double *ty, const double *tz,
                 const double *r, double *x, int m) {
  or_level L = make_view(dim, nx, ny, nz, tx, ty, tz);
  mjac_steps(&L, r, x, m);
}

/* one Gauss-Seidel half sweep over one colour (0 red, 1 black), in place */
void oracle_gs_colour(int dim, int nx, int ny, int nz, const double *tx, const double *ty, const double *tz,
                      const double *r, double *x, int colour) {
  or_level L = make_view(dim, nx, ny, nz, tx, ty, tz);
  gs_colour(&L, r, x, colour);
}

void oracle_prolong_add(int dim, const int fd[3], const int s[3], int interp, const double *yc, double *xf) {
  or_level F, C;
  g_interp = interp == 1 ? 1 : 0;
  memset(&F, 0, sizeof(F)); memset(&C, 0, sizeof(C));
  F.nx = fd[0]; F.ny = fd[1]; F.nz = dim == 3 ? fd[2] : 1;
  F.sx = s[0]; F.sy = s[1]; F.sz = dim == 3 ? s[2] : 1;
  C.nx = F.nx / F.sx; C.ny = F.ny / F.sy; C.nz = F.nz / F.sz; C.n = C.nx * C.ny * C.nz;
  prolong_add(&F, &C, yc, xf);
}

void oracle_restrict(int dim, const int fd[3], const int s[3], int interp, const double *rf, double *gc) {
  or_level F, C;
  g_interp = interp == 1 ? 1 : 0;
  memset(&F, 0, sizeof(F)); memset(&C, 0, sizeof(C));
  F.nx = fd[0]; F.ny = fd[1]; F.nz = dim == 3 ? fd[2] : 1;
  F.sx = s[0]; F.sy = s[1]; F.sz = dim == 3 ? s[2] : 1;
  C.nx = F.nx / F.sx; C.ny = F.ny / F.sy; C.nz = F.nz / F.sz; C.n = C.nx * C.ny * C.nz;
  restrict_T(&F, &C, rf, gc);
}

/* The same transfers between a fine grid fd and any coarser grid cd (the
 * factors fd / cd need not be integers). */
void oracle_prolong_add_dims(int dim, const int fd[3], const int cd[3], int interp, const double *yc, double *xf) {
  or_level F, C;
  memset(&F, 0, sizeof(F)); memset(&C, 0, sizeof(C));
  F.nx = fd[0]; F.ny = fd[1]; F.nz = dim == 3 ? fd[2] : 1; F.n = F.nx * F.ny * F.nz;
  C.nx = cd[0]; C.ny = cd[1]; C.nz = dim == 3 ? cd[2] : 1; C.n = C.nx * C.ny * C.nz;
  g_interp = interp == 1 ? 1 : 0;
  prolong_add(&F, &C, yc, xf);
}

void oracle_restrict_dims(int dim, const int fd[3], const int cd[3], int interp, const double *rf, double *gc) {
  or_level F, C;
  memset(&F, 0, sizeof(F)); memset(&C, 0, sizeof(C));
  F.nx = fd[0]; F.ny = fd[1]; F.nz = dim == 3 ? fd[2] : 1; F.n = F.nx * F.ny * F.nz;
  C.nx = cd[0]; C.ny = cd[1]; C.nz = dim == 3 ? cd[2] : 1; C.n = C.nx * C.ny * C.nz;
  g_interp = interp == 1 ? 1 : 0;
  restrict_T(&F, &C, rf, gc);
}

/* Applies the level-0 preconditioner M_0^-1 of a full hierarchy to r.
 * eps2 sets the absolute criterion of the inner levels (eps2 = 0 with
 * max_inner large runs the inner PCGs to their iteration cap; a 2-level
 * hierarchy has an exact coarse solve regardless). */
int oracle_precond(int dim, const int n[3], const double Ldom_in[3], const double *kx, const double *ky,
                   const double *kz, const int bc_type[6], const int iopt[9], double flvl, double eps2,
                   const double *r, double *z, const double *axis_w) {
  int scale = iopt && iopt[0] > 0 ? iopt[0] : 4;
  int min_side = iopt && iopt[1] > 0 ? iopt[1] : 8;
  int m = iopt && iopt[2] > 0 ? iopt[2] : scale;
  int max_inner = iopt && iopt[4] > 0 ? iopt[4] : 200;
  int max_levels = iopt && iopt[5] > 0 ? iopt[5] : OR_MAX_LEVELS;
  g_interp = iopt && iopt[6] == 1 ? 1 : 0;
  g_split = iopt && iopt[7] == 1 ? 1 : 0;
  g_cycle = iopt && (iopt[8] == 1 || iopt[8] == 2) ? iopt[8] : 0;
  double Ldom[3] = {1.0, 1.0, 1.0};
  if (Ldom_in) for (int a = 0; a < 3; ++a) if (Ldom_in[a] > 0.0) Ldom[a] = Ldom_in[a];
  or_problem P;
  int rc = build_problem(&P, dim, n, Ldom, kx, ky, kz, bc_type, scale, min_side, max_levels, 4096, 1, axis_w);
  if (rc != 0 || P.nlev < 2) { free_problem(&P); return rc != 0 ? rc : -1; }
  P.m = m; P.flvl = flvl > 0 ? flvl : 0.1; P.max_inner = max_inner; P.eps2 = eps2;
  precond(&P, 0, r, z);
  free_problem(&P);
  return 0;
}

/* Face arrays of every level of the hierarchy, concatenated level by level
 * (tx, ty, tz per level).  Returns nlev, or a negative error. */
int oracle_hierarchy_T(int dim, const int n[3], const double Ldom_in[3], const double *kx, const double *ky,
                       const double *kz, const int bc_type[6], int scale, int min_side, int max_levels,
                       double *out, size_t out_len, const double *axis_w) {
  double Ldom[3] = {1.0, 1.0, 1.0};
  if (Ldom_in) for (int a = 0; a < 3; ++a) if (Ldom_in[a] > 0.0) Ldom[a] = Ldom_in[a];
  or_problem P;
  build_problem(&P, dim, n, Ldom, kx, ky, kz, bc_type, scale, min_side, max_levels, 0, 0, axis_w);
  size_t off = 0;
  for (int l = 0; l < P.nlev; ++l) {
    or_level *L = &P.lev[l];
    size_t a = (size_t)(L->nx + 1) * L->ny * L->nz, b = (size_t)L->nx * (L->ny + 1) * L->nz;
    size_t c = dim == 3 ? (size_t)L->nx * L->ny * (L->nz + 1) : 0;
    if (off + a + b + c > out_len) { free_problem(&P); return -2; }
    memcpy(out + off, L->tx, a * 8); off += a;
    memcpy(out + off, L->ty, b * 8); off += b;
    if (c) { memcpy(out + off, L->tz, c * 8); off += c; }
  }
  int nl = P.nlev;
  free_problem(&P);
  return nl;
}
