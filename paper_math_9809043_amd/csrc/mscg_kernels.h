// mscg_kernels.h -- launcher interface between the host engine and the gfx950
// kernels of the recursive multi-scale PCG.
#pragma once

#include <hip/hip_runtime.h>

#include "mscg_dev.h"

namespace mscg {

constexpr int kMaxPartials = 1024;  // blocks of a grid-wide reduction
constexpr int kPartSlots = 8192;    // partials the workspace holds (the tiled post-smoother's r . z per tile)
constexpr int kPartPq = 4096;       // offsets of the p.q and |r|^2 partials when the finishes are folded in
constexpr int kPartRr = 6144;

// Device-resident scalars of one level's CG (Templates Figure 2.5).
struct Scal {
  double bb;    // |b|^2 (finest level)
  double rr;    // |r|^2 after the last update
  double rho;   // r . z of the current iteration
  double beta;  // rho / rho_previous
  double alpha; // rho / (p . A p)
  double tol;   // absolute criterion on |r|^2: N_k f^k eps^2
  double zq;    // z_new . q_old (flexible beta)
  double rel_floor2;  // mixed precision: the entry check raises tol to rel_floor2 |r|^2 (0 = off)
  int it;       // iterations done in the current call
  int converged;  // also the gate of speculatively queued iterations: set, they do nothing
  int status;   // 0, 1 (r.z or p.Ap <= 0) or -4 (non-finite)
  int flexible; // beta: 0 Fletcher-Reeves rho/rho_old, 1 Polak-Ribiere z.(r - r_old)/rho_old
  int started;  // iterations begun in the current call (counted at r.z)
  int pad_;
};

enum { kOpBB = 0, kOpEntry = 1, kOpRho = 2, kOpPq = 3, kOpRr = 4, kOpZq = 5 };

struct FaceTArgs {
  int dim, nx, ny, nz;
  double ax, ay, az;  // area / distance per axis
  const double *kx, *ky, *kz;
  int bc_type[6];
  double *tx, *ty, *tz;
};

struct CoarsenArgs {
  int axis;
  int frac;  // 1: the factors fd / cd need not be integers (s unused)
  int fd[3], cd[3], s[3];
  const double* f;
  double* c;
};

struct RhsArgs {
  int dim, nx, ny, nz, n;
  double vol;
  const double* f;
  const double *tx, *ty, *tz;
  int bc_type[6];
  double bc_value[6];
  double* b;
};

template <typename R>
struct SmallDesc {
  Lv<R> L[kMaxLevels];
  Xfer X[kMaxLevels];
  R *x[kMaxLevels], *r[kMaxLevels], *z[kMaxLevels], *p[kMaxLevels], *q[kMaxLevels];
  double tol[kMaxLevels];
  int ks, nlev, m, max_inner;
  double rel_floor2;
  const double* Ainv;
  const double* Asym;  // lower triangle of Ainv in 16 x 16 tiles (launch_pack_sym), or null
  int ntile;           // its tiles per side
  int ncoarse;
  long long *iters, *calls;
  int* status;
  int variant;  // one-workgroup kernel for 2-D levels: 0 2x2-block where it fits, else colour-split;
                // 1 cell-strided; 2 colour-split
  const int* gate;  // see the gate of the grid-wide kernels
};

hipError_t launch_face_T(const FaceTArgs& a, hipStream_t s);
hipError_t launch_check_positive(const double* k, long long n, int* bad, hipStream_t s);
hipError_t launch_coarsen(const CoarsenArgs& a, hipStream_t s);
hipError_t launch_to_f32(const double* a, float* b, long long n, hipStream_t s);
hipError_t launch_coarse_factor(const Lv<double>& L, double* A, double* Lrows, double* Ainv, int* status,
                                hipStream_t s);
hipError_t launch_finish(const double* part, int nparts, Scal* sc, int op, hipStream_t s, const int* gate = nullptr);
// Tile t = I (I + 1) / 2 + J (I >= J) of out holds A^-1[16 I + (s xor c)][16 J + c]
// at t 256 + 16 s + c (skewed: slot s of column c is row s xor c), zero past n;
// ntile = ceil(n / 16) tiles per side.
hipError_t launch_pack_sym(const double* Ainv, int n, int ntile, double* out, hipStream_t s);
hipError_t launch_rhs(const RhsArgs& a, hipStream_t s);
hipError_t launch_init_x(double* x, int n, int nx, double hx, double Lx, double p0, double p1, int ramp, hipStream_t s);
hipError_t launch_scale_to_f32(const double* a, float* b, int n, const Scal* sc, hipStream_t s);
hipError_t launch_scale_to_f64(const float* a, double* b, int n, const Scal* sc, hipStream_t s);

template <typename R>
hipError_t launch_spmv(const Lv<R>& L, const R* x, R* y, double* part, int nparts, hipStream_t s);
template <typename R>
hipError_t launch_residual(const Lv<R>& L, const R* b, const R* x, R* r, double* part, int nparts, hipStream_t s);
template <typename R>
hipError_t launch_dot(const R* a, const R* b, int n, double* part, int nparts, hipStream_t s);
template <typename R>
hipError_t launch_update_p(const R* z, R* p, int n, const Scal* sc, hipStream_t s);
template <typename R>
hipError_t launch_cg_update(R* x, R* r, const R* p, const R* q, int n, const Scal* sc, double* part, int nparts,
                            hipStream_t s);
// Kernels of an inner iteration take `gate`: when non-null and *gate != 0 (the
// level has converged or stopped) they return at once, so iterations queued
// ahead of the convergence test cost only their launch.
template <typename R>
hipError_t launch_gs_half(const Lv<R>& L, const R* r, R* x, int colour, int first, hipStream_t s,
                          const int* gate = nullptr);
// One modified Jacobi step xout = xin + (r - A xin) / (2d) (xin = 0 when first);
// xout must not alias xin.
template <typename R>
hipError_t launch_mjac_step(const Lv<R>& L, const R* r, const R* xin, R* xout, int first, hipStream_t s,
                            const int* gate = nullptr);
template <typename R>
hipError_t launch_restrict(const Lv<R>& F, const Xfer& X, const R* r, const R* x, R* g, hipStream_t s);
template <typename R>
hipError_t launch_residual_restrict(const Lv<R>& F, const Xfer& X, const R* r, const R* x, R* tmp, R* g,
                                    hipStream_t s, const int* gate = nullptr);
template <typename R>
hipError_t launch_prolong(const Lv<R>& F, const Xfer& X, const R* y, R* x, hipStream_t s, const int* gate = nullptr);
template <typename R>
hipError_t launch_coarse_solve(const double* Ainv, const R* g, R* y, int n, hipStream_t s,
                               const int* gate = nullptr);
// A reduction kernel (gated) followed by its one-workgroup finish (gated),
// which sums the partials in block order and updates sc with op.
template <typename R>
hipError_t launch_dot_fin(const R* a, const R* b, int n, double* part, int nparts, Scal* sc, int op, hipStream_t s,
                          const int* gate = nullptr);
// p_new = z (+ beta p_old), q = A p_new; finish: alpha = rho / p_new.q
template <typename R>
hipError_t launch_pspmv_fin(const Lv<R>& L, const R* z, const R* pold, R* pnew, R* q, double* part, int nparts,
                            Scal* sc, hipStream_t s, const int* gate = nullptr);
// x += alpha p, r -= alpha q; finish: rr = |r|^2 and the convergence test
template <typename R>
hipError_t launch_cg_update_fin(R* x, R* r, const R* p, const R* q, int n, double* part, int nparts, Scal* sc,
                                hipStream_t s, const int* gate = nullptr);
// The CG iteration with the r.z and p.q finishes folded into the kernels that
// consume them: launch_dot_part leaves r.z partials (no finish);
// launch_pspmv_rho sums them in every workgroup (beta), forms p and q = A p
// and leaves p.q partials in ppq; launch_update_pq_fin sums both (alpha),
// updates x and r, leaves |r|^2 partials in prr and runs their finish.  The
// three partial arrays must not overlap.  Bitwise the same as the finished
// path (same sums in the same order).
template <typename R>
hipError_t launch_dot_part(const R* a, const R* b, int n, double* part, int nparts, hipStream_t s,
                           const int* gate = nullptr);
template <typename R>
hipError_t launch_pspmv_rho(const Lv<R>& L, const R* z, const R* pold, R* pnew, R* q, const double* prho, int nrho,
                            double* ppq, int nparts, Scal* sc, hipStream_t s, const int* gate = nullptr);
template <typename R>
hipError_t launch_update_pq_fin(R* x, R* r, const R* p, const R* q, int n, const double* prho, int nrho,
                                const double* ppq, double* prr, int nparts, Scal* sc, hipStream_t s,
                                const int* gate = nullptr);
template <typename R>
hipError_t launch_fill(R* a, long long n, R v, hipStream_t s);
template <typename R>
hipError_t launch_copy(const R* a, R* b, long long n, hipStream_t s);
template <typename R>
hipError_t launch_small_pcg(const SmallDesc<R>& d, hipStream_t s);
// Register-resident variant for one small level directly above the coarsest
// (at most 4096 cells); hipErrorNotSupported when the hierarchy does not fit.
template <typename R>
hipError_t launch_small_reg(const SmallDesc<R>& d, hipStream_t s);

// The same for a 2-D level with at most 2048 cells of each colour (colour-
// split LDS layout); hipErrorNotSupported otherwise.
template <typename R>
hipError_t launch_small_2d(const SmallDesc<R>& d, hipStream_t s);

// The same for a 2-D level of at most 64 x 64 cells, one 2 x 2 block of cells
// per thread with the iterate in registers; hipErrorNotSupported otherwise.
template <typename R>
hipError_t launch_small_2x2(const SmallDesc<R>& d, hipStream_t s);

// m symmetric Gauss-Seidel steps (2m+1 red-black half sweeps) on a 2-D level,
// temporally blocked in LDS.  X == nullptr: pre-smoothing from zero into zout;
// otherwise post-smoothing from zin + E y into zout (zout must not alias zin).
// Tiles are built for m = 4; smooth_tile_supported says whether a level can use
// them (hipErrorNotSupported otherwise).  shape: tile shape 0..3, or -1 to
// choose by the level size.  With part (post-smoothing only), tile t also
// writes part[t] = its share of r . zout, smooth_tile_count tiles in all.
bool smooth_tile_supported(int nz, bool has_tz, int m);
int smooth_tile_count(int nx, int ny, int shape);
template <typename R>
hipError_t launch_smooth_tile(const Lv<R>& L, const Xfer* X, const R* r, const R* zin, const R* y, R* zout, int m,
                              int shape, hipStream_t s, const int* gate = nullptr, double* part = nullptr);

// g = E^T (r - A z) on a 2-D level in one launch (factors s <= 4 per axis);
// hipErrorNotSupported otherwise.  Same sums, in the same order, as
// launch_residual_restrict.
bool resid_restrict_tile_supported(const Lv<double>& L, const Xfer& X);
template <typename R>
hipError_t launch_resid_restrict_tile(const Lv<R>& L, const Xfer& X, const R* r, const R* z, R* g, hipStream_t s,
                                      const int* gate = nullptr);

// Number of blocks (= partials) of a grid-wide reduction over n cells.
inline int reduce_blocks(long long n) {
  long long b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > kMaxPartials) b = kMaxPartials;
  return (int)b;
}

}  // namespace mscg
