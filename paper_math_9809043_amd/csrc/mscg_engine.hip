// mscg_engine.hip -- host engine and C ABI of the recursive multi-scale PCG.
//
// The finest levels run grid-wide kernels driven from the host, one small
// device-to-host read per CG iteration for the convergence decision.  From
// the first level whose cell count is at most kSmallN downwards, the whole
// inner PCG (with its own recursion and the coarsest solve) runs inside one
// workgroup launch, so those many short iterations never leave the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/mscg.h"
#include "mscg_kernels.h"

using namespace mscg;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(MSCG_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kSmallNDefault = 4096;

int small_n() {
  static int v = [] {
    const char* e = getenv("MSCG_SMALL_N");
    return e ? atoi(e) : kSmallNDefault;
  }();
  return v;
}

struct LevelPlan {
  int n3[3];
  int n;
};

struct Plan {
  int nlev;
  LevelPlan lv[MSCG_MAX_LEVELS];
  size_t bytes;
};

// Level hierarchy (Section 3: factor `scale` per axis, exact divisibility,
// coarsen while every side / scale >= min_coarse_side).
int make_plan(const mscg_grid* g, const mscg_options* o, Plan* P) {
  if (!g) return fail(MSCG_E_ARG, "grid is NULL");
  if (g->dim != 2 && g->dim != 3) return fail(MSCG_E_ARG, "dim must be 2 or 3 (got %d)", g->dim);
  int d[3] = {g->n[0], g->n[1], g->dim == 3 ? g->n[2] : 1};
  for (int a = 0; a < g->dim; ++a)
    if (d[a] < 1) return fail(MSCG_E_ARG, "n[%d] = %d must be >= 1", a, d[a]);
  const long long N = (long long)d[0] * d[1] * d[2];
  if (N > (1LL << 30)) return fail(MSCG_E_ARG, "grid too large (%lld cells)", N);
  for (int f = 0; f < 6; ++f)
    if (g->bc_type[f] != MSCG_NEUMANN && g->bc_type[f] != MSCG_DIRICHLET)
      return fail(MSCG_E_ARG, "bc_type[%d] must be MSCG_NEUMANN or MSCG_DIRICHLET", f);
  if (o->scale < 2 || o->scale > 8) return fail(MSCG_E_ARG, "scale must be in [2, 8]");
  if (o->smooth_steps < 1) return fail(MSCG_E_ARG, "smooth_steps must be >= 1");
  if (!(o->level_factor > 0.0)) return fail(MSCG_E_ARG, "level_factor must be > 0");
  if (o->interp != MSCG_INTERP_LINEAR && o->interp != MSCG_INTERP_CONSTANT) return fail(MSCG_E_ARG, "bad interp");
  if (o->precision != MSCG_FP64 && o->precision != MSCG_MIXED) return fail(MSCG_E_ARG, "bad precision");
  if (o->max_outer_iters < 1 || o->max_inner_iters < 1) return fail(MSCG_E_ARG, "iteration caps must be >= 1");
  int maxl = o->max_levels < 1 ? 1 : (o->max_levels > MSCG_MAX_LEVELS ? MSCG_MAX_LEVELS : o->max_levels);
  if (o->semi_coarsen != 0 && o->semi_coarsen != 1) return fail(MSCG_E_ARG, "semi_coarsen must be 0 or 1");
  if (o->splitting != MSCG_SPLIT_SGS && o->splitting != MSCG_SPLIT_JACOBI) return fail(MSCG_E_ARG, "bad splitting");
  if (o->cycle != MSCG_CYCLE_RECURSIVE && o->cycle != MSCG_CYCLE_MGCG && o->cycle != MSCG_CYCLE_POLY)
    return fail(MSCG_E_ARG, "bad cycle");
  if (o->semi_coarsen)
    for (int a = 0; a < g->dim; ++a)
      if (!(o->axis_weight[a] > 0.0)) return fail(MSCG_E_ARG, "axis_weight[%d] must be > 0", a);
  const bool frac = o->frac_scale != 0.0;
  if (frac && !(o->frac_scale > 1.0 && o->frac_scale <= 16.0))
    return fail(MSCG_E_ARG, "frac_scale must be 0 or in (1, 16]");
  if (frac && o->semi_coarsen) return fail(MSCG_E_ARG, "frac_scale cannot be combined with semi_coarsen");
  int nl = 0;
  for (;;) {
    LevelPlan& L = P->lv[nl];
    L.n3[0] = d[0]; L.n3[1] = d[1]; L.n3[2] = d[2];
    L.n = d[0] * d[1] * d[2];
    ++nl;
    if (nl >= maxl) break;
    if (frac) {
      // a factor that need not be an integer: round(d / frac_scale) per axis
      int c[3] = {d[0], d[1], d[2]};
      bool ok = true;
      for (int a = 0; a < g->dim; ++a) {
        c[a] = (int)std::floor(d[a] / o->frac_scale + 0.5);
        if (c[a] < o->min_coarse_side || c[a] >= d[a]) ok = false;
      }
      if (!ok) break;
      for (int a = 0; a < g->dim; ++a) d[a] = c[a];
      continue;
    }
    if (o->semi_coarsen) {
      // aspect-ratio-aware: coarsen the axes whose effective cell size is within
      // sqrt(scale) of the smallest among those that can be coarsened
      bool can[3] = {false, false, false}, any = false;
      double e[3] = {0.0, 0.0, 0.0}, emin = 0.0;
      for (int a = 0; a < g->dim; ++a) {
        const double len = g->length[a] > 0.0 ? g->length[a] : 1.0;
        can[a] = d[a] % o->scale == 0 && d[a] / o->scale >= o->min_coarse_side;
        e[a] = (len / d[a]) / std::sqrt(o->axis_weight[a]);
        if (can[a] && (!any || e[a] < emin)) emin = e[a];
        any = any || can[a];
      }
      if (!any) break;
      for (int a = 0; a < g->dim; ++a)
        if (can[a] && e[a] <= emin * std::sqrt((double)o->scale) * (1.0 + 1e-12)) d[a] /= o->scale;
      continue;
    }
    bool ok = true;
    for (int a = 0; a < g->dim; ++a)
      if (d[a] % o->scale != 0 || d[a] / o->scale < o->min_coarse_side) ok = false;
    if (!ok) break;
    for (int a = 0; a < g->dim; ++a) d[a] /= o->scale;
  }
  P->nlev = nl;
  if (P->lv[nl - 1].n > MSCG_MAX_COARSE)
    return fail(MSCG_E_ARG, "coarsest level has %d cells > %d: grid sides must allow coarsening by %d", P->lv[nl - 1].n,
                MSCG_MAX_COARSE, o->scale);
  // bytes
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~(size_t)255; };
  const bool mixed = o->precision == MSCG_MIXED;
  for (int l = 0; l < nl; ++l) {
    const LevelPlan& L = P->lv[l];
    const size_t fx = (size_t)(L.n3[0] + 1) * L.n3[1] * L.n3[2], fy = (size_t)L.n3[0] * (L.n3[1] + 1) * L.n3[2];
    const size_t fz = g->dim == 3 ? (size_t)L.n3[0] * L.n3[1] * (L.n3[2] + 1) : 0;
    add(fx * 8); add(fy * 8); if (fz) add(fz * 8);
    if (mixed) { add(fx * 4); add(fy * 4); if (fz) add(fz * 4); }
    const bool fp64_vec = !mixed || l == 0;
    for (int v = 0; v < 7; ++v) add((size_t)L.n * (fp64_vec ? 8 : 4));
    if (mixed && l == 0) { add((size_t)L.n * 4); add((size_t)L.n * 4); add((size_t)L.n * 4); }  // scaled r, iterate, output
    add(sizeof(Scal));
  }
  add((size_t)P->lv[0].n * 8);  // b
  const size_t nc = (size_t)P->lv[nl - 1].n;
  add(nc * nc * 8); add(nc * nc * 8); add(nc * nc * 8);  // A (then its factor), row-major factor, A^-1
  add((size_t)kPartSlots * 8);
  add(64);                                              // flags
  add(2 * MSCG_MAX_LEVELS * sizeof(long long));         // small-kernel counters
  P->bytes = b;
  return MSCG_OK;
}

struct LevelH {
  int nx, ny, nz, n;
  double hx, hy, hz;
  int sx, sy, sz;
  double *tx, *ty, *tz;
  float *tx32, *ty32, *tz32;
  double *x, *r, *z, *p, *q, *w, *p2;  // FP64 vectors (FP64 mode, or level 0); w: residual / post-smoothing
                                       // output; p, p2: directions, alternating
  float *x32, *r32, *z32, *p32, *q32, *w32, *p232;  // FP32 vectors (mixed inner levels; level 0: r32, z32, w32)
  Scal* sc;
};

}  // namespace

struct mscg_problem {
  mscg_grid g;
  mscg_options o;
  hipStream_t stream;
  int device;
  int nlev, ks;
  LevelH lev[MSCG_MAX_LEVELS];
  double *Atmp, *Lrows, *Ainv;
  const double* Asym;  // packed lower triangle of Ainv (in Atmp), or null
  int ntile;
  int ncoarse;
  double* part;
  double* b;
  int* dflags;        // [0] coarse factor status, [1] bad K, [2] small-kernel status
  int spec_hint[MSCG_MAX_LEVELS];  // iterations of the level's last call: how many to queue ahead
  bool queue_ahead;   // queue inner iterations ahead of their convergence test
  // launch timing of the one-workgroup solver of the last inner level
  bool ktime;
  std::vector<hipEvent_t> kev;  // event pairs around its launches, reused
  size_t kev_used;
  double ktime_ms, kflops;
  long long klaunches, kiters;
  long long* dcount;  // [0..7] small iters, [8..15] small calls
  Scal* hsc;          // pinned mirror of one Scal
  int* hflags;        // pinned
  long long* hcount;  // pinned
  char* ws;
  size_t ws_bytes;
  bool owns_ws;
  bool ready;
  bool tiled;         // 2-D levels smooth with the tiled kernel
  int tile_shape;     // its tile shape (-1: by level size)
  bool fuse_dot;      // the tiled post-smoother also forms the CG's r . z
  bool sym_coarse;    // one-workgroup solvers apply the coarsest inverse from its lower triangle
  bool fuse_finish;   // the SpMV and update kernels sum the r.z and p.q partials themselves
  int small_variant;  // one-workgroup kernel of 2-D small levels (0 2x2-block, else colour-split; 1 cell-strided; 2 colour-split)
  // per-solve state
  double eps2;
  double tol_scale;   // mixed: 1 / |r|^2 of the current outer iteration
  long long iters[MSCG_MAX_LEVELS], calls[MSCG_MAX_LEVELS];
  int status;
};

namespace {

bool mixed(const mscg_problem* P) { return P->o.precision == MSCG_MIXED; }

Lv<double> lv64(const mscg_problem* P, int k) {
  const LevelH& L = P->lev[k];
  return Lv<double>{L.nx, L.ny, L.nz, L.n, L.tx, L.ty, P->g.dim == 3 ? L.tz : nullptr};
}
Lv<float> lv32(const mscg_problem* P, int k) {
  const LevelH& L = P->lev[k];
  return Lv<float>{L.nx, L.ny, L.nz, L.n, L.tx32, L.ty32, P->g.dim == 3 ? L.tz32 : nullptr};
}
Xfer xfer(const mscg_problem* P, int k) {
  const LevelH& F = P->lev[k];
  const LevelH& C = P->lev[k + 1];
  return Xfer{F.sx, F.sy, F.sz, C.nx, C.ny, C.nz, P->o.interp, P->o.frac_scale != 0.0 ? 1 : 0};
}

double level_tol(const mscg_problem* P, int k) {
  return (double)P->lev[k].n * std::pow(P->o.level_factor, k) * P->eps2;
}

int read_scal(mscg_problem* P, int k) {
  HIP_TRY(hipMemcpyAsync(P->hsc, P->lev[k].sc, sizeof(Scal), hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

// Device scalars live in the caller's workspace, whose contents are arbitrary.
int clear_scalars(mscg_problem* P) {
  static_assert(sizeof(Scal) % sizeof(double) == 0, "Scal is cleared as doubles");
  for (int l = 0; l < P->nlev; ++l) {
    HIP_TRY(launch_fill<double>(reinterpret_cast<double*>(P->lev[l].sc), sizeof(Scal) / sizeof(double), 0.0, P->stream));
    if (P->o.flexible) HIP_TRY(launch_fill<int>(&P->lev[l].sc->flexible, 1, 1, P->stream));
    if (mixed(P) && l > 0 && P->o.inner_rel_floor > 0.0)
      HIP_TRY(launch_fill<double>(&P->lev[l].sc->rel_floor2, 1, P->o.inner_rel_floor * P->o.inner_rel_floor,
                                  P->stream));
  }
  return MSCG_OK;
}

int set_tol(mscg_problem* P, int k, double tol) {
  // the tolerance lives in device scalars; a one-element fill keeps it stream ordered
  HIP_TRY(launch_fill<double>(&P->lev[k].sc->tol, 1, tol, P->stream));
  return MSCG_OK;
}

// ---------------------------------------------------------------------------
// Host-driven recursion for the large levels.  T is the storage type of the
// level's preconditioner vectors (FP64, or FP32 in mixed mode).
// ---------------------------------------------------------------------------

int pcg_host(mscg_problem* P, int k);

// Next event of the launch-timing pool (created on first use, kept until the
// problem is destroyed).
hipEvent_t timing_event(mscg_problem* P) {
  if (P->kev_used == P->kev.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    P->kev.push_back(e);
  }
  return P->kev[P->kev_used++];
}

// Algorithmic FP64 operations of one iteration of the one-workgroup solver on
// a 2-D level of n cells (nx x ny) above a coarsest level of nc cells (ncx
// wide): 2m+1 half sweeps before and after (9 per cell update: four products,
// four sums, one division), residual (10 n), restriction (4 n + 4 ny ncx),
// dense coarsest solve (2 nc^2), prolongation (10 n), CG vectors (21 n).
double small_level_flops(const mscg_problem* P) {
  const int ks = P->nlev - 2;
  if (ks < 0) return 0.0;
  const LevelH& S = P->lev[ks];
  const LevelH& C = P->lev[ks + 1];
  const double n = S.n, nc = C.n, m = P->o.smooth_steps;
  return (9.0 * (2.0 * m + 1.0) + 45.0) * n + 4.0 * S.ny * S.nz * C.nx + 2.0 * nc * nc;
}

template <typename R>
R* precond_host(mscg_problem* P, int k, const Lv<R>& L, const R* r, R* z, R* w, R* const* xs, R* const* rs,
                R* const* zs, R* const* ps, R* const* qs, int* rc, const int* gate, int* nfused);

// Coarse part of the preconditioner on level k: y_{k+1} = A_{k+1}^-1 g, or
// y_{k+1} = M_{k+1}^-1 g with Tatebe's multigrid form.
template <typename R>
int coarse_correction(mscg_problem* P, int k, R* const* xs, R* const* rs, R* const* zs, R* const* ps, R* const* qs,
                      const int* gate) {
  const int kc = k + 1;
  if (kc == P->nlev - 1) {
    HIP_TRY(launch_coarse_solve<R>(P->Ainv, rs[kc], xs[kc], P->ncoarse, P->stream, gate));
    if (!gate) P->calls[kc]++;  // queued-ahead iterations are counted by cg_loop
    return MSCG_OK;
  }
  if (P->o.cycle == MSCG_CYCLE_MGCG) {
    // eq. 2.9: the next level's preconditioner applied once to g, in place of
    // its PCG solve.  Its pre-smoothing iterate goes to z_{k+1}; its result
    // is wanted in x_{k+1}, which also serves as its second work vector.
    Lv<R> Lc;
    if constexpr (std::is_same<R, float>::value) Lc = lv32(P, kc);
    else Lc = lv64(P, kc);
    int rc = MSCG_OK;
    R* out = precond_host<R>(P, kc, Lc, rs[kc], zs[kc], xs[kc], xs, rs, zs, ps, qs, &rc, gate, nullptr);
    if (rc) return rc;
    if (out != xs[kc]) HIP_TRY(launch_copy<R>(out, xs[kc], Lc.n, P->stream));
    if (!gate) P->calls[kc]++;
    return MSCG_OK;
  }
  if (kc >= P->ks) {
    SmallDesc<R> d{};
    for (int l = 0; l < P->nlev; ++l) {
      if (l + 1 < P->nlev) d.X[l] = xfer(P, l);
      d.x[l] = xs[l]; d.r[l] = rs[l]; d.z[l] = zs[l]; d.p[l] = ps[l]; d.q[l] = qs[l];
      d.tol[l] = level_tol(P, l) * P->tol_scale;
    }
    if constexpr (std::is_same<R, float>::value) {
      for (int l = 0; l < P->nlev; ++l) d.L[l] = lv32(P, l);
    } else {
      for (int l = 0; l < P->nlev; ++l) d.L[l] = lv64(P, l);
    }
    d.ks = kc;
    d.nlev = P->nlev;
    d.m = P->o.smooth_steps;
    d.max_inner = P->o.max_inner_iters;
    d.rel_floor2 = mixed(P) ? P->o.inner_rel_floor * P->o.inner_rel_floor : 0.0;
    d.Ainv = P->Ainv;
    d.Asym = P->Asym;
    d.ntile = P->ntile;
    d.ncoarse = P->ncoarse;
    d.iters = P->dcount;
    d.calls = P->dcount + MSCG_MAX_LEVELS;
    d.status = P->dflags + 2;
    d.variant = P->small_variant;
    d.gate = gate;
    if (P->ktime) HIP_TRY(hipEventRecord(timing_event(P), P->stream));
    const hipError_t e = launch_small_reg<R>(d, P->stream);
    if (e == hipErrorNotSupported) HIP_TRY(launch_small_pcg<R>(d, P->stream));
    else HIP_TRY(e);
    if (P->ktime) HIP_TRY(hipEventRecord(timing_event(P), P->stream));
    return MSCG_OK;
  }
  return pcg_host(P, kc);
}

// z_k = M_k^-1 r_k (eq. 2.10 as a two-grid cycle).  Vectors of type R.  The
// pre-smoothing iterate is z; w holds the residual for the restriction and
// then, on 2-D levels, the output of the tiled post-smoothing (which cannot
// run in place: its halos read neighbouring tiles).  Returns the vector that
// holds M_k^-1 r_k.  q is not touched, so the flexible beta can still use it.
template <typename R>
R* precond_host(mscg_problem* P, int k, const Lv<R>& L, const R* r, R* z, R* w, R* const* xs, R* const* rs,
                R* const* zs, R* const* ps, R* const* qs, int* rc, const int* gate, int* nfused) {
  const int m = P->o.smooth_steps;
  const Xfer X = xfer(P, k);
  *rc = MSCG_OK;
  if (nfused) *nfused = 0;
  auto chk = [&](hipError_t e) {
    if (e != hipSuccess && *rc == MSCG_OK) *rc = fail(MSCG_E_DEVICE, "precond level %d: %s", k, hipGetErrorString(e));
    return e == hipSuccess;
  };
  if (P->o.cycle == MSCG_CYCLE_POLY) {
    // polynomial preconditioner (Section 2.1): W = P^-1 turns eq. 2.6 into
    // 2m+1 steps of the splitting from zero on this level alone
    const int steps = 2 * m + 1;
    if (P->o.splitting == MSCG_SPLIT_JACOBI) {
      R* cur = z;
      R* nxt = w;
      for (int step = 0; step < steps; ++step) {
        if (!chk(launch_mjac_step<R>(L, r, cur, nxt, step == 0, P->stream, gate))) return nullptr;
        std::swap(cur, nxt);
      }
      return cur;
    }
    for (int h = 0; h <= 2 * steps; ++h)
      if (!chk(launch_gs_half<R>(L, r, z, h & 1, h == 0, P->stream, gate))) return nullptr;
    return z;
  }
  if (P->o.splitting == MSCG_SPLIT_JACOBI) {
    // m modified Jacobi steps from zero, alternating between z and w; the
    // restriction's residual goes to the buffer not holding the iterate
    R* cur = z;
    R* nxt = w;
    for (int step = 0; step < m; ++step) {
      if (!chk(launch_mjac_step<R>(L, r, cur, nxt, step == 0, P->stream, gate))) return nullptr;
      std::swap(cur, nxt);
    }
    if (!chk(launch_residual_restrict<R>(L, X, r, cur, nxt, rs[k + 1], P->stream, gate))) return nullptr;
    *rc = coarse_correction<R>(P, k, xs, rs, zs, ps, qs, gate);
    if (*rc) return nullptr;
    if (!chk(launch_prolong<R>(L, X, xs[k + 1], cur, P->stream, gate))) return nullptr;
    for (int step = 0; step < m; ++step) {
      if (!chk(launch_mjac_step<R>(L, r, cur, nxt, 0, P->stream, gate))) return nullptr;
      std::swap(cur, nxt);
    }
    return cur;
  }
  const bool tiled = P->tiled && smooth_tile_supported(L.nz, L.tz != nullptr, m);
  if (tiled) {
    if (!chk(launch_smooth_tile<R>(L, nullptr, r, nullptr, nullptr, z, m, P->tile_shape, P->stream, gate)))
      return nullptr;
  } else {
    for (int h = 0; h <= 2 * m; ++h)
      if (!chk(launch_gs_half<R>(L, r, z, h & 1, h == 0, P->stream, gate))) return nullptr;
  }
  if (tiled) {
    const hipError_t e = launch_resid_restrict_tile<R>(L, X, r, z, rs[k + 1], P->stream, gate);
    if (e == hipErrorNotSupported) {
      if (!chk(launch_residual_restrict<R>(L, X, r, z, w, rs[k + 1], P->stream, gate))) return nullptr;
    } else if (!chk(e)) {
      return nullptr;
    }
  } else if (!chk(launch_residual_restrict<R>(L, X, r, z, w, rs[k + 1], P->stream, gate))) {
    return nullptr;
  }
  *rc = coarse_correction<R>(P, k, xs, rs, zs, ps, qs, gate);
  if (*rc) return nullptr;
  // the tiled post-smoother's fused prolongation assumes integer factors; the
  // tiled residual + restriction above falls back by itself
  if (tiled && !X.frac) {
    // the post-smoother also leaves the CG's r . z in per-tile partials
    double* fpart = nullptr;
    if (nfused && P->fuse_dot && !P->o.flexible) {
      const int nt = smooth_tile_count(L.nx, L.ny, P->tile_shape);
      if (nt <= kPartPq) {
        fpart = P->part;
        *nfused = nt;
      }
    }
    if (!chk(launch_smooth_tile<R>(L, &X, r, z, xs[k + 1], w, m, P->tile_shape, P->stream, gate, fpart)))
      return nullptr;
    return w;
  }
  if (!chk(launch_prolong<R>(L, X, xs[k + 1], z, P->stream, gate))) return nullptr;
  for (int h = 0; h <= 2 * m; ++h)
    if (!chk(launch_gs_half<R>(L, r, z, h & 1, 0, P->stream, gate))) return nullptr;
  return z;
}

template <typename R>
void vec_tables(mscg_problem* P, R** xs, R** rs, R** zs, R** ps, R** qs) {
  for (int l = 0; l < P->nlev; ++l) {
    LevelH& L = P->lev[l];
    if constexpr (std::is_same<R, double>::value) {
      xs[l] = L.x; rs[l] = L.r; zs[l] = L.z; ps[l] = L.p; qs[l] = L.q;
    } else {
      xs[l] = L.x32; rs[l] = L.r32; zs[l] = L.z32; ps[l] = L.p32; qs[l] = L.q32;
    }
  }
}

// Applies the level-k preconditioner to the level's residual; *out receives
// the vector (in the level's CG precision) that holds the result.  With
// nfused, *nfused > 0 says that P->part holds that many partials of r . out.
int apply_prec(mscg_problem* P, int k, void** out, const int* gate, int* nfused = nullptr) {
  if (nfused) *nfused = 0;
  int rc = MSCG_OK;
  if (!mixed(P)) {
    double *xs[MSCG_MAX_LEVELS], *rs[MSCG_MAX_LEVELS], *zs[MSCG_MAX_LEVELS], *ps[MSCG_MAX_LEVELS], *qs[MSCG_MAX_LEVELS];
    vec_tables<double>(P, xs, rs, zs, ps, qs);
    LevelH& H = P->lev[k];
    *out = precond_host<double>(P, k, lv64(P, k), H.r, H.z, H.w, xs, rs, zs, ps, qs, &rc, gate, nfused);
    return rc;
  }
  float *xs[MSCG_MAX_LEVELS], *rs[MSCG_MAX_LEVELS], *zs[MSCG_MAX_LEVELS], *ps[MSCG_MAX_LEVELS], *qs[MSCG_MAX_LEVELS];
  vec_tables<float>(P, xs, rs, zs, ps, qs);
  if (k == 0) {
    // FP64 residual -> unit-norm FP32, precondition in FP32, scale back (Section 2.3:
    // the inner solves only need the overall accuracy; the outer CG recovers FP64)
    LevelH& L0 = P->lev[0];
    HIP_TRY(launch_scale_to_f32(L0.r, L0.r32, L0.n, L0.sc, P->stream));
    float* z32 =
        precond_host<float>(P, 0, lv32(P, 0), L0.r32, L0.z32, L0.w32, xs, rs, zs, ps, qs, &rc, gate, nullptr);
    if (rc) return rc;
    HIP_TRY(launch_scale_to_f64(z32, L0.z, L0.n, L0.sc, P->stream));
    *out = L0.z;
    return MSCG_OK;
  }
  LevelH& H = P->lev[k];
  *out = precond_host<float>(P, k, lv32(P, k), H.r32, H.z32, H.w32, xs, rs, zs, ps, qs, &rc, gate, nfused);
  return rc;
}

// One level's CG loop (Templates Figure 2.5) on vectors of type R; the residual
// is in r_k and the entry check has been done (sc->converged).  Per iteration:
// the preconditioner, r.z, p and A p with p.q, then the x / r update with
// |r|^2.  r.z comes as per-tile partials from the tiled post-smoother where
// that runs; the SpMV kernel sums them itself (beta) and the update kernel
// sums them and the p.q partials (alpha), so only |r|^2 has a one-workgroup
// finish (with the flexible beta, every reduction has one).  The directions
// alternate between p and p2 (the next one is formed from the current one on
// the fly, inside the SpMV).
//
// On the deepest host-driven level the iteration holds no host decision (the
// coarse correction runs entirely on the device), so iterations are queued
// ahead in batches, gated on the level's converged flag, and the host waits
// once per batch: as many as the level's last call needed, then two at a
// time.  Iterations queued past convergence return at once.
template <typename R>
int cg_loop(mscg_problem* P, int k, const Lv<R>& L, R* x, R* r, R* z, R* p, R* p2, R* q, int max_iter) {
  LevelH& H = P->lev[k];
  const int nb = reduce_blocks(L.n);
  // With Tatebe's or the polynomial preconditioner a finest-level iteration
  // holds no host decision either (no inner PCG; the mixed-precision
  // rescaling of inner tolerances has nothing to act on), so it is queued the
  // same way.  The FP64 <-> FP32 conversions around the mixed preconditioner
  // are not gated; past convergence they only rewrite work vectors.
  const bool outer_device = k == 0 && !P->o.flexible && P->o.cycle != MSCG_CYCLE_RECURSIVE;
  const bool ahead = P->queue_ahead && ((k > 0 && (k + 1 == P->nlev - 1 || k + 1 >= P->ks)) || outer_device);
  const int* gate = ahead ? &H.sc->converged : nullptr;
  R* pc = p;
  R* pn = p2;
  int queued = 0;
  int rc = MSCG_OK;
  while (queued < max_iter) {
    int batch = 1;
    if (ahead) batch = std::max(1, std::min(queued == 0 ? P->spec_hint[k] : 2, max_iter - queued));
    for (int b = 0; b < batch; ++b, ++queued) {
      void* zres = nullptr;
      int nfused = 0;
      rc = apply_prec(P, k, &zres, gate, &nfused);
      if (rc) return rc;
      z = static_cast<R*>(zres);
      if (P->fuse_finish && !P->o.flexible) {
        // r.z and p.q summed by the kernels that need them (no finish kernels)
        int nrho = nfused;
        if (!nrho) {
          HIP_TRY(launch_dot_part<R>(r, z, L.n, P->part, nb, P->stream, gate));
          nrho = nb;
        }
        HIP_TRY(launch_pspmv_rho<R>(L, z, pc, pn, q, P->part, nrho, P->part + kPartPq, nb, H.sc, P->stream, gate));
        HIP_TRY(launch_update_pq_fin<R>(x, r, pn, q, L.n, P->part, nrho, P->part + kPartPq, P->part + kPartRr, nb,
                                        H.sc, P->stream, gate));
      } else {
        if (P->o.flexible && queued > 0)
          HIP_TRY(launch_dot_fin<R>(z, q, L.n, P->part, nb, H.sc, kOpZq, P->stream, gate));
        if (nfused)
          HIP_TRY(launch_finish(P->part, nfused, H.sc, kOpRho, P->stream, gate));
        else
          HIP_TRY(launch_dot_fin<R>(r, z, L.n, P->part, nb, H.sc, kOpRho, P->stream, gate));
        HIP_TRY(launch_pspmv_fin<R>(L, z, pc, pn, q, P->part, nb, H.sc, P->stream, gate));
        HIP_TRY(launch_cg_update_fin<R>(x, r, pn, q, L.n, P->part, nb, H.sc, P->stream, gate));
      }
      std::swap(pc, pn);
    }
    rc = read_scal(P, k);
    if (rc) return rc;
    // a stall (r.z or p.Ap <= 0 in finite precision) ends an inner level
    // quietly; on the finest level, and for non-finite values, it is a breakdown
    if (P->hsc->status < 0 || (P->hsc->status > 0 && k == 0)) {
      P->status = MSCG_E_BREAKDOWN;
      fail(MSCG_E_BREAKDOWN, "level %d iteration %d: %s (rho %g, alpha %g, rr %g)", k, P->hsc->started,
           P->hsc->status < 0 ? "non-finite reduction" : "r.z or p.Ap <= 0", P->hsc->rho, P->hsc->alpha, P->hsc->rr);
      break;
    }
    if (P->hsc->status > 0 || P->hsc->converged) break;
    if (k == 0 && mixed(P)) P->tol_scale = P->hsc->rr > 0.0 ? 1.0 / P->hsc->rr : 1.0;
  }
  P->iters[k] += P->hsc->started;
  if (ahead) {
    P->spec_hint[k] = P->hsc->started;
    if (outer_device) {
      // every coarser level is visited once per finest-level iteration (eq. 2.9)
      if (P->o.cycle == MSCG_CYCLE_MGCG)
        for (int l = 1; l < P->nlev; ++l) P->calls[l] += P->hsc->started;
    } else if (k + 1 == P->nlev - 1) {
      P->calls[k + 1] += P->hsc->started;
    }
  }
  return MSCG_OK;
}

// Inner PCG on a large level k >= 1: rhs already in r_k, x_k = 0.  The entry
// check (with the mixed-precision floor) runs on the device; a queued-ahead
// level does not wait for it, its iterations are gated on the result.
int pcg_host(mscg_problem* P, int k) {
  LevelH& H = P->lev[k];
  const int nb = reduce_blocks(H.n);
  P->calls[k]++;
  int rc = set_tol(P, k, level_tol(P, k) * P->tol_scale);
  if (rc) return rc;
  if (!mixed(P)) {
    HIP_TRY(launch_fill<double>(H.x, H.n, 0.0, P->stream));
    HIP_TRY(launch_dot_fin<double>(H.r, H.r, H.n, P->part, nb, H.sc, kOpEntry, P->stream));
  } else {
    HIP_TRY(launch_fill<float>(H.x32, H.n, 0.0f, P->stream));
    HIP_TRY(launch_dot_fin<float>(H.r32, H.r32, H.n, P->part, nb, H.sc, kOpEntry, P->stream));
  }
  const bool ahead = P->queue_ahead && (k + 1 == P->nlev - 1 || k + 1 >= P->ks);
  if (!ahead) {
    rc = read_scal(P, k);
    if (rc) return rc;
    if (P->hsc->converged) return MSCG_OK;
  }
  if (!mixed(P)) return cg_loop<double>(P, k, lv64(P, k), H.x, H.r, H.z, H.p, H.p2, H.q, P->o.max_inner_iters);
  return cg_loop<float>(P, k, lv32(P, k), H.x32, H.r32, H.z32, H.p32, H.p232, H.q32, P->o.max_inner_iters);
}

int carve(mscg_problem* P, const Plan& plan) {
  char* base = P->ws;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const bool mx = mixed(P);
  const int dim = P->g.dim;
  for (int l = 0; l < plan.nlev; ++l) {
    LevelH& L = P->lev[l];
    const LevelPlan& lp = plan.lv[l];
    L.nx = lp.n3[0]; L.ny = lp.n3[1]; L.nz = lp.n3[2]; L.n = lp.n;
    const size_t fx = (size_t)(L.nx + 1) * L.ny * L.nz, fy = (size_t)L.nx * (L.ny + 1) * L.nz;
    const size_t fz = dim == 3 ? (size_t)L.nx * L.ny * (L.nz + 1) : 0;
    L.tx = (double*)take(fx * 8); L.ty = (double*)take(fy * 8); L.tz = fz ? (double*)take(fz * 8) : nullptr;
    L.tx32 = L.ty32 = L.tz32 = nullptr;
    if (mx) { L.tx32 = (float*)take(fx * 4); L.ty32 = (float*)take(fy * 4); L.tz32 = fz ? (float*)take(fz * 4) : nullptr; }
    L.x = L.r = L.z = L.p = L.q = L.w = L.p2 = nullptr;
    L.x32 = L.r32 = L.z32 = L.p32 = L.q32 = L.w32 = L.p232 = nullptr;
    if (!mx || l == 0) {
      L.x = (double*)take((size_t)L.n * 8); L.r = (double*)take((size_t)L.n * 8); L.z = (double*)take((size_t)L.n * 8);
      L.p = (double*)take((size_t)L.n * 8); L.q = (double*)take((size_t)L.n * 8); L.w = (double*)take((size_t)L.n * 8);
      L.p2 = (double*)take((size_t)L.n * 8);
    } else {
      L.x32 = (float*)take((size_t)L.n * 4); L.r32 = (float*)take((size_t)L.n * 4); L.z32 = (float*)take((size_t)L.n * 4);
      L.p32 = (float*)take((size_t)L.n * 4); L.q32 = (float*)take((size_t)L.n * 4); L.w32 = (float*)take((size_t)L.n * 4);
      L.p232 = (float*)take((size_t)L.n * 4);
    }
    if (mx && l == 0) {
      L.r32 = (float*)take((size_t)L.n * 4);
      L.z32 = (float*)take((size_t)L.n * 4);
      L.w32 = (float*)take((size_t)L.n * 4);
    }
    L.sc = (Scal*)take(sizeof(Scal));
  }
  P->b = (double*)take((size_t)plan.lv[0].n * 8);
  const size_t nc = (size_t)plan.lv[plan.nlev - 1].n;
  P->Atmp = (double*)take(nc * nc * 8);
  P->Lrows = (double*)take(nc * nc * 8);
  P->Ainv = (double*)take(nc * nc * 8);
  P->ncoarse = (int)nc;
  P->part = (double*)take((size_t)kPartSlots * 8);
  P->dflags = (int*)take(64);
  P->dcount = (long long*)take(2 * MSCG_MAX_LEVELS * sizeof(long long));
  if (off > P->ws_bytes) return fail(MSCG_E_NOMEM, "workspace carving overflow");
  return MSCG_OK;
}

int validate_problem(const mscg_problem* P) {
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  return MSCG_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void mscg_default_options(mscg_options* o) {
  if (!o) return;
  o->precision = MSCG_FP64;
  o->scale = 4;
  o->smooth_steps = 4;
  o->level_factor = 0.1;
  o->min_coarse_side = 8;
  o->max_levels = MSCG_MAX_LEVELS;
  o->max_outer_iters = 200;
  o->max_inner_iters = 200;
  o->interp = MSCG_INTERP_LINEAR;
  o->flexible = 0;
  o->inner_rel_floor = 1e-6;
  o->semi_coarsen = 0;
  o->axis_weight[0] = o->axis_weight[1] = o->axis_weight[2] = 1.0;
  o->splitting = MSCG_SPLIT_SGS;
  o->cycle = MSCG_CYCLE_RECURSIVE;
  o->frac_scale = 0.0;
}

const char* mscg_last_error(void) { return g_err.c_str(); }

static mscg_options resolve_opts(const mscg_options* opt) {
  mscg_options o;
  mscg_default_options(&o);
  if (opt) {
    o = *opt;
    if (o.smooth_steps <= 0) o.smooth_steps = o.scale;
  }
  return o;
}

size_t mscg_footprint_bytes(const mscg_grid* grid, const mscg_options* opt) {
  g_err.clear();
  mscg_options o = resolve_opts(opt);
  Plan plan;
  if (make_plan(grid, &o, &plan) != MSCG_OK) return 0;
  return plan.bytes;
}

int mscg_create_problem(const mscg_grid* grid, const mscg_options* opt, void* workspace, size_t ws_bytes,
                        void* hip_stream, mscg_problem** out) {
  g_err.clear();
  if (!out) return fail(MSCG_E_ARG, "out is NULL");
  *out = nullptr;
  mscg_options o = resolve_opts(opt);
  Plan plan;
  int rc = make_plan(grid, &o, &plan);
  if (rc) return rc;
  if (workspace && ws_bytes < plan.bytes)
    return fail(MSCG_E_NOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, plan.bytes);
  if (workspace && ((uintptr_t)workspace & 255)) return fail(MSCG_E_ARG, "workspace must be 256-byte aligned");
  mscg_problem* P = new (std::nothrow) mscg_problem();
  if (!P) return fail(MSCG_E_NOMEM, "host allocation failed");
  P->g = *grid;
  if (P->g.dim == 2) P->g.n[2] = 1;
  for (int a = 0; a < 3; ++a)
    if (!(P->g.length[a] > 0.0)) P->g.length[a] = 1.0;
  P->o = o;
  P->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&P->device) != hipSuccess) { delete P; return fail(MSCG_E_DEVICE, "hipGetDevice failed"); }
  P->ws_bytes = plan.bytes;
  if (workspace) {
    P->ws = (char*)workspace;
    P->owns_ws = false;
  } else {
    if (hipMalloc(&P->ws, plan.bytes) != hipSuccess) { delete P; return fail(MSCG_E_NOMEM, "hipMalloc of %zu bytes failed", plan.bytes); }
    P->owns_ws = true;
  }
  if (hipHostMalloc(&P->hsc, sizeof(Scal)) != hipSuccess || hipHostMalloc(&P->hflags, 64) != hipSuccess ||
      hipHostMalloc(&P->hcount, 2 * MSCG_MAX_LEVELS * sizeof(long long)) != hipSuccess) {
    if (P->owns_ws) (void)hipFree(P->ws);
    delete P;
    return fail(MSCG_E_NOMEM, "pinned host allocation failed");
  }
  P->nlev = plan.nlev;
  rc = carve(P, plan);
  if (rc) { mscg_destroy_problem(P); return rc; }
  const int sn = small_n();
  P->ks = P->nlev;  // no small level
  // the one-workgroup solvers smooth by red-black SGS only and run an inner
  // PCG (with non-integer factors the generic one takes the level)
  if (P->o.splitting == MSCG_SPLIT_SGS && P->o.cycle == MSCG_CYCLE_RECURSIVE)
    for (int l = 1; l < P->nlev - 1; ++l)
      if (P->lev[l].n <= sn) { P->ks = l; break; }
  for (int l = 0; l < P->nlev; ++l) {
    LevelH& L = P->lev[l];
    L.hx = P->g.length[0] / L.nx;
    L.hy = P->g.length[1] / L.ny;
    L.hz = P->g.dim == 3 ? P->g.length[2] / L.nz : 1.0;
    if (l + 1 < P->nlev) {
      L.sx = L.nx / plan.lv[l + 1].n3[0];
      L.sy = L.ny / plan.lv[l + 1].n3[1];
      L.sz = L.nz / plan.lv[l + 1].n3[2];
    } else {
      L.sx = L.sy = L.sz = 1;
    }
  }
  P->ready = false;
  {
    const char* e = getenv("MSCG_UNTILED");
    P->tiled = !(e && e[0] == '1');
    const char* fd = getenv("MSCG_FUSED_DOT");
    P->fuse_dot = !(fd && fd[0] == '0');
    const char* ff = getenv("MSCG_FUSED_FINISH");
    P->fuse_finish = !(ff && ff[0] == '0');
    const char* sy = getenv("MSCG_SYM_COARSE");
    P->sym_coarse = !(sy && sy[0] == '0');
    const char* t = getenv("MSCG_TILE_SHAPE");
    P->tile_shape = t ? atoi(t) : -1;
    const char* v = getenv("MSCG_SMALL_VARIANT");
    P->small_variant = v ? atoi(v) : 0;
    const char* qa = getenv("MSCG_QUEUE_AHEAD");
    P->queue_ahead = !(qa && qa[0] == '0');
  }
  *out = P;
  return MSCG_OK;
}

int mscg_destroy_problem(mscg_problem* P) {
  if (!P) return MSCG_OK;
  for (hipEvent_t e : P->kev)
    if (e) (void)hipEventDestroy(e);
  if (P->owns_ws && P->ws) (void)hipFree(P->ws);
  if (P->hsc) (void)hipHostFree(P->hsc);
  if (P->hflags) (void)hipHostFree(P->hflags);
  if (P->hcount) (void)hipHostFree(P->hcount);
  delete P;
  return MSCG_OK;
}

int mscg_set_permeability(mscg_problem* P, const double* kx, const double* ky, const double* kz) {
  g_err.clear();
  int rc = validate_problem(P);
  if (rc) return rc;
  if (!kx) return fail(MSCG_E_ARG, "kx is NULL");
  if (!ky) ky = kx;
  if (P->g.dim == 3 && !kz) kz = kx;
  LevelH& L0 = P->lev[0];
  const long long N = L0.n;
  // validate K > 0 and finite
  HIP_TRY(launch_fill<int>(P->dflags, 16, 0, P->stream));
  HIP_TRY(launch_check_positive(kx, N, P->dflags + 1, P->stream));
  HIP_TRY(launch_check_positive(ky, N, P->dflags + 1, P->stream));
  if (P->g.dim == 3) HIP_TRY(launch_check_positive(kz, N, P->dflags + 1, P->stream));
  HIP_TRY(hipMemcpyAsync(P->hflags, P->dflags, 16, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (P->hflags[1]) return fail(MSCG_E_ARG, "permeability must be finite and > 0 everywhere");
  // face transmissibilities of level 0
  FaceTArgs fa{};
  fa.dim = P->g.dim; fa.nx = L0.nx; fa.ny = L0.ny; fa.nz = L0.nz;
  fa.ax = L0.hy * L0.hz / L0.hx;
  fa.ay = L0.hx * L0.hz / L0.hy;
  fa.az = L0.hx * L0.hy / L0.hz;
  fa.kx = kx; fa.ky = ky; fa.kz = kz;
  for (int f = 0; f < 6; ++f) fa.bc_type[f] = P->g.bc_type[f];
  if (P->g.dim == 2) { fa.bc_type[4] = fa.bc_type[5] = 0; }
  fa.tx = L0.tx; fa.ty = L0.ty; fa.tz = L0.tz;
  HIP_TRY(launch_face_T(fa, P->stream));
  // coarse graining level by level
  for (int l = 1; l < P->nlev; ++l) {
    LevelH& F = P->lev[l - 1];
    LevelH& C = P->lev[l];
    const double* fsrc[3] = {F.tx, F.ty, F.tz};
    double* cdst[3] = {C.tx, C.ty, C.tz};
    for (int ax = 0; ax < P->g.dim; ++ax) {
      CoarsenArgs ca{};
      ca.axis = ax;
      ca.frac = P->o.frac_scale != 0.0 ? 1 : 0;
      ca.fd[0] = F.nx; ca.fd[1] = F.ny; ca.fd[2] = F.nz;
      ca.cd[0] = C.nx; ca.cd[1] = C.ny; ca.cd[2] = C.nz;
      ca.s[0] = F.sx; ca.s[1] = F.sy; ca.s[2] = F.sz;
      ca.f = fsrc[ax];
      ca.c = cdst[ax];
      HIP_TRY(launch_coarsen(ca, P->stream));
    }
  }
  if (mixed(P)) {
    for (int l = 0; l < P->nlev; ++l) {
      LevelH& L = P->lev[l];
      HIP_TRY(launch_to_f32(L.tx, L.tx32, (long long)(L.nx + 1) * L.ny * L.nz, P->stream));
      HIP_TRY(launch_to_f32(L.ty, L.ty32, (long long)L.nx * (L.ny + 1) * L.nz, P->stream));
      if (P->g.dim == 3) HIP_TRY(launch_to_f32(L.tz, L.tz32, (long long)L.nx * L.ny * (L.nz + 1), P->stream));
    }
  }
  // coarsest factorisation
  HIP_TRY(launch_coarse_factor(lv64(P, P->nlev - 1), P->Atmp, P->Lrows, P->Ainv, P->dflags, P->stream));
  // the lower triangle of the inverse in 16 x 16 tiles for the one-workgroup
  // solvers, in the factorisation's scratch (free from here on)
  P->Asym = nullptr;
  {
    const int nc = P->ncoarse, nt = (nc + 15) / 16;
    if (P->sym_coarse && nc <= 256 && (long long)nt * (nt + 1) / 2 * 256 <= (long long)nc * nc) {
      HIP_TRY(launch_pack_sym(P->Ainv, nc, nt, P->Atmp, P->stream));
      P->Asym = P->Atmp;
      P->ntile = nt;
    }
  }
  HIP_TRY(hipMemcpyAsync(P->hflags, P->dflags, 16, hipMemcpyDeviceToHost, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  if (P->hflags[0]) {
    P->ready = false;
    return fail(MSCG_E_SINGULAR, "coarsest operator is not positive definite (no Dirichlet boundary?)");
  }
  P->ready = true;
  return MSCG_OK;
}

static int solve_impl(mscg_problem* P, const double* f, double* p, double rel_tol, int use_x0, mscg_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  LevelH& L0 = P->lev[0];
  const int N = L0.n;
  const int nb = reduce_blocks(N);
  for (int l = 0; l < MSCG_MAX_LEVELS; ++l) { P->iters[l] = 0; P->calls[l] = 0; }
  P->status = MSCG_OK;
  P->tol_scale = 1.0;
  HIP_TRY(launch_fill<long long>(P->dcount, 2 * MSCG_MAX_LEVELS, 0, P->stream));
  HIP_TRY(launch_fill<int>(P->dflags + 2, 1, 0, P->stream));
  int rc = clear_scalars(P);
  if (rc) return rc;
  // right-hand side and tolerance
  RhsArgs ra{};
  ra.dim = P->g.dim; ra.nx = L0.nx; ra.ny = L0.ny; ra.nz = L0.nz; ra.n = N;
  ra.vol = L0.hx * L0.hy * L0.hz;
  ra.f = f; ra.tx = L0.tx; ra.ty = L0.ty; ra.tz = L0.tz;
  for (int q = 0; q < 6; ++q) { ra.bc_type[q] = P->g.bc_type[q]; ra.bc_value[q] = P->g.bc_value[q]; }
  if (P->g.dim == 2) { ra.bc_type[4] = ra.bc_type[5] = 0; }
  ra.b = P->b;
  HIP_TRY(launch_rhs(ra, P->stream));
  HIP_TRY(launch_dot<double>(P->b, P->b, N, P->part, nb, P->stream));
  HIP_TRY(launch_finish(P->part, nb, L0.sc, kOpBB, P->stream));
  rc = read_scal(P, 0);
  if (rc) return rc;
  const double bb = P->hsc->bb;
  P->eps2 = rel_tol * rel_tol * bb / N;
  // initial guess
  bool only_x = P->g.bc_type[0] == MSCG_DIRICHLET && P->g.bc_type[1] == MSCG_DIRICHLET;
  for (int q = 2; q < 2 * P->g.dim; ++q) if (P->g.bc_type[q] == MSCG_DIRICHLET) only_x = false;
  if (!use_x0)
    HIP_TRY(launch_init_x(p, N, L0.nx, L0.hx, P->g.length[0], P->g.bc_value[0], P->g.bc_value[1], only_x ? 1 : 0,
                          P->stream));
  int outer = 0;
  if (P->nlev == 1) {
    HIP_TRY(launch_coarse_solve<double>(P->Ainv, P->b, p, N, P->stream));
    P->calls[0]++;
  } else {
    rc = set_tol(P, 0, level_tol(P, 0));
    if (rc) return rc;
    HIP_TRY(launch_residual<double>(lv64(P, 0), P->b, p, L0.r, P->part, nb, P->stream));
    HIP_TRY(launch_finish(P->part, nb, L0.sc, kOpEntry, P->stream));
    rc = read_scal(P, 0);
    if (rc) return rc;
    P->calls[0]++;
    if (!P->hsc->converged) {
      if (mixed(P)) P->tol_scale = P->hsc->rr > 0.0 ? 1.0 / P->hsc->rr : 1.0;
      rc = cg_loop<double>(P, 0, lv64(P, 0), p, L0.r, L0.z, L0.p, L0.p2, L0.q, P->o.max_outer_iters);
      if (rc) return rc;
    }
    outer = (int)P->iters[0];
  }
  // true residual in FP64
  HIP_TRY(launch_residual<double>(lv64(P, 0), P->b, p, L0.z, P->part, nb, P->stream));
  HIP_TRY(launch_finish(P->part, nb, L0.sc, kOpBB, P->stream));
  HIP_TRY(hipMemcpyAsync(P->hcount, P->dcount, 2 * MSCG_MAX_LEVELS * sizeof(long long), hipMemcpyDeviceToHost,
                         P->stream));
  HIP_TRY(hipMemcpyAsync(P->hflags, P->dflags, 16, hipMemcpyDeviceToHost, P->stream));
  rc = read_scal(P, 0);
  if (rc) return rc;
  const double rt = P->hsc->bb;
  auto t1 = std::chrono::steady_clock::now();
  if (P->ktime) {
    for (size_t q = 0; q + 1 < P->kev_used; q += 2) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, P->kev[q], P->kev[q + 1]));
      P->ktime_ms += ms;
      P->klaunches += 1;
    }
    P->kev_used = 0;
    if (P->ks == P->nlev - 2) {
      P->kiters += P->hcount[P->ks];
      P->kflops += small_level_flops(P) * (double)P->hcount[P->ks];
    }
  }
  int status = P->status;
  if (P->hflags[2]) {
    status = MSCG_E_BREAKDOWN;
    fail(MSCG_E_BREAKDOWN, "non-finite reduction in the one-workgroup inner solver (level >= %d)", P->ks);
  }
  const bool converged_rec = P->nlev == 1 || P->hsc->converged;
  if (status == MSCG_OK && !converged_rec) status = MSCG_NOT_CONVERGED;
  if (st) {
    memset(st, 0, sizeof(*st));
    st->status = status;
    st->outer_iters = outer;
    st->n_levels = P->nlev;
    for (int l = 0; l < P->nlev; ++l) {
      st->level_n[l][0] = P->lev[l].nx; st->level_n[l][1] = P->lev[l].ny; st->level_n[l][2] = P->lev[l].nz;
      st->level_iters[l] = P->iters[l] + P->hcount[l];
      st->level_calls[l] = P->calls[l] + P->hcount[MSCG_MAX_LEVELS + l];
    }
    st->b_norm = std::sqrt(bb);
    st->rel_residual_true = bb > 0.0 ? std::sqrt(rt / bb) : std::sqrt(rt);
    st->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  return status;
}

int mscg_solve(mscg_problem* P, const double* f, double* p, double rel_tol, int use_x0, mscg_stats* st) {
  g_err.clear();
  int rc = validate_problem(P);
  if (rc) return rc;
  if (!P->ready) return fail(MSCG_E_STATE, "mscg_set_permeability must succeed before mscg_solve");
  if (!f || !p) return fail(MSCG_E_ARG, "f and p must be device pointers");
  if (!(rel_tol > 0.0) || !(rel_tol < 1.0)) return fail(MSCG_E_ARG, "rel_tol must be in (0, 1)");
  return solve_impl(P, f, p, rel_tol, use_x0, st);
}

int mscg_solve_batch(mscg_problem* const* probs, const double* const* f, double* const* p, const double* rel_tol,
                     int count, mscg_stats* stats) {
  g_err.clear();
  if (count < 0 || (count > 0 && (!probs || !f || !p || !rel_tol))) return fail(MSCG_E_ARG, "bad batch arguments");
  for (int i = 0; i < count; ++i) {
    if (!probs[i]) return fail(MSCG_E_ARG, "probs[%d] is NULL", i);
    for (int j = 0; j < i; ++j)
      if (probs[j] == probs[i]) return fail(MSCG_E_ARG, "probs[%d] and probs[%d] are the same problem", j, i);
  }
  // one host thread per problem: each drives its problem's own stream, so the
  // solves' kernels overlap on the device
  std::vector<int> rcs(count, MSCG_OK);
  std::vector<std::string> errs(count);
  std::vector<std::thread> th;
  th.reserve(count);
  int dev = 0;
  (void)hipGetDevice(&dev);
  for (int i = 0; i < count; ++i)
    th.emplace_back([&, i]() {
      (void)hipSetDevice(dev);
      rcs[i] = mscg_solve(probs[i], f[i], p[i], rel_tol[i], 0, stats ? &stats[i] : nullptr);
      if (rcs[i] < 0) errs[i] = g_err;
    });
  for (auto& t : th) t.join();
  int worst = MSCG_OK;
  for (int i = 0; i < count; ++i) {
    const int rc = rcs[i];
    if (rc < 0 && (worst >= 0 || rc < worst)) { worst = rc; g_err = errs[i]; }
    else if (rc > 0 && worst == MSCG_OK) worst = rc;
  }
  return worst;
}

int mscg_level_info(const mscg_problem* P, int level, int dims[3]) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level >= P->nlev) return fail(MSCG_E_ARG, "level %d out of range (%d levels)", level, P->nlev);
  if (dims) { dims[0] = P->lev[level].nx; dims[1] = P->lev[level].ny; dims[2] = P->lev[level].nz; }
  return P->nlev;
}

int mscg_get_transmissibility(const mscg_problem* P, int level, double* tx, double* ty, double* tz) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level >= P->nlev) return fail(MSCG_E_ARG, "level out of range");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  const LevelH& L = P->lev[level];
  HIP_TRY(launch_copy<double>(L.tx, tx, (long long)(L.nx + 1) * L.ny * L.nz, P->stream));
  HIP_TRY(launch_copy<double>(L.ty, ty, (long long)L.nx * (L.ny + 1) * L.nz, P->stream));
  if (P->g.dim == 3 && tz) HIP_TRY(launch_copy<double>(L.tz, tz, (long long)L.nx * L.ny * (L.nz + 1), P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

int mscg_apply_operator(mscg_problem* P, int level, const double* x, double* y) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level >= P->nlev) return fail(MSCG_E_ARG, "level out of range");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  HIP_TRY(launch_spmv<double>(lv64(P, level), x, y, nullptr, reduce_blocks(P->lev[level].n), P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

int mscg_apply_smoother(mscg_problem* P, int level, const double* r, double* x, int steps) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level >= P->nlev) return fail(MSCG_E_ARG, "level out of range");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  if (steps < 1) return fail(MSCG_E_ARG, "steps must be >= 1");
  // steps forward+backward pairs (R,B | B,R) with repeated colours elided: R,B,R,...,R
  for (int h = 0; h <= 2 * steps; ++h) HIP_TRY(launch_gs_half<double>(lv64(P, level), r, x, h & 1, 0, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

int mscg_restrict_residual(mscg_problem* P, int level, const double* r, const double* x, double* g) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level + 1 >= P->nlev) return fail(MSCG_E_ARG, "level must have a coarser level");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  if (P->o.frac_scale != 0.0) return fail(MSCG_E_ARG, "not available on hierarchies with non-integer factors");
  HIP_TRY(launch_restrict<double>(lv64(P, level), xfer(P, level), r, x, g, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

int mscg_prolong_add(mscg_problem* P, int level, const double* y, double* x) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (level < 0 || level + 1 >= P->nlev) return fail(MSCG_E_ARG, "level must have a coarser level");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  HIP_TRY(launch_prolong<double>(lv64(P, level), xfer(P, level), y, x, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return MSCG_OK;
}

int mscg_apply_preconditioner(mscg_problem* P, const double* r, double* z, double eps2) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  if (mixed(P)) return fail(MSCG_E_ARG, "mscg_apply_preconditioner needs an FP64 problem");
  if (P->nlev < 2) return fail(MSCG_E_ARG, "a preconditioner needs at least two levels");
  for (int l = 0; l < MSCG_MAX_LEVELS; ++l) { P->iters[l] = 0; P->calls[l] = 0; }
  P->eps2 = eps2;
  P->tol_scale = 1.0;
  P->status = MSCG_OK;
  LevelH& L0 = P->lev[0];
  HIP_TRY(launch_copy<double>(r, L0.r, L0.n, P->stream));
  HIP_TRY(launch_fill<long long>(P->dcount, 2 * MSCG_MAX_LEVELS, 0, P->stream));
  int rc = clear_scalars(P);
  if (rc) return rc;
  void* zres = nullptr;
  rc = apply_prec(P, 0, &zres, nullptr);
  if (rc) return rc;
  HIP_TRY(launch_copy<double>(static_cast<const double*>(zres), z, L0.n, P->stream));
  HIP_TRY(hipStreamSynchronize(P->stream));
  return P->status;
}

int mscg_enable_kernel_timing(mscg_problem* P, int on) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (P->ks != P->nlev - 2 || P->nlev < 3 || P->g.dim != 2)
    return fail(MSCG_E_ARG, "no one-workgroup solver of a 2-D last inner level in this hierarchy");
  P->ktime = on != 0;
  P->kev_used = 0;
  P->ktime_ms = P->kflops = 0.0;
  P->klaunches = P->kiters = 0;
  return MSCG_OK;
}

int mscg_small_level_timing(const mscg_problem* P, double* total_ms, long long* launches, long long* iterations,
                            double* flops) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (total_ms) *total_ms = P->ktime_ms;
  if (launches) *launches = P->klaunches;
  if (iterations) *iterations = P->kiters;
  if (flops) *flops = P->kflops;
  return MSCG_OK;
}

int mscg_time_kernel(mscg_problem* P, int kernel, int level, int reps, double* avg_us, double* alg_bytes) {
  g_err.clear();
  if (!P) return fail(MSCG_E_ARG, "problem is NULL");
  if (!P->ready) return fail(MSCG_E_STATE, "permeability not set");
  if (level < 0 || level >= P->nlev) return fail(MSCG_E_ARG, "level out of range");
  if (reps < 1) return fail(MSCG_E_ARG, "reps must be >= 1");
  if ((kernel == MSCG_KERNEL_RESTRICT || kernel == MSCG_KERNEL_PROLONG || kernel == MSCG_KERNEL_SMOOTH_PRE ||
       kernel == MSCG_KERNEL_SMOOTH_POST) && level + 1 >= P->nlev)
    return fail(MSCG_E_ARG, "transfer and smoothing kernels need a coarser level");
  if (P->o.frac_scale != 0.0 && (kernel == MSCG_KERNEL_RESTRICT || kernel == MSCG_KERNEL_SMOOTH_POST))
    return fail(MSCG_E_ARG, "kernel not timed on hierarchies with non-integer factors");
  if ((kernel == MSCG_KERNEL_SMOOTH_PRE || kernel == MSCG_KERNEL_SMOOTH_POST) &&
      !smooth_tile_supported(P->lev[level].nz, P->g.dim == 3, P->o.smooth_steps))
    return fail(MSCG_E_ARG, "level %d has no tiled smoother", level);
  const bool fp32 = mixed(P) && level > 0;
  if (fp32 && kernel != MSCG_KERNEL_SMOOTH_HALF) return fail(MSCG_E_ARG, "FP32 timing covers the smoother only");
  if (mixed(P) && (kernel == MSCG_KERNEL_SMOOTH_PRE || kernel == MSCG_KERNEL_SMOOTH_POST))
    return fail(MSCG_E_ARG, "tiled smoother timing needs an FP64 problem");
  LevelH& L = P->lev[level];
  const double w = fp32 ? 4.0 : 8.0;
  const double n = L.n;
  const double faces = (double)(L.nx + 1) * L.ny * L.nz + (double)L.nx * (L.ny + 1) * L.nz +
                       (P->g.dim == 3 ? (double)L.nx * L.ny * (L.nz + 1) : 0.0);
  double bytes = 0.0;
  const int nb = reduce_blocks(L.n);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto launch = [&]() -> hipError_t {
    switch (kernel) {
      case MSCG_KERNEL_SMOOTH_HALF:
        if (fp32 || (mixed(P) && level == 0)) return launch_gs_half<float>(lv32(P, level), level == 0 ? L.r32 : L.r32, L.z32, 0, 0, P->stream);
        return launch_gs_half<double>(lv64(P, level), L.r, L.z, 0, 0, P->stream);
      case MSCG_KERNEL_SPMV:
        return launch_spmv<double>(lv64(P, level), L.p, L.q, P->part, nb, P->stream);
      case MSCG_KERNEL_RESTRICT:
        return launch_restrict<double>(lv64(P, level), xfer(P, level), L.r, L.z, P->lev[level + 1].r, P->stream);
      case MSCG_KERNEL_PROLONG:
        return launch_prolong<double>(lv64(P, level), xfer(P, level), P->lev[level + 1].x, L.z, P->stream);
      case MSCG_KERNEL_CG_UPDATE:
        return launch_cg_update<double>(L.x, L.r, L.p, L.q, L.n, L.sc, P->part, nb, P->stream);
      case MSCG_KERNEL_SMOOTH_PRE:
        return launch_smooth_tile<double>(lv64(P, level), nullptr, L.r, nullptr, nullptr, L.z, P->o.smooth_steps,
                                          P->tile_shape, P->stream);
      case MSCG_KERNEL_SMOOTH_POST: {
        const Xfer X = xfer(P, level);
        return launch_smooth_tile<double>(lv64(P, level), &X, L.r, L.z, P->lev[level + 1].x, L.w,
                                          P->o.smooth_steps, P->tile_shape, P->stream);
      }
      default:
        return hipErrorInvalidValue;
    }
  };
  const double ws = (mixed(P) && level == 0 && kernel == MSCG_KERNEL_SMOOTH_HALF) ? 4.0 : w;
  switch (kernel) {
    case MSCG_KERNEL_SMOOTH_HALF: bytes = ws * (faces + n + 0.5 * n + 0.5 * n); break;  // T, x, r (one colour), x (one colour)
    case MSCG_KERNEL_SPMV: bytes = w * (faces + 2.0 * n); break;                       // T, p in; q out
    case MSCG_KERNEL_RESTRICT: bytes = w * (faces + 2.0 * n + (double)P->lev[level + 1].n); break;
    case MSCG_KERNEL_PROLONG: bytes = w * (2.0 * n + (double)P->lev[level + 1].n); break;
    case MSCG_KERNEL_CG_UPDATE: bytes = w * 6.0 * n; break;                            // x, r, p, q in; x, r out
    case MSCG_KERNEL_SMOOTH_PRE: bytes = w * (faces + 2.0 * n); break;                  // T, r in; z out
    case MSCG_KERNEL_SMOOTH_POST: bytes = w * (faces + 3.0 * n + (double)P->lev[level + 1].n); break;  // T, r, z, y; w
    default: return fail(MSCG_E_ARG, "unknown kernel id %d", kernel);
  }
  HIP_TRY(launch());  // warm
  HIP_TRY(hipEventRecord(e0, P->stream));
  for (int i = 0; i < reps; ++i) HIP_TRY(launch());
  HIP_TRY(hipEventRecord(e1, P->stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (avg_us) *avg_us = 1000.0 * ms / reps;
  if (alg_bytes) *alg_bytes = bytes;
  return MSCG_OK;
}

}  // extern "C"
