// mscg_small2d.hip -- one-workgroup solver for a 2-D last inner level, laid
// out by colour.
//
// The inner PCG of the level just above the coarsest grid runs all its
// iterations in one launch (Section 2.3: the coarse inverse is applied by the
// same PCG; Section 3: the level stops at |r|^2 / N_k < f^k eps^2).
//
// Cells are numbered by colour slot, as in the grid-wide half sweep: slot q of
// colour cl is row j = q / H, column i = 2 (q mod H) + ((j + cl) & 1),
// H = ceil(nx / 2).  Thread t owns slots t and t + 1024 of both colours, so
// every thread updates two cells in each half sweep.  The vectors that
// neighbours read (the smoother iterate z, the direction p) and the residual
// handed to the restriction sit in LDS split by colour, each colour padded by
// H zero slots on both sides: the four neighbours of slot q (all of the other
// colour) are then at q + p - 1, q + p, q - H and q + H with p = (j + cl) & 1,
// in bounds for every slot and zero outside the grid, so the sweep needs no
// clamps or branches.  Slots past the grid (ragged rows, q >= S) are owned
// as ghost cells with zero coefficients, zero right-hand side and unit
// diagonal: they stay zero.
//
// Per owned cell the thread keeps its four neighbour coefficients (zero
// across the boundary), diagonal and its inverse, residual r and iterate x in
// registers.  The
// restriction E^T runs as an x pass over (fine row, coarse column) and a y
// pass over (coarse row, coarse column), each output with its footprint
// weights tabulated in LDS once per launch; the prolongation E reads the
// per-column and per-row extension weights from LDS tables.  The coarsest
// solve is the dense FP64 inverse applied by the whole workgroup, each lane
// reading two adjacent entries of a row at once, eight rows in flight.  Reductions: DPP within each wave, then the 16
// wave sums in order, so every result is independent of scheduling.
#include <hip/hip_runtime.h>

#include "mscg_kernels.h"

#ifndef MSCG_S2D_THREADS
#define MSCG_S2D_THREADS 1024
#endif

namespace mscg {

namespace {

constexpr int kThreads2 = MSCG_S2D_THREADS;
constexpr int kSlots = 2048;                // slots per colour a launch can own
constexpr int kV = kSlots / kThreads2;      // slots per colour per thread
constexpr int kU = 2 * kV;                  // owned cells per thread
constexpr int kFoot = 12;              // >= footprint of one coarse cell along an axis (linear, s <= 4)
constexpr int kBatch = 8;              // inverse entries loaded per batch

struct Small2dArgs {
  int nx, ny, H, S;             // level dims, slots per colour row, slots per colour
  int sx, sy, cnx, cny, nc;     // factors and dims of the coarsest level
  int interp, m, max_inner;
  double tol, rel_floor2;
  const void *tx, *ty, *rhs;
  void* x;
  const double* Ainv;
  long long *iters, *calls;
  int level;
  int* status;
  const int* gate;
  int pitch;                    // entries per colour in the padded arrays: kSlots + 2 H
  int off_z, off_p, off_res, off_tx1, off_g, off_y, off_part, off_wx, off_wy, off_ci, off_cw, off_ri, off_rw;
};

template <typename R>
__global__ void __launch_bounds__(kThreads2, 1) k_small_2d(Small2dArgs a) {
  if (a.gate && *a.gate) return;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ __align__(16) double sm[2][kThreads2 / kWave];
  R* z = reinterpret_cast<R*>(lds + a.off_z);
  R* pv = reinterpret_cast<R*>(lds + a.off_p);
  R* res = reinterpret_cast<R*>(lds + a.off_res);
  R* tx1 = reinterpret_cast<R*>(lds + a.off_tx1);
  double* g = reinterpret_cast<double*>(lds + a.off_g);
  double* y = reinterpret_cast<double*>(lds + a.off_y);
  double* part = reinterpret_cast<double*>(lds + a.off_part);
  R* wx = reinterpret_cast<R*>(lds + a.off_wx);   // [I][kFoot] x-pass weights from fine column lo(I) + b
  R* wy = reinterpret_cast<R*>(lds + a.off_wy);   // [J][kFoot] y-pass weights from fine row lo(J) + b
  int* ci = reinterpret_cast<int*>(lds + a.off_ci);  // fine column i: I0 | I1 << 16
  R* cw = reinterpret_cast<R*>(lds + a.off_cw);      // fine column i: w0, w1
  int* ri = reinterpret_cast<int*>(lds + a.off_ri);
  R* rw = reinterpret_cast<R*>(lds + a.off_rw);
  const R* TX = static_cast<const R*>(a.tx);
  const R* TY = static_cast<const R*>(a.ty);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int nx = a.nx, ny = a.ny, H = a.H, S = a.S, pitch = a.pitch;
  const int ncx = a.cnx, ncy = a.cny, nc = a.nc;

  int red = 0;  // alternating partial-sum buffer: one barrier per reduction
  auto block_sum = [&](double v) {
    v = wave_sum_dpp(v);
    if (lane == kWave - 1) sm[red][wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kThreads2 / kWave; ++w) s += sm[red][w];
    red ^= 1;
    return s;
  };
  // colour-split padded address of fine cell (i, j)
  auto at = [&](int i, int j) { return ((i + j) & 1) * pitch + H + j * H + (i >> 1); };

  // ---- set-up: clear the padded arrays, tabulate the transfer weights
  for (int e = tid; e < 2 * pitch; e += kThreads2) {
    z[e] = R(0);
    pv[e] = R(0);
    res[e] = R(0);
  }
  for (int i = tid; i < nx; i += kThreads2) {
    int I0, I1;
    R w0, w1;
    ext_weights<R>(i, a.sx, ncx, a.interp, I0, w0, I1, w1);
    ci[i] = I0 | (I1 << 16);
    cw[2 * i] = w0;
    cw[2 * i + 1] = w1;
  }
  for (int j = tid; j < ny; j += kThreads2) {
    int J0, J1;
    R w0, w1;
    ext_weights<R>(j, a.sy, ncy, a.interp, J0, w0, J1, w1);
    ri[j] = J0 | (J1 << 16);
    rw[2 * j] = w0;
    rw[2 * j + 1] = w1;
  }
  for (int e = tid; e < ncx * kFoot; e += kThreads2) {
    const int I = e / kFoot, b = e - I * kFoot;
    int lo, hi;
    ext_support(I, a.sx, nx, a.interp, lo, hi);
    wx[e] = lo + b <= hi ? ext_weight_of<R>(lo + b, I, a.sx, ncx, a.interp) : R(0);
  }
  for (int e = tid; e < ncy * kFoot; e += kThreads2) {
    const int J = e / kFoot, b = e - J * kFoot;
    int lo, hi;
    ext_support(J, a.sy, ny, a.interp, lo, hi);
    wy[e] = lo + b <= hi ? ext_weight_of<R>(lo + b, J, a.sy, ncy, a.interp) : R(0);
  }

  // ---- owned cells: u = 2 cl + v is slot q_v = tid + v kThreads2 of colour cl
  int jv[kV], mv[kV];
#pragma unroll
  for (int v = 0; v < kV; ++v) {
    const int q = tid + v * kThreads2;
    jv[v] = q / H;
    mv[v] = q - jv[v] * H;
  }
  R ccw[kU], cce[kU], ccs[kU], ccn[kU], dg[kU], di[kU], r[kU], x[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int cl = u / kV, v = u % kV;
    const int j = jv[v], i = 2 * mv[v] + ((j + cl) & 1);
    const bool ok = tid + v * kThreads2 < S && i < nx;
    const int ii = ok ? i : 0, jj = ok ? j : 0;
    const int fx = ii + (nx + 1) * jj, fy = ii + nx * jj;
    const R tw = TX[fx], te = TX[fx + 1], ts = TY[fy], tn = TY[fy + nx];
    dg[u] = ok ? tw + te + ts + tn : R(1);
    di[u] = R(1) / dg[u];
    ccw[u] = ok && ii > 0 ? tw : R(0);
    cce[u] = ok && ii < nx - 1 ? te : R(0);
    ccs[u] = ok && jj > 0 ? ts : R(0);
    ccn[u] = ok && jj < ny - 1 ? tn : R(0);
    r[u] = ok ? static_cast<const R*>(a.rhs)[ii + nx * jj] : R(0);
    x[u] = R(0);
  }
  // own address of cell u and the base of its neighbours in the other colour
  auto own_at = [&](int u) { return (u / kV) * pitch + H + tid + (u % kV) * kThreads2; };
  auto nb_at = [&](int u) { return (1 - u / kV) * pitch + H + tid + (u % kV) * kThreads2; };
  auto par = [&](int u) { return (jv[u % kV] + u / kV) & 1; };
  auto offsum = [&](const R* vec, int u) -> R {
    const int b = nb_at(u), p = par(u);
    return ccw[u] * vec[b + p - 1] + cce[u] * vec[b + p] + ccs[u] * vec[b - H] + ccn[u] * vec[b + H];
  };
  // one red-black half sweep (Section 3 splitting) of colour CL
  auto half_sweep = [&](int cl, bool first) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (u / kV != cl) continue;
      z[own_at(u)] = first ? r[u] * di[u] : (r[u] + offsum(z, u)) * di[u];
    }
    __syncthreads();
  };
  auto sweeps = [&](bool from_zero) {
    for (int h = 0; h <= 2 * a.m; ++h) {
      if (h & 1)
        half_sweep(1, false);
      else
        half_sweep(0, from_zero && h == 0);
    }
  };

  double rr = 0.0;
#pragma unroll
  for (int u = 0; u < kU; ++u) rr += (double)r[u] * (double)r[u];
  rr = block_sum(rr);  // its barrier also orders the set-up writes before their use
  double tol = a.tol;
  if (a.rel_floor2 > 0.0 && a.rel_floor2 * rr > tol) tol = a.rel_floor2 * rr;
  long long iters = 0, coarse_calls = 0;
  int status = 0;
  double rho_old = 0.0;
  const int half_nc = nc / 2;  // nc is even (checked at launch)
  const int groups = kThreads2 / half_nc;
  const int per = (nc + groups - 1) / groups;

  if (!(rr < tol)) {
    for (int it = 0; it < a.max_inner; ++it) {
      // -- pre-smoothing from zero, then the residual for the restriction
      sweeps(true);
#pragma unroll
      for (int u = 0; u < kU; ++u) res[own_at(u)] = r[u] - (dg[u] * z[own_at(u)] - offsum(z, u));
      __syncthreads();
      // -- g = E^T res: x pass over (fine row, I), y pass over (J, I)
      for (int e = tid; e < ny * ncx; e += kThreads2) {
        const int row = e / ncx, I = e - row * ncx;
        int lo, hi;
        ext_support(I, a.sx, nx, a.interp, lo, hi);
        R s = R(0);
#pragma unroll
        for (int b = 0; b < kFoot; ++b) {
          const int i = min(lo + b, hi);
          s += wx[I * kFoot + b] * res[at(i, row)];
        }
        tx1[e] = s;
      }
      __syncthreads();
      for (int e = tid; e < nc; e += kThreads2) {
        const int J = e / ncx, I = e - J * ncx;
        int lo, hi;
        ext_support(J, a.sy, ny, a.interp, lo, hi);
        R s = R(0);
#pragma unroll
        for (int b = 0; b < kFoot; ++b) {
          const int j = min(lo + b, hi);
          s += wy[J * kFoot + b] * tx1[j * ncx + I];
        }
        g[e] = (double)s;
      }
      __syncthreads();
      // -- coarsest: y = A^-1 g.  Thread (group, pair) sums two adjacent outputs over
      // its column range in order, reading 16 bytes per row; the group partials
      // are then summed in group order.
      if (tid < groups * half_nc) {
        const int ip = tid % half_nc, grp = tid / half_nc;
        const int j0 = grp * per, j1 = min(j0 + per, nc);
        double s0 = 0.0, s1 = 0.0;
        for (int jb = j0; jb < j1; jb += kBatch) {
          double2 av[kBatch];
#pragma unroll
          for (int t = 0; t < kBatch; ++t)
            av[t] = jb + t < j1 ? *reinterpret_cast<const double2*>(a.Ainv + (long long)(jb + t) * nc + 2 * ip)
                              : make_double2(0.0, 0.0);
#pragma unroll
          for (int t = 0; t < kBatch; ++t)
            if (jb + t < j1) {
              s0 += av[t].x * g[jb + t];
              s1 += av[t].y * g[jb + t];
            }
        }
        part[grp * nc + 2 * ip] = s0;
        part[grp * nc + 2 * ip + 1] = s1;
      }
      __syncthreads();
      for (int i = tid; i < nc; i += kThreads2) {
        double s = 0.0;
        for (int grp = 0; grp < groups; ++grp) s += part[grp * nc + i];
        y[i] = s;
      }
      coarse_calls++;
      __syncthreads();
      // -- prolongation z += E y on owned cells
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int v = u % kV, j = jv[v], i = 2 * mv[v] + ((j + u / kV) & 1);
        if (tid + v * kThreads2 >= S || i >= nx) continue;
        const int pi = ci[i], pj = ri[j];
        const int I0 = pi & 0xffff, I1 = pi >> 16, b0 = ncx * (pj & 0xffff), b1 = ncx * (pj >> 16);
        const R wi0 = cw[2 * i], wi1 = cw[2 * i + 1], wj0 = rw[2 * j], wj1 = rw[2 * j + 1];
        z[own_at(u)] += wj0 * (wi0 * (R)y[I0 + b0] + wi1 * (R)y[I1 + b0]) +
                        wj1 * (wi0 * (R)y[I0 + b1] + wi1 * (R)y[I1 + b1]);
      }
      __syncthreads();
      // -- post-smoothing
      sweeps(false);
      // -- CG step (Templates Figure 2.5)
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) acc += (double)r[u] * (double)z[own_at(u)];
      const double rho = block_sum(acc);
      if (!(rho == rho) || rho == INFINITY) { status = -4; break; }
      if (!(rho > 0.0)) break;  // no further progress in this precision: the level stops
      const R beta = it == 0 ? R(0) : (R)(rho / rho_old);
#pragma unroll
      for (int u = 0; u < kU; ++u) pv[own_at(u)] = it == 0 ? z[own_at(u)] : z[own_at(u)] + beta * pv[own_at(u)];
      __syncthreads();
      R q[kU], po[kU];
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        po[u] = pv[own_at(u)];
        q[u] = dg[u] * po[u] - offsum(pv, u);
        acc += (double)po[u] * (double)q[u];
      }
      const double pq = block_sum(acc);
      if (!(pq == pq) || pq == INFINITY) { status = -4; break; }
      if (!(pq > 0.0)) break;
      const R alpha = (R)(rho / pq);
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        x[u] += alpha * po[u];
        r[u] -= alpha * q[u];
        acc += (double)r[u] * (double)r[u];
      }
      rr = block_sum(acc);
      rho_old = rho;
      iters++;
      if (rr < tol) break;
    }
  }
  R* xo = static_cast<R*>(a.x);
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    const int v = u % kV, j = jv[v], i = 2 * mv[v] + ((j + u / kV) & 1);
    if (tid + v * kThreads2 < S && i < nx) xo[i + nx * j] = x[u];
  }
  if (tid == 0) {
    a.iters[a.level] += iters;
    a.calls[a.level] += 1;
    a.calls[a.level + 1] += coarse_calls;
    if (status) a.status[0] = status;
  }
}

}  // namespace

template <typename R>
hipError_t launch_small_2d(const SmallDesc<R>& d, hipStream_t s) {
  const int ks = d.ks;
  if (ks + 1 != d.nlev - 1) return hipErrorNotSupported;
  const Lv<R>& V = d.L[ks];
  const Xfer& X = d.X[ks];
  const int H = (V.nx + 1) / 2;
  const long long S = (long long)H * V.ny;
  if (V.tz || V.nz != 1 || S > kSlots) return hipErrorNotSupported;
  if (V.nx >= (1 << 15) || V.ny >= (1 << 15) || X.cnx >= (1 << 15) || X.cny >= (1 << 15)) return hipErrorNotSupported;
  const int nc = X.cnx * X.cny;
  if (nc > kThreads2 || nc % 2) return hipErrorNotSupported;  // the coarsest product reads output pairs
  // footprints must fit the tables: s + 2 (s / 2) + 2 fine cells (linear), s (constant)
  auto foot = [&](int f) { return f == 1 ? 1 : X.interp == 1 ? f : f + 2 * (f / 2) + 2; };
  if (foot(X.sx) > kFoot || foot(X.sy) > kFoot) return hipErrorNotSupported;
  Small2dArgs a{};
  a.nx = V.nx; a.ny = V.ny; a.H = H; a.S = (int)S;
  a.sx = X.sx; a.sy = X.sy; a.cnx = X.cnx; a.cny = X.cny; a.nc = nc;
  a.interp = X.interp; a.m = d.m; a.max_inner = d.max_inner;
  a.tol = d.tol[ks]; a.rel_floor2 = d.rel_floor2;
  a.tx = V.tx; a.ty = V.ty; a.rhs = d.r[ks]; a.x = d.x[ks];
  a.Ainv = d.Ainv;
  a.iters = d.iters; a.calls = d.calls; a.level = ks; a.status = d.status;
  a.gate = d.gate;
  a.pitch = kSlots + 2 * H;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const int o = (int)off;
    off += (bytes + 15) & ~(size_t)15;
    return o;
  };
  a.off_z = take((size_t)2 * a.pitch * sizeof(R));
  a.off_p = take((size_t)2 * a.pitch * sizeof(R));
  a.off_res = take((size_t)2 * a.pitch * sizeof(R));
  a.off_tx1 = take((size_t)V.ny * X.cnx * sizeof(R));
  a.off_g = take((size_t)nc * sizeof(double));
  a.off_y = take((size_t)nc * sizeof(double));
  a.off_part = take((size_t)2 * kThreads2 * sizeof(double));
  a.off_wx = take((size_t)X.cnx * kFoot * sizeof(R));
  a.off_wy = take((size_t)X.cny * kFoot * sizeof(R));
  a.off_ci = take((size_t)V.nx * sizeof(int));
  a.off_cw = take((size_t)2 * V.nx * sizeof(R));
  a.off_ri = take((size_t)V.ny * sizeof(int));
  a.off_rw = take((size_t)2 * V.ny * sizeof(R));
  if (off > 156 * 1024) return hipErrorNotSupported;
  static bool attr[2] = {false, false};
  const int ri = sizeof(R) == 8 ? 1 : 0;
  if (!attr[ri]) {
    hipError_t e = hipFuncSetAttribute((const void*)k_small_2d<R>, hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    if (e != hipSuccess) return e;
    attr[ri] = true;
  }
  hipLaunchKernelGGL((k_small_2d<R>), dim3(1), dim3(kThreads2), off, s, a);
  return hipGetLastError();
}

template hipError_t launch_small_2d<double>(const SmallDesc<double>&, hipStream_t);
template hipError_t launch_small_2d<float>(const SmallDesc<float>&, hipStream_t);

}  // namespace mscg
