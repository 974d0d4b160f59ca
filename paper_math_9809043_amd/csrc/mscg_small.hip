// mscg_small.hip -- one-workgroup solver for the last inner level above the
// coarsest grid, with the cells held in registers.
//
// The inner PCG of that level runs its iterations without leaving the
// device (Section 2.3: the coarse inverse is applied by the same PCG; Section 3:
// the level's criterion |r|^2 / N_k < f^k eps^2).  One workgroup of 1024
// threads; thread t owns cells t, t + 1024, ... (at most kOwn of them) and
// keeps their four (2-D) or six (3-D) neighbour coefficients, diagonal,
// inverse diagonal, residual r, iterate x and direction p in registers.
// Only what neighbours read lives in LDS: the smoother iterate z, the
// direction p and the residual passed to the restriction.  The coarsest solve
// is the dense FP64 inverse applied by the whole workgroup.
#include <hip/hip_runtime.h>

#include "mscg_kernels.h"

namespace mscg {

namespace {

constexpr int kOwn = 4;        // cells per thread (level size <= 4096)
constexpr int kThreads = 1024;

struct RegArgs {
  int dim, nx, ny, nz, n;      // the small level
  int sx, sy, sz;              // factors to the coarsest level
  int cnx, cny, cnz, nc;       // coarsest dims, cells
  int interp, m, max_inner;
  double tol;                  // absolute criterion on |r|^2
  double rel_floor2;           // mixed-precision floor relative to |rhs|^2 (0 = off)
  const void *tx, *ty, *tz;    // faces of the small level (type R)
  const void* rhs;             // restricted residual from the finer level (R)
  void* x;                     // solution out (R)
  const double* Ainv;          // coarsest inverse, nc x nc
  long long *iters, *calls;    // counters: [level] of the small level, [level + 1] of the coarsest
  int level;
  int* status;
  const int* gate;
  // LDS layout (byte offsets)
  int off_z, off_p, off_x, off_res, off_tx, off_ty, off_g, off_y, off_part;
};

__device__ __forceinline__ double wsum_block(double v, double* sm) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kThreads / kWave; ++w) s += sm[w];
  __syncthreads();
  return s;
}

template <typename R, int DIM>
__global__ void __launch_bounds__(kThreads, 1) k_small_reg(RegArgs a) {
  if (a.gate && *a.gate) return;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ double sm[kThreads / kWave];
  R* z = reinterpret_cast<R*>(lds + a.off_z);
  R* pv = reinterpret_cast<R*>(lds + a.off_p);
  R* xv = reinterpret_cast<R*>(lds + a.off_x);
  R* res = reinterpret_cast<R*>(lds + a.off_res);
  R* tx1 = reinterpret_cast<R*>(lds + a.off_tx);    // x-pass of the restriction
  R* ty1 = reinterpret_cast<R*>(lds + a.off_ty);    // y-pass (3-D only)
  double* g = reinterpret_cast<double*>(lds + a.off_g);
  double* y = reinterpret_cast<double*>(lds + a.off_y);
  double* part = reinterpret_cast<double*>(lds + a.off_part);
  const R* TX = static_cast<const R*>(a.tx);
  const R* TY = static_cast<const R*>(a.ty);
  const R* TZ = static_cast<const R*>(a.tz);
  const int tid = threadIdx.x;
  const int nx = a.nx, ny = a.ny, nz = a.nz, n = a.n, plane = nx * ny;

  // ---- per-cell constants in registers: the neighbour coefficients (zero
  // across the domain boundary), diagonal and its inverse, the residual, and
  // the cell coordinates packed as i | j << 12 | k << 24.
  int ijk[kOwn];
  R cw[kOwn], ce[kOwn], cs[kOwn], cn[kOwn], cb[kOwn], ct[kOwn], dg[kOwn], di[kOwn];
  R r[kOwn];
#pragma unroll
  for (int u = 0; u < kOwn; ++u) {
    const int c = tid + u * kThreads;
    const int cc = c < n ? c : 0;
    const int i = cc % nx, t = cc / nx, j = t % ny, k = t / ny;
    ijk[u] = i | (j << 12) | (k << 24);
    const int fx = i + (nx + 1) * (j + ny * k), fy = i + nx * (j + (ny + 1) * k);
    const R tw = TX[fx], te = TX[fx + 1], ts = TY[fy], tn = TY[fy + nx];
    R d = tw + te + ts + tn;
    cw[u] = i > 0 ? tw : R(0);
    ce[u] = i < nx - 1 ? te : R(0);
    cs[u] = j > 0 ? ts : R(0);
    cn[u] = j < ny - 1 ? tn : R(0);
    cb[u] = R(0);
    ct[u] = R(0);
    if (DIM == 3) {
      const int fz = i + nx * j + plane * k;
      const R tb = TZ[fz], tt = TZ[fz + plane];
      d += tb + tt;
      cb[u] = k > 0 ? tb : R(0);
      ct[u] = k < nz - 1 ? tt : R(0);
    }
    dg[u] = d;
    di[u] = R(1) / d;
    r[u] = c < n ? static_cast<const R*>(a.rhs)[cc] : R(0);
    // z and p are cleared too: at the domain boundary a cell's neighbour index
    // falls back to the cell itself with a zero coefficient, and in the first
    // half sweep that cell has not been written yet; LDS keeps whatever the
    // previous kernel left there, and 0 times a NaN or Inf pattern is NaN
    if (c < n) {
      xv[c] = R(0);
      z[c] = R(0);
      pv[c] = R(0);
    }
  }
  auto own = [&](int u) { return tid + u * kThreads < n; };
  auto colour = [&](int u) { return ((ijk[u] & 0xfff) + ((ijk[u] >> 12) & 0xfff) + (ijk[u] >> 24)) & 1; };

  // sum over the neighbours of cell u of coefficient * v[neighbour]
  auto offsum = [&](const R* v, int u) -> R {
    const int c = tid + u * kThreads;
    const int i = ijk[u] & 0xfff, j = (ijk[u] >> 12) & 0xfff;
    const int cwi = i > 0 ? c - 1 : c, cei = i < nx - 1 ? c + 1 : c;
    const int csi = j > 0 ? c - nx : c, cni = j < ny - 1 ? c + nx : c;
    R o = cw[u] * v[cwi] + ce[u] * v[cei] + cs[u] * v[csi] + cn[u] * v[cni];
    if (DIM == 3) {
      const int k = ijk[u] >> 24;
      const int cbi = k > 0 ? c - plane : c, cti = k < nz - 1 ? c + plane : c;
      o += cb[u] * v[cbi] + ct[u] * v[cti];
    }
    return o;
  };
  // one red-black half sweep of colour `cl` on z (Section 3 splitting)
  auto half = [&](int cl, bool first) {
#pragma unroll
    for (int u = 0; u < kOwn; ++u)
      if (own(u) && colour(u) == cl) {
        const int c = tid + u * kThreads;
        z[c] = first ? r[u] * di[u] : (r[u] + offsum(z, u)) * di[u];
      }
    __syncthreads();
  };

  double rr = 0.0;
#pragma unroll
  for (int u = 0; u < kOwn; ++u) rr += (double)r[u] * (double)r[u];
  rr = wsum_block(rr, sm);
  double tol = a.tol;
  if (a.rel_floor2 > 0.0 && a.rel_floor2 * rr > tol) tol = a.rel_floor2 * rr;
  long long iters = 0, coarse_calls = 0;
  int status = 0;
  double rho_old = 0.0;
  const int ncx = a.cnx, ncy = a.cny, ncz = a.cnz, nc = a.nc;
  const int rows = ny * nz;

  if (!(rr < tol)) {
    for (int it = 0; it < a.max_inner; ++it) {
      // -- pre-smoothing from zero: R,B,...,R (2m+1 half sweeps)
      for (int h = 0; h <= 2 * a.m; ++h) half(h & 1, h == 0);
      // -- residual, then g = E^T res in separable passes
#pragma unroll
      for (int u = 0; u < kOwn; ++u)
        if (own(u)) {
          const int c = tid + u * kThreads;
          res[c] = r[u] - (dg[u] * z[c] - offsum(z, u));
        }
      __syncthreads();
      for (int e = tid; e < rows * ncx; e += kThreads) {  // x pass: (fine row, I)
        const int row = e / ncx, I = e - row * ncx;
        int lo, hi;
        ext_support(I, a.sx, nx, a.interp, lo, hi);
        R s = R(0);
        for (int i = lo; i <= hi; ++i) s += ext_weight_of<R>(i, I, a.sx, ncx, a.interp) * res[i + nx * row];
        tx1[e] = s;
      }
      __syncthreads();
      if (DIM == 2) {
        for (int e = tid; e < nc; e += kThreads) {  // y pass: (J, I)
          const int J = e / ncx, I = e - J * ncx;
          int lo, hi;
          ext_support(J, a.sy, ny, a.interp, lo, hi);
          R s = R(0);
          for (int j = lo; j <= hi; ++j) s += ext_weight_of<R>(j, J, a.sy, ncy, a.interp) * tx1[j * ncx + I];
          g[e] = (double)s;
        }
      } else {
        for (int e = tid; e < nz * ncy * ncx; e += kThreads) {  // y pass: (k, J, I)
          const int I = e % ncx, t = e / ncx, J = t % ncy, k = t / ncy;
          int lo, hi;
          ext_support(J, a.sy, ny, a.interp, lo, hi);
          R s = R(0);
          for (int j = lo; j <= hi; ++j)
            s += ext_weight_of<R>(j, J, a.sy, ncy, a.interp) * tx1[(j + ny * k) * ncx + I];
          ty1[e] = s;
        }
        __syncthreads();
        for (int e = tid; e < nc; e += kThreads) {  // z pass: (K, J, I)
          const int IJ = e % (ncx * ncy), K = e / (ncx * ncy);
          int lo, hi;
          ext_support(K, a.sz, nz, a.interp, lo, hi);
          R s = R(0);
          for (int k = lo; k <= hi; ++k) s += ext_weight_of<R>(k, K, a.sz, ncz, a.interp) * ty1[k * ncx * ncy + IJ];
          g[e] = (double)s;
        }
      }
      __syncthreads();
      // -- coarsest: y = A^-1 g, columns split into groups summed in order
      {
        const int groups = nc >= kThreads ? 1 : kThreads / nc;
        const int per = (nc + groups - 1) / groups;
        if (tid < groups * nc) {
          for (int i = tid % nc; i < nc; i += kThreads) {
            const int grp = tid / nc;
            const int j0 = grp * per, j1 = j0 + per < nc ? j0 + per : nc;
            double s = 0.0;
            for (int j = j0; j < j1; ++j) s += a.Ainv[(long long)j * nc + i] * g[j];
            part[grp * nc + i] = s;
          }
        }
        __syncthreads();
        for (int i = tid; i < nc; i += kThreads) {
          double s = 0.0;
          for (int grp = 0; grp < groups; ++grp) s += part[grp * nc + i];
          y[i] = s;
        }
        coarse_calls++;
        __syncthreads();
      }
      // -- prolongation z += E y on own cells
#pragma unroll
      for (int u = 0; u < kOwn; ++u)
        if (own(u)) {
          int I0, I1, J0, J1, K0 = 0, K1 = 0;
          R wi0, wi1, wj0, wj1, wk0 = R(1), wk1 = R(0);
          ext_weights<R>(ijk[u] & 0xfff, a.sx, ncx, a.interp, I0, wi0, I1, wi1);
          ext_weights<R>((ijk[u] >> 12) & 0xfff, a.sy, ncy, a.interp, J0, wj0, J1, wj1);
          if (DIM == 3) ext_weights<R>(ijk[u] >> 24, a.sz, ncz, a.interp, K0, wk0, K1, wk1);
          const int b0 = ncx * (J0 + ncy * K0), b1 = ncx * (J1 + ncy * K0);
          R v = wk0 * (wj0 * (wi0 * (R)y[I0 + b0] + wi1 * (R)y[I1 + b0]) + wj1 * (wi0 * (R)y[I0 + b1] + wi1 * (R)y[I1 + b1]));
          if (DIM == 3 && wk1 != R(0)) {
            const int c0 = ncx * (J0 + ncy * K1), c1 = ncx * (J1 + ncy * K1);
            v += wk1 * (wj0 * (wi0 * (R)y[I0 + c0] + wi1 * (R)y[I1 + c0]) + wj1 * (wi0 * (R)y[I0 + c1] + wi1 * (R)y[I1 + c1]));
          }
          z[tid + u * kThreads] += v;
        }
      __syncthreads();
      // -- post-smoothing
      for (int h = 0; h <= 2 * a.m; ++h) half(h & 1, false);
      // -- CG step (Templates Figure 2.5); p and x live in LDS
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < kOwn; ++u)
        if (own(u)) acc += (double)r[u] * (double)z[tid + u * kThreads];
      const double rho = wsum_block(acc, sm);
      if (!(rho == rho) || rho == INFINITY) { status = -4; break; }
      if (!(rho > 0.0)) break;  // no further progress in this precision: the level stops
      const R beta = it == 0 ? R(0) : (R)(rho / rho_old);
#pragma unroll
      for (int u = 0; u < kOwn; ++u)
        if (own(u)) {
          const int c = tid + u * kThreads;
          pv[c] = it == 0 ? z[c] : z[c] + beta * pv[c];
        }
      __syncthreads();
      R q[kOwn];
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < kOwn; ++u) {
        const int c = tid + u * kThreads;
        q[u] = own(u) ? dg[u] * pv[c] - offsum(pv, u) : R(0);
        acc += own(u) ? (double)pv[c] * (double)q[u] : 0.0;
      }
      const double pq = wsum_block(acc, sm);
      if (!(pq == pq) || pq == INFINITY) { status = -4; break; }
      if (!(pq > 0.0)) break;
      const R alpha = (R)(rho / pq);
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < kOwn; ++u)
        if (own(u)) {
          const int c = tid + u * kThreads;
          xv[c] += alpha * pv[c];
          r[u] -= alpha * q[u];
          acc += (double)r[u] * (double)r[u];
        }
      rr = wsum_block(acc, sm);
      rho_old = rho;
      iters++;
      if (rr < tol) break;
    }
  }
  R* xo = static_cast<R*>(a.x);
#pragma unroll
  for (int u = 0; u < kOwn; ++u)
    if (own(u)) xo[tid + u * kThreads] = xv[tid + u * kThreads];
  if (tid == 0) {
    a.iters[a.level] += iters;
    a.calls[a.level] += 1;
    a.calls[a.level + 1] += coarse_calls;
    if (status) a.status[0] = status;
  }
}

}  // namespace

template <typename R>
hipError_t launch_small_reg(const SmallDesc<R>& d, hipStream_t s) {
  // 2-D levels go to the 2x2-block kernel where they fit, else to the
  // colour-split kernel (both precisions); the rest to the cell-strided kernel
  // below.
  const int ks = d.ks, L = d.nlev - 1;
  // these kernels bake in integer factors; the generic one takes the rest
  for (int l = ks; l < L; ++l)
    if (d.X[l].frac) return hipErrorNotSupported;
  if (ks + 1 != L) return hipErrorNotSupported;
  const Lv<R>& V = d.L[ks];
  if (V.n > kOwn * kThreads) return hipErrorNotSupported;
  const Xfer& X = d.X[ks];
  const int nc = X.cnx * X.cny * X.cnz;
  if (nc > 1024) return hipErrorNotSupported;
  if (d.variant == 0) {
    const hipError_t e = launch_small_2x2<R>(d, s);
    if (e != hipErrorNotSupported) return e;
  }
  if (d.variant == 0 || d.variant == 2) {
    const hipError_t e = launch_small_2d<R>(d, s);
    if (e != hipErrorNotSupported) return e;
  }
  RegArgs a{};
  a.dim = V.tz ? 3 : 2;
  a.nx = V.nx; a.ny = V.ny; a.nz = V.nz; a.n = V.n;
  a.sx = X.sx; a.sy = X.sy; a.sz = X.sz;
  a.cnx = X.cnx; a.cny = X.cny; a.cnz = X.cnz; a.nc = nc;
  a.interp = X.interp; a.m = d.m; a.max_inner = d.max_inner;
  a.tol = d.tol[ks]; a.rel_floor2 = d.rel_floor2;
  a.tx = V.tx; a.ty = V.ty; a.tz = V.tz;
  a.rhs = d.r[ks]; a.x = d.x[ks];
  a.Ainv = d.Ainv;
  a.iters = d.iters; a.calls = d.calls; a.level = ks; a.status = d.status;
  a.gate = d.gate;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const int o = (int)off;
    off += (bytes + 15) & ~(size_t)15;
    return o;
  };
  a.off_z = take((size_t)V.n * sizeof(R));
  a.off_p = take((size_t)V.n * sizeof(R));
  a.off_x = take((size_t)V.n * sizeof(R));
  a.off_res = take((size_t)V.n * sizeof(R));
  a.off_tx = take((size_t)V.ny * V.nz * X.cnx * sizeof(R));
  a.off_ty = take((size_t)V.nz * X.cny * X.cnx * sizeof(R));
  a.off_g = take((size_t)nc * sizeof(double));
  a.off_y = take((size_t)nc * sizeof(double));
  a.off_part = take((size_t)1024 * sizeof(double));
  if (off > 156 * 1024) return hipErrorNotSupported;
  static bool attr[2][2] = {{false, false}, {false, false}};
  const int di = a.dim == 3 ? 1 : 0, ri = sizeof(R) == 8 ? 1 : 0;
  const void* fn = a.dim == 3 ? (const void*)k_small_reg<R, 3> : (const void*)k_small_reg<R, 2>;
  if (!attr[di][ri]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    if (e != hipSuccess) return e;
    attr[di][ri] = true;
  }
  if (a.dim == 3)
    hipLaunchKernelGGL((k_small_reg<R, 3>), dim3(1), dim3(kThreads), off, s, a);
  else
    hipLaunchKernelGGL((k_small_reg<R, 2>), dim3(1), dim3(kThreads), off, s, a);
  return hipGetLastError();
}

template hipError_t launch_small_reg<double>(const SmallDesc<double>&, hipStream_t);
template hipError_t launch_small_reg<float>(const SmallDesc<float>&, hipStream_t);

}  // namespace mscg
