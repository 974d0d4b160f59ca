// mscg_dev.h -- device-side building blocks of the recursive multi-scale PCG
// (stencil, red-black Gauss-Seidel, grid transfers, reductions).  Every
// routine takes an explicit (first thread, thread count) range so the same
// code runs in grid-wide kernels and inside the single-workgroup solver of
// the small levels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mscg {

constexpr int kMaxLevels = 8;
constexpr int kWave = 64;

// Device view of one level: cell counts and face transmissibilities.
//   tx: (nx+1)*ny*nz, face i lies between cells i-1 and i (i = 0, nx: boundary)
//   ty: nx*(ny+1)*nz, tz: nx*ny*(nz+1) (nullptr in 2-D)
template <typename R>
struct Lv {
  int nx, ny, nz, n;
  const R *tx, *ty, *tz;
};

// DPP move of a double (two 32-bit halves); lanes without a source read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// DPP move of a double for a pattern in which every lane has a source lane
// (mirrors, quad permutations, row broadcasts): no old value to set up.
template <int CTRL>
__device__ __forceinline__ double dpp_full(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the wave, exact order fixed by the lane pattern; valid in lane 63.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0x111, 0xf>(v);  // row_shr:1
  v += dpp_d<0x112, 0xf>(v);  // row_shr:2
  v += dpp_d<0x114, 0xf>(v);  // row_shr:4
  v += dpp_d<0x118, 0xf>(v);  // row_shr:8: lane 15 of each row holds the row sum
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3: lane 63 holds the sum
  return v;
}

// wave_sum_dpp broadcast to every lane of the wave
__device__ __forceinline__ double wave_total(double v) {
  v = wave_sum_dpp(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Diagonal and off-diagonal sum of the 5/7-point finite-volume operator at
// cell c = (i, j, k): (A x)_c = diag * x_c - off, off = sum_f T_f x_nb over
// interior faces (Section 3).  A boundary face contributes T_f to the
// diagonal only: its neighbour value is zero after lifting.
template <typename R>
__device__ __forceinline__ void stencil_at(const Lv<R>& L, const R* __restrict__ x, int i, int j, int k, int c,
                                           R& diag, R& off) {
  const int nx = L.nx, ny = L.ny;
  const int fx = i + (nx + 1) * (j + ny * k);
  const int fy = i + nx * (j + (ny + 1) * k);
  const R tw = L.tx[fx], te = L.tx[fx + 1], ts = L.ty[fy], tn = L.ty[fy + nx];
  R d = tw + te + ts + tn;
  R o = R(0);
  if (i > 0) o += tw * x[c - 1];
  if (i < nx - 1) o += te * x[c + 1];
  if (j > 0) o += ts * x[c - nx];
  if (j < ny - 1) o += tn * x[c + nx];
  if (L.tz) {
    const int plane = nx * ny;
    const int fz = i + nx * j + plane * k;
    const R tb = L.tz[fz], tt = L.tz[fz + plane];
    d += tb + tt;
    if (k > 0) o += tb * x[c - plane];
    if (k < L.nz - 1) o += tt * x[c + plane];
  }
  diag = d;
  off = o;
}

__device__ __forceinline__ void cell_ijk(int c, int nx, int ny, int& i, int& j, int& k) {
  i = c % nx;
  const int t = c / nx;
  j = t % ny;
  k = t / ny;
}

// Workgroups go to the 8 XCDs in turn.  xcd_block() renumbers them (a
// bijection of [0, gridDim.x)) so that XCD x holds the x-th contiguous run of
// workgroup numbers; block_cells() gives the workgroup its contiguous run of
// cells [c0, c1).  A row's neighbour rows then stay on the same L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, lin = blockIdx.x;
  const int x = lin % 8, d = lin / 8;
  return x * (nb / 8) + min(x, nb % 8) + d;
}

__device__ __forceinline__ void block_cells(int n, int& c0, int& c1) {
  const int nb = gridDim.x, b = xcd_block();
  const int per = (n + nb - 1) / nb;
  c0 = min(n, b * per);
  c1 = min(n, c0 + per);
}

// y = A x over cells [t0, n) step nt; returns the thread's share of x . y.
template <typename R, typename A>
__device__ __forceinline__ A spmv_range(const Lv<R>& L, const R* __restrict__ x, R* __restrict__ y, int t0, int nt) {
  A acc = A(0);
  for (int c = t0; c < L.n; c += nt) {
    int i, j, k;
    cell_ijk(c, L.nx, L.ny, i, j, k);
    R d, o;
    stencil_at(L, x, i, j, k, c, d, o);
    const R v = d * x[c] - o;
    y[c] = v;
    acc += A(x[c]) * A(v);
  }
  return acc;
}

// One red-black Gauss-Seidel half sweep: every cell of `colour` ((i+j+k) mod 2,
// red = 0) gets x_c = (r_c + sum T_f x_nb) * (1 / diag) (Section 3, symmetric
// Gauss-Seidel splitting in red-black order).  `first`: the sweep starts from
// x = 0, so the neighbours are not read.
template <typename R>
__device__ __forceinline__ void gs_half_range(const Lv<R>& L, const R* __restrict__ r, R* __restrict__ x, int colour,
                                              bool first, int t0, int nt) {
  const int half = (L.nx + 1) >> 1;      // colour cells per row, upper bound
  const int rows = L.ny * L.nz;
  const int total = half * rows;
  for (int q = t0; q < total; q += nt) {
    const int row = q / half;
    const int m = q - row * half;
    const int j = row % L.ny, k = row / L.ny;
    const int i = 2 * m + ((j + k + colour) & 1);
    if (i >= L.nx) continue;
    const int c = i + L.nx * row;
    R d, o;
    if (first) {
      const int fx = i + (L.nx + 1) * row;
      const int fy = i + L.nx * (j + (L.ny + 1) * k);
      d = L.tx[fx] + L.tx[fx + 1] + L.ty[fy] + L.ty[fy + L.nx];
      if (L.tz) {
        const int plane = L.nx * L.ny;
        const int fz = i + L.nx * j + plane * k;
        d += L.tz[fz] + L.tz[fz + plane];
      }
      o = R(0);
    } else {
      stencil_at(L, x, i, j, k, c, d, o);
    }
    x[c] = (r[c] + o) * (R(1) / d);  // the tiled smoother forms the same inverse once per cell
  }
}

// 1-D extension weights (Section 3).  Fine cell i of an axis with factor s
// and nc coarse cells takes coarse cells I0, I1 with weights w0, w1.
// Linear: coarse coordinate (i + 1/2)/s - 1/2, clamped to [0, nc-1] (zero
// slope at the boundary).  Constant: the coarse cell that contains i.
template <typename R>
__device__ __forceinline__ void ext_weights(int i, int s, int nc, int interp, int& I0, R& w0, int& I1, R& w1) {
  if (s == 1) { I0 = I1 = i; w0 = R(1); w1 = R(0); return; }
  if (interp == 1) { I0 = I1 = i / s; w0 = R(1); w1 = R(0); return; }
  // xi = (2i + 1 - s) / (2s); exact in binary for s a power of two
  const int num = 2 * i + 1 - s;
  if (num <= 0) { I0 = I1 = 0; w0 = R(1); w1 = R(0); return; }
  if (num >= 2 * s * (nc - 1)) { I0 = I1 = nc - 1; w0 = R(1); w1 = R(0); return; }
  const int b = num / (2 * s);
  const R t = R(num - 2 * s * b) / R(2 * s);
  I0 = b; I1 = b + 1; w0 = R(1) - t; w1 = t;
}

// weight of coarse cell I in fine cell i's extension
template <typename R>
__device__ __forceinline__ R ext_weight_of(int i, int I, int s, int nc, int interp) {
  int I0, I1;
  R w0, w1;
  ext_weights<R>(i, s, nc, interp, I0, w0, I1, w1);
  R w = R(0);
  if (I0 == I) w += w0;
  if (I1 == I && I1 != I0) w += w1;
  return w;
}

// Range of fine cells whose extension touches coarse cell I.
__device__ __forceinline__ void ext_support(int I, int s, int nf, int interp, int& lo, int& hi) {
  if (s == 1) { lo = hi = I; return; }
  if (interp == 1) { lo = I * s; hi = I * s + s - 1; return; }
  lo = I * s - s / 2 - 1;
  hi = I * s + s + s / 2;
  if (lo < 0) lo = 0;
  if (hi > nf - 1) hi = nf - 1;
}

struct Xfer {
  int sx, sy, sz;       // factors fine -> coarse
  int cnx, cny, cnz;    // coarse dims
  int interp;
  int frac;             // 1: factors fine / coarse need not be integers (sx.. unused)
};

// 1-D extension weights for a factor f = nf / nc that need not be an integer
// (Section 3): linear interpolation at the coarse coordinate
// xi = (i + 1/2) / f - 1/2 clamped to [0, nc - 1] (zero slope at the
// boundary), or the coarse cell holding the fine cell's centre.  Computed in
// FP64 and rounded once to R.
template <typename R>
__device__ __forceinline__ void ext_weights_frac(int i, int nf, int nc, int interp, int& I0, R& w0, int& I1, R& w1) {
  I0 = I1 = i;
  w0 = R(1);
  w1 = R(0);
  if (nf == nc) return;
  const double f = (double)nf / nc;
  if (interp == 1) {
    int I = (int)floor((i + 0.5) / f);
    I0 = I1 = I > nc - 1 ? nc - 1 : I;
    return;
  }
  const double xi = (i + 0.5) / f - 0.5;
  if (xi <= 0.0) { I0 = I1 = 0; return; }
  if (xi >= nc - 1) { I0 = I1 = nc - 1; return; }
  const int b = (int)floor(xi);
  const double t = xi - b;
  I0 = b;
  I1 = b + 1;
  w0 = R(1.0 - t);
  w1 = R(t);
}

// weight of coarse cell I in fine cell i's extension, any factor
template <typename R>
__device__ __forceinline__ R ext_weight_of_frac(int i, int I, int nf, int nc, int interp) {
  int I0, I1;
  R w0, w1;
  ext_weights_frac<R>(i, nf, nc, interp, I0, w0, I1, w1);
  R w = R(0);
  if (I0 == I) w += w0;
  if (I1 == I && I1 != I0) w += w1;
  return w;
}

// g_coarse = E^T (r - A x) on the fine level F for coarse cells [t0, nc) step nt.
// x == nullptr means x = 0.
template <typename R>
__device__ __forceinline__ void restrict_range(const Lv<R>& F, const Xfer& X, const R* __restrict__ r,
                                               const R* __restrict__ x, R* __restrict__ g, int t0, int nt) {
  const int nc = X.cnx * X.cny * X.cnz;
  for (int C = t0; C < nc; C += nt) {
    int I, J, K;
    cell_ijk(C, X.cnx, X.cny, I, J, K);
    int ilo, ihi, jlo, jhi, klo, khi;
    ext_support(I, X.sx, F.nx, X.interp, ilo, ihi);
    ext_support(J, X.sy, F.ny, X.interp, jlo, jhi);
    ext_support(K, X.sz, F.nz, X.interp, klo, khi);
    R acc = R(0);
    for (int k = klo; k <= khi; ++k) {
      const R wk = ext_weight_of<R>(k, K, X.sz, X.cnz, X.interp);
      if (wk == R(0)) continue;
      for (int j = jlo; j <= jhi; ++j) {
        const R wj = ext_weight_of<R>(j, J, X.sy, X.cny, X.interp);
        if (wj == R(0)) continue;
        for (int i = ilo; i <= ihi; ++i) {
          const R wi = ext_weight_of<R>(i, I, X.sx, X.cnx, X.interp);
          if (wi == R(0)) continue;
          const int c = i + F.nx * (j + F.ny * k);
          R res = r[c];
          if (x) {
            R d, o;
            stencil_at(F, x, i, j, k, c, d, o);
            res -= d * x[c] - o;
          }
          acc += (wk * wj * wi) * res;
        }
      }
    }
    g[C] = acc;
  }
}

// g_coarse = E^T res for coarse cells [t0, nc) step nt, res already stored
// (no stencil evaluation in the footprint loop).  The x weights of a coarse
// cell are computed once into registers and reused for every fine row.
constexpr int kMaxFoot = 20;  // >= 2s + 2 (linear) and >= s (constant) for s <= 8

template <typename R>
__device__ __forceinline__ void restrict_stored_range(const Lv<R>& F, const Xfer& X, const R* __restrict__ res,
                                                      R* __restrict__ g, int t0, int nt) {
  const int nc = X.cnx * X.cny * X.cnz;
  for (int C = t0; C < nc; C += nt) {
    int I, J, K;
    cell_ijk(C, X.cnx, X.cny, I, J, K);
    int ilo, ihi, jlo, jhi, klo, khi;
    ext_support(I, X.sx, F.nx, X.interp, ilo, ihi);
    ext_support(J, X.sy, F.ny, X.interp, jlo, jhi);
    ext_support(K, X.sz, F.nz, X.interp, klo, khi);
    R wx[kMaxFoot];
#pragma unroll
    for (int a = 0; a < kMaxFoot; ++a) wx[a] = (ilo + a <= ihi) ? ext_weight_of<R>(ilo + a, I, X.sx, X.cnx, X.interp) : R(0);
    R acc = R(0);
    for (int k = klo; k <= khi; ++k) {
      const R wk = ext_weight_of<R>(k, K, X.sz, X.cnz, X.interp);
      if (wk == R(0)) continue;
      for (int j = jlo; j <= jhi; ++j) {
        const R wj = ext_weight_of<R>(j, J, X.sy, X.cny, X.interp);
        if (wj == R(0)) continue;
        const R* row = res + F.nx * (j + F.ny * k) + ilo;
        R racc = R(0);
#pragma unroll
        for (int a = 0; a < kMaxFoot; ++a)
          if (ilo + a <= ihi) racc += wx[a] * row[a];
        acc += (wk * wj) * racc;
      }
    }
    g[C] = acc;
  }
}

// The same transfers for factors that need not be integers (X.frac): x_fine
// += E y over fine cells [t0, n) step nt, and g = E^T res over coarse cells
// [t0, nc) step nt, gathering the fine cells whose extension touches each
// coarse cell.  Weights from ext_weights_frac.
template <typename R>
__device__ __forceinline__ void prolong_frac_range(const Lv<R>& F, const Xfer& X, const R* __restrict__ y,
                                                   R* __restrict__ x, int t0, int nt) {
  for (int c = t0; c < F.n; c += nt) {
    int i, j, k;
    cell_ijk(c, F.nx, F.ny, i, j, k);
    int I[2], J[2], K[2];
    R wi[2], wj[2], wk[2];
    ext_weights_frac<R>(i, F.nx, X.cnx, X.interp, I[0], wi[0], I[1], wi[1]);
    ext_weights_frac<R>(j, F.ny, X.cny, X.interp, J[0], wj[0], J[1], wj[1]);
    ext_weights_frac<R>(k, F.nz, X.cnz, X.interp, K[0], wk[0], K[1], wk[1]);
    R v = R(0);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 2; ++e) {
          const R w = wk[a] * wj[b] * wi[e];
          if (w != R(0)) v += w * y[I[e] + X.cnx * (J[b] + X.cny * K[a])];
        }
    x[c] += v;
  }
}

__device__ __forceinline__ void frac_support(int I, int nf, int nc, int& lo, int& hi) {
  if (nf == nc) { lo = hi = I; return; }
  const double f = (double)nf / nc;
  lo = max((int)floor((I - 1) * f) - 1, 0);
  hi = min((int)ceil((I + 2) * f) + 1, nf - 1);
}

template <typename R>
__device__ __forceinline__ void restrict_frac_range(const Lv<R>& F, const Xfer& X, const R* __restrict__ res,
                                                    R* __restrict__ g, int t0, int nt) {
  const int nc = X.cnx * X.cny * X.cnz;
  for (int c = t0; c < nc; c += nt) {
    const int I = c % X.cnx, J = (c / X.cnx) % X.cny, K = c / (X.cnx * X.cny);
    int ilo, ihi, jlo, jhi, klo, khi;
    frac_support(I, F.nx, X.cnx, ilo, ihi);
    frac_support(J, F.ny, X.cny, jlo, jhi);
    frac_support(K, F.nz, X.cnz, klo, khi);
    R acc = R(0);
    for (int k = klo; k <= khi; ++k) {
      const R wk = ext_weight_of_frac<R>(k, K, F.nz, X.cnz, X.interp);
      if (wk == R(0)) continue;
      for (int j = jlo; j <= jhi; ++j) {
        const R wj = ext_weight_of_frac<R>(j, J, F.ny, X.cny, X.interp);
        if (wj == R(0)) continue;
        for (int i = ilo; i <= ihi; ++i) {
          const R wi = ext_weight_of_frac<R>(i, I, F.nx, X.cnx, X.interp);
          if (wi != R(0)) acc += wk * wj * wi * res[i + F.nx * (j + F.ny * k)];
        }
      }
    }
    g[c] = acc;
  }
}

// x_fine += E y_coarse for fine cells [t0, n) step nt.
template <typename R>
__device__ __forceinline__ void prolong_range(const Lv<R>& F, const Xfer& X, const R* __restrict__ y,
                                              R* __restrict__ x, int t0, int nt) {
  for (int c = t0; c < F.n; c += nt) {
    int i, j, k;
    cell_ijk(c, F.nx, F.ny, i, j, k);
    int I[2], J[2], K[2];
    R wi[2], wj[2], wk[2];
    ext_weights<R>(i, X.sx, X.cnx, X.interp, I[0], wi[0], I[1], wi[1]);
    ext_weights<R>(j, X.sy, X.cny, X.interp, J[0], wj[0], J[1], wj[1]);
    ext_weights<R>(k, X.sz, X.cnz, X.interp, K[0], wk[0], K[1], wk[1]);
    R v = R(0);
    for (int a = 0; a < 2; ++a) {
      if (wk[a] == R(0)) continue;
      for (int b = 0; b < 2; ++b) {
        if (wj[b] == R(0)) continue;
        for (int e = 0; e < 2; ++e) {
          if (wi[e] == R(0)) continue;
          v += (wk[a] * wj[b] * wi[e]) * y[I[e] + X.cnx * (J[b] + X.cny * K[a])];
        }
      }
    }
    x[c] += v;
  }
}

// Deterministic workgroup sum: wavefront butterfly, then waves in order.
// `smem` holds at least blockDim.x / 64 doubles.  Result in every thread.
__device__ __forceinline__ double block_sum(double v, double* smem) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += smem[w];
  __syncthreads();
  return s;
}

}  // namespace mscg
