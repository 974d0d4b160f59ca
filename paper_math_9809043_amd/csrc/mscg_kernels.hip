// mscg_kernels.hip -- gfx950 kernels of the recursive multi-scale PCG and
// their launchers.  All work is stream ordered; nothing here synchronises.
#include "mscg_kernels.h"

#include <hip/hip_runtime.h>

#include "mscg_dev.h"

namespace mscg {

namespace {

constexpr int kBlock = 256;
#define MSCG_COARSE_CAP 1024  // largest coarsest level (LDS of the inverse kernel)
constexpr size_t kBandLds = 144 * 1024;  // LDS of the in-LDS band factorisation and inverse
// dynamic LDS of the small-level solver: 160 KB per CU minus its static arrays
constexpr size_t kSmallLdsBytes = 140 * 1024;

inline int grid_for(long long n, int max_blocks = kMaxPartials) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (int)b;
}

// ---------------------------------------------------------------------------
// Setup: face transmissibilities (Section 3: harmonic mean of the adjacent
// cells times area / distance; a Dirichlet boundary face is held at the face,
// half a cell away, so T = 2 K area / width; a Neumann face has T = 0).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double harm(double a, double b) { return 2.0 * a * b / (a + b); }

__global__ void k_face_T(FaceTArgs a) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long long nfx = (long long)(nx + 1) * ny * nz, nfy = (long long)nx * (ny + 1) * nz;
  const long long nfz = a.dim == 3 ? (long long)nx * ny * (nz + 1) : 0;
  if (t < nfx) {
    const int i = (int)(t % (nx + 1));
    const long long row = t / (nx + 1);  // j + ny*k
    const long long c = (long long)nx * row + i;
    double v;
    if (i == 0) v = a.bc_type[0] == 1 ? 2.0 * a.ax * a.kx[c] : 0.0;
    else if (i == nx) v = a.bc_type[1] == 1 ? 2.0 * a.ax * a.kx[c - 1] : 0.0;
    else v = a.ax * harm(a.kx[c - 1], a.kx[c]);
    a.tx[t] = v;
    return;
  }
  long long u = t - nfx;
  if (u < nfy) {
    const int i = (int)(u % nx);
    const long long r2 = u / nx;
    const int j = (int)(r2 % (ny + 1));
    const long long k = r2 / (ny + 1);
    const long long c = i + (long long)nx * (j + (long long)ny * k);
    double v;
    if (j == 0) v = a.bc_type[2] == 1 ? 2.0 * a.ay * a.ky[c] : 0.0;
    else if (j == ny) v = a.bc_type[3] == 1 ? 2.0 * a.ay * a.ky[c - nx] : 0.0;
    else v = a.ay * harm(a.ky[c - nx], a.ky[c]);
    a.ty[u] = v;
    return;
  }
  u -= nfy;
  if (u < nfz) {
    const long long plane = (long long)nx * ny;
    const long long k = u / plane;
    const long long cxy = u - k * plane;
    double v;
    if (k == 0) v = a.bc_type[4] == 1 ? 2.0 * a.az * a.kz[cxy] : 0.0;
    else if (k == nz) v = a.bc_type[5] == 1 ? 2.0 * a.az * a.kz[cxy + plane * (nz - 1)] : 0.0;
    else v = a.az * harm(a.kz[cxy + plane * (k - 1)], a.kz[cxy + plane * k]);
    a.tz[u] = v;
  }
}

// Validation of K: counts entries that are not finite or not > 0.
__global__ void k_check_positive(const double* __restrict__ k, long long n, int* __restrict__ bad) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  int b = 0;
  for (long long c = t; c < n; c += stride) {
    const double v = k[c];
    if (!(v > 0.0) || !(v < INFINITY)) b = 1;
  }
  if (b) atomicOr(bad, 1);
}

// ---------------------------------------------------------------------------
// Coarse graining (Section 3): 1/T^c = sum_i alpha_i / (sum_j T(i, j)).
// The control volume of a face spans the two adjacent cell centres (half a
// cell at the boundary).  Fine face i covers [i-1/2, i+1/2] (fine units,
// clipped to [0, nf]); coarse face I covers [s(I-1/2), s(I+1/2)] clipped to
// [0, s nc].  alpha_i = overlap / width of the fine span; j runs over the
// fine faces inside the coarse face.  A zero parallel sum (no-flow column)
// gives a zero coarse face.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double span_overlap(int i, int I, int s, int nf, int nc) {
  const double a0 = i == 0 ? 0.0 : i - 0.5, a1 = i == nf ? (double)nf : i + 0.5;
  const double b0 = I == 0 ? 0.0 : s * (I - 0.5), b1 = I == nc ? (double)s * nc : s * (I + 0.5);
  const double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  return hi > lo ? (hi - lo) / (a1 - a0) : 0.0;
}

__global__ void k_coarsen_axis(CoarsenArgs a) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // coarse face array dims (face axis extended by one)
  int ce[3] = {a.cd[0], a.cd[1], a.cd[2]};
  int fe[3] = {a.fd[0], a.fd[1], a.fd[2]};
  ce[a.axis] += 1;
  fe[a.axis] += 1;
  const long long total = (long long)ce[0] * ce[1] * ce[2];
  if (t >= total) return;
  int C[3];
  C[0] = (int)(t % ce[0]);
  C[1] = (int)((t / ce[0]) % ce[1]);
  C[2] = (int)(t / ((long long)ce[0] * ce[1]));
  const int ax = a.axis, a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
  const int s = a.s[ax], I = C[ax];
  int lo = s * I - s, hi = s * I + s;
  if (lo < 0) lo = 0;
  if (hi > a.fd[ax]) hi = a.fd[ax];
  double inv = 0.0;
  bool blocked = false;
  for (int i = lo; i <= hi && !blocked; ++i) {
    const double alpha = span_overlap(i, I, s, a.fd[ax], a.cd[ax]);
    if (alpha == 0.0) continue;
    double par = 0.0;
    for (int u = 0; u < a.s[a1]; ++u)
      for (int v = 0; v < a.s[a2]; ++v) {
        int F[3];
        F[ax] = i;
        F[a1] = C[a1] * a.s[a1] + u;
        F[a2] = C[a2] * a.s[a2] + v;
        par += a.f[F[0] + (long long)fe[0] * (F[1] + (long long)fe[1] * F[2])];
      }
    if (par == 0.0) blocked = true;
    else inv += alpha / par;
  }
  a.c[t] = blocked ? 0.0 : 1.0 / inv;
}

// The same coarse graining for factors that need not be integers (Section 3):
// a fine face that only partly overlaps the coarse face counts with the
// fraction of the height in the overlap in the parallel sum and inversely
// with the fraction of the width in the series sum.
__device__ __forceinline__ double frac_face_overlap(int i, int I, int nf, int nc) {
  const double f = (double)nf / nc;
  const double a0 = i == 0 ? 0.0 : i - 0.5, a1 = i == nf ? (double)nf : i + 0.5;
  const double b0 = I == 0 ? 0.0 : f * I - 0.5 * f, b1 = I == nc ? (double)nf : f * I + 0.5 * f;
  const double lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
  return hi > lo ? (hi - lo) / (a1 - a0) : 0.0;
}

__device__ __forceinline__ double frac_cell_overlap(int j, int J, int nf, int nc) {
  const double f = (double)nf / nc;
  const double b0 = f * J, b1 = J + 1 == nc ? (double)nf : f * (J + 1);
  const double lo = j > b0 ? (double)j : b0, hi = j + 1 < b1 ? (double)(j + 1) : b1;
  return hi > lo ? hi - lo : 0.0;
}

__global__ void k_coarsen_frac(CoarsenArgs a) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int ce[3] = {a.cd[0], a.cd[1], a.cd[2]};
  int fe[3] = {a.fd[0], a.fd[1], a.fd[2]};
  ce[a.axis] += 1;
  fe[a.axis] += 1;
  const long long total = (long long)ce[0] * ce[1] * ce[2];
  if (t >= total) return;
  int C[3];
  C[0] = (int)(t % ce[0]);
  C[1] = (int)((t / ce[0]) % ce[1]);
  C[2] = (int)(t / ((long long)ce[0] * ce[1]));
  const int ax = a.axis, a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
  const int I = C[ax];
  const double fa = (double)a.fd[ax] / a.cd[ax];
  int lo = (int)floor(fa * (I - 1)), hi = (int)ceil(fa * (I + 1));
  if (lo < 0) lo = 0;
  if (hi > a.fd[ax]) hi = a.fd[ax];
  const double f1 = (double)a.fd[a1] / a.cd[a1], f2 = (double)a.fd[a2] / a.cd[a2];
  const int ulo = (int)floor(f1 * C[a1]), vlo = (int)floor(f2 * C[a2]);
  const int uhi = min((int)ceil(f1 * (C[a1] + 1)), a.fd[a1]), vhi = min((int)ceil(f2 * (C[a2] + 1)), a.fd[a2]);
  double inv = 0.0;
  bool blocked = false;
  for (int i = lo; i <= hi && !blocked; ++i) {
    const double alpha = frac_face_overlap(i, I, a.fd[ax], a.cd[ax]);
    if (alpha == 0.0) continue;
    double par = 0.0;
    for (int u = ulo; u < uhi; ++u) {
      const double bu = frac_cell_overlap(u, C[a1], a.fd[a1], a.cd[a1]);
      if (bu == 0.0) continue;
      for (int v = vlo; v < vhi; ++v) {
        const double bv = frac_cell_overlap(v, C[a2], a.fd[a2], a.cd[a2]);
        if (bv == 0.0) continue;
        int F[3];
        F[ax] = i;
        F[a1] = u;
        F[a2] = v;
        par += bu * bv * a.f[F[0] + (long long)fe[0] * (F[1] + (long long)fe[1] * F[2])];
      }
    }
    if (par == 0.0) blocked = true;
    else inv += alpha / par;
  }
  a.c[t] = blocked ? 0.0 : 1.0 / inv;
}

// x_fine += E y for factors that need not be integers: one thread per fine cell
template <typename R>
__global__ void __launch_bounds__(kBlock) k_prolong_frac(Lv<R> F, Xfer X, const R* __restrict__ y, R* __restrict__ x,
                                                          const int* __restrict__ gate) {
  if (gate && *gate) return;
  prolong_frac_range(F, X, y, x, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// g = E^T res for factors that need not be integers: one thread per coarse
// cell gathers the fine cells whose extension touches it
template <typename R>
__global__ void __launch_bounds__(kBlock) k_restrict_frac(Lv<R> F, Xfer X, const R* __restrict__ res, R* __restrict__ g,
                                                           const int* __restrict__ gate) {
  if (gate && *gate) return;
  restrict_frac_range(F, X, res, g, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = t; c < n; c += stride) b[c] = (float)a[c];
}

// Dense operator of the coarsest level, column c = A e_c, row-major n x n.
__global__ void k_dense_assemble(Lv<double> L, double* __restrict__ A) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = L.n;
  if (c >= n) return;
  int i, j, k;
  cell_ijk(c, L.nx, L.ny, i, j, k);
  // row c of A: diag at c, -T at neighbours (A is symmetric)
  for (int q = 0; q < n; ++q) A[(long long)c * n + q] = 0.0;
  const int fx = i + (L.nx + 1) * (j + L.ny * k), fy = i + L.nx * (j + (L.ny + 1) * k);
  double d = L.tx[fx] + L.tx[fx + 1] + L.ty[fy] + L.ty[fy + L.nx];
  if (i > 0) A[(long long)c * n + c - 1] = -L.tx[fx];
  if (i < L.nx - 1) A[(long long)c * n + c + 1] = -L.tx[fx + 1];
  if (j > 0) A[(long long)c * n + c - L.nx] = -L.ty[fy];
  if (j < L.ny - 1) A[(long long)c * n + c + L.nx] = -L.ty[fy + L.nx];
  if (L.tz) {
    const int plane = L.nx * L.ny, fz = i + L.nx * j + plane * k;
    d += L.tz[fz] + L.tz[fz + plane];
    if (k > 0) A[(long long)c * n + c - plane] = -L.tz[fz];
    if (k < L.nz - 1) A[(long long)c * n + c + plane] = -L.tz[fz + plane];
  }
  A[(long long)c * n + c] = d;
}

// Coarsest factorisation (Section 2.2/2.3: the recursion ends with an exact
// solve).  A is symmetric, so its row-major assembly is also column-major;
// the factor L (A = L L^T) overwrites the lower triangle in column-major
// order, L[i][k] at A[k n + i], so a column is contiguous.  One workgroup,
// right-looking: scale column j, then each wave updates whole trailing
// columns with its lanes along i (coalesced).  status[0] = 1 if A is not
// positive definite.
__global__ void __launch_bounds__(1024) k_chol_factor(double* __restrict__ A, int n, int* __restrict__ status) {
  __shared__ int bad;
  __shared__ double sd;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid / kWave, lane = tid % kWave, nw = nt / kWave;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      const double d = A[(long long)j * n + j];
      if (!(d > 0.0)) bad = 1;
      sd = d > 0.0 ? sqrt(d) : 1.0;
      A[(long long)j * n + j] = sd;
    }
    __syncthreads();
    if (bad) break;
    const double d = sd;
    double* colj = A + (long long)j * n;
    for (int i = j + 1 + tid; i < n; i += nt) colj[i] /= d;
    __syncthreads();
    for (int l = j + 1 + wave; l < n; l += nw) {
      const double ljl = colj[l];
      double* coll = A + (long long)l * n;
      for (int i = l + lane; i < n; i += kWave) coll[i] -= colj[i] * ljl;
    }
    __syncthreads();
  }
  if (tid == 0) status[0] = bad;
}

// Row-major copy of the lower factor: Lr[i n + k] = L[i][k] (k <= i).
__global__ void k_factor_rows(const double* __restrict__ Lc, double* __restrict__ Lr, int n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), k = (int)(e % n);
  Lr[e] = k <= i ? Lc[(long long)k * n + i] : 0.0;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// A^-1 from the factor, one wave per column c: solve L w = e_c (forward),
// then L^T x = w (backward); column c of A^-1 equals row c by symmetry and is
// written to Ainv[c n + k].  The lanes split every row's dot product; lane l
// owns the entries k = l (mod 64) of w and x, so each entry is written and
// read by the same lane.  Forward rows read the row-major copy, backward rows
// the column-major factor: both coalesced.
__global__ void __launch_bounds__(256) k_chol_inverse(const double* __restrict__ Lc, const double* __restrict__ Lr,
                                                      double* __restrict__ Ainv, int n) {
  __shared__ double wbuf[4][MSCG_COARSE_CAP];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int c = blockIdx.x * 4 + wave;
  if (c >= n) return;  // whole wave; no workgroup barrier in this kernel
  double* w = wbuf[wave];
  for (int k = lane; k < n; k += kWave) w[k] = 0.0;
  // first owned index >= c for this lane
  const int kc = c + ((lane - c % kWave) + kWave) % kWave;
  for (int i = c; i < n; ++i) {
    double part = 0.0;
    for (int k = kc; k < i; k += kWave) part += Lr[(long long)i * n + k] * w[k];
    part = wave_sum(part);
    const double wi = ((i == c ? 1.0 : 0.0) - part) / Lr[(long long)i * n + i];
    if ((i & (kWave - 1)) == lane) w[i] = wi;
  }
  for (int i = n - 1; i >= 0; --i) {
    // owned indices k > i
    const int k0 = i + 1 + ((lane - (i + 1) % kWave) + kWave) % kWave;
    double part = 0.0;
    for (int k = k0; k < n; k += kWave) part += Lc[(long long)i * n + k] * w[k];
    part = wave_sum(part);
    const double wi = (i & (kWave - 1)) == lane ? w[i] : 0.0;
    const double wval = wave_sum(wi);  // broadcast w_i from its owner
    const double xi = (wval - part) / Lc[(long long)i * n + i];
    if ((i & (kWave - 1)) == lane) w[i] = xi;
  }
  for (int k = lane; k < n; k += kWave) Ainv[(long long)c * n + k] = w[k];
}

// Banded coarsest factorisation.  Every nonzero A[i][k] of the 5/7-point
// operator has |i - k| <= b (b = nx in 2-D, nx ny in 3-D, natural order), and
// the Cholesky factor keeps that band.  One workgroup; the b + 1 rows j..j+b
// that step j updates sit in LDS as a window (row i in slot i mod (b+1),
// entry t holding column i - b + t), so a step touches LDS only: scale column
// j, update the trailing b x b triangle, and refill the freed slot with row
// j + b + 1 of A.  Outputs: Lb[i (b+1) + t] = L[i][i - b + t] (row band) and
// Lt[i (b+1) + t] = L[i + t][i] (column band), zero outside the matrix.
// status[0] = 1 if A is not positive definite.
__global__ void __launch_bounds__(1024) k_chol_band(const double* __restrict__ A, int n, int b,
                                                    double* __restrict__ Lb, double* __restrict__ Lt,
                                                    int* __restrict__ status) {
  extern __shared__ double win[];  // (b + 1) x (b + 1)
  const int W = b + 1, tid = threadIdx.x, nt = blockDim.x;
  auto row_entry = [&](int i, int t) {  // A[i][i - b + t], zero outside the matrix
    const int k = i - b + t;
    return (i < n && k >= 0) ? A[(long long)i * n + k] : 0.0;
  };
  for (int e = tid; e < W * W; e += nt) win[e] = row_entry(e / W, e % W);
  __syncthreads();
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    const int sj = j % W;
    const double djj = win[sj * W + b];
    if (!(djj > 0.0)) { bad = 1; break; }  // every thread reads the same value
    const double ljj = sqrt(djj);
    // scale column j of rows j+1..j+b; row j is final
    for (int t = tid; t < b; t += nt) {
      const int i = j + 1 + t;
      if (i < n) win[(i % W) * W + (j - i + b)] /= ljj;
    }
    for (int t = tid; t < W; t += nt) Lb[(long long)j * W + t] = t == b ? ljj : win[sj * W + t];
    __syncthreads();
    // column j of L, then the trailing update a_ik -= l_ij l_kj (j < k <= i <= j+b),
    // and row j + b + 1 of A into the freed slot
    for (int t = tid; t < W; t += nt) {
      const int i = j + t;
      Lt[(long long)j * W + t] = t == 0 ? ljj : (i < n ? win[(i % W) * W + (j - i + b)] : 0.0);
    }
    for (int e = tid; e < b * b; e += nt) {
      const int ii = e / b, kk = e - ii * b;
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      if (i >= n) continue;
      const int si = i % W, sk = k % W;
      win[si * W + (k - i + b)] -= win[si * W + (j - i + b)] * win[sk * W + (j - k + b)];
    }
    for (int t = tid; t < W; t += nt) win[sj * W + t] = row_entry(j + W, t);
    __syncthreads();
  }
  if (tid == 0) status[0] = bad;
}

// Entry A[i][i + off] (-b <= off <= 0) of the 5/7-point operator, with the
// sums of k_dense_assemble in the same order.
__device__ double band_entry(const Lv<double>& L, int c, int off) {
  int i, j, k;
  cell_ijk(c, L.nx, L.ny, i, j, k);
  const int fx = i + (L.nx + 1) * (j + L.ny * k), fy = i + L.nx * (j + (L.ny + 1) * k);
  const int plane = L.nx * L.ny;
  if (off == 0) {
    double d = L.tx[fx] + L.tx[fx + 1] + L.ty[fy] + L.ty[fy + L.nx];
    if (L.tz) {
      const int fz = i + L.nx * j + plane * k;
      d += L.tz[fz] + L.tz[fz + plane];
    }
    return d;
  }
  if (off == -1 && i > 0) return -L.tx[fx];
  if (off == -L.nx && j > 0) return -L.ty[fy];
  if (L.tz && off == -plane && k > 0) return -L.tz[i + L.nx * j + plane * k];
  return 0.0;
}

// The same banded factorisation with the whole band in LDS (n (b + 1)
// doubles), assembled there from the transmissibilities: a step reads and
// writes LDS only, with no wait on memory.  Row i of the band holds
// A[i][i - b + t] and, once the steps before i are done, L[i][i - b + t].
// Same operations, in the same order, as k_chol_band.
__global__ void __launch_bounds__(256) k_chol_band_lds(Lv<double> L, int b, double* __restrict__ Lb,
                                                       double* __restrict__ Lt, int* __restrict__ status) {
  extern __shared__ double band[];
  const int n = L.n, W = b + 1, tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < n * W; e += nt) {
    const int i = e / W, t = e - i * W;
    band[e] = i - b + t >= 0 ? band_entry(L, i, t - b) : 0.0;
  }
  __syncthreads();
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    const double djj = band[j * W + b];
    if (!(djj > 0.0)) { bad = 1; break; }  // every thread reads the same value
    const double ljj = sqrt(djj);
    for (int t = tid; t < b; t += nt) {
      const int i = j + 1 + t;
      if (i < n) band[i * W + (b - 1 - t)] /= ljj;
    }
    __syncthreads();  // every thread has read band[j][b]
    if (tid == 0) band[j * W + b] = ljj;
    for (int e = tid; e < b * b; e += nt) {
      const int ii = e / b, kk = e - ii * b;
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      if (i >= n) continue;
      band[i * W + (k - i + b)] -= band[i * W + (j - i + b)] * band[k * W + (j - k + b)];
    }
    __syncthreads();
  }
  if (!bad)
    for (int e = tid; e < n * W; e += nt) {
      const int i = e / W, t = e - i * W;
      Lb[e] = band[e];
      Lt[e] = i + t < n ? band[(i + t) * W + (b - t)] : 0.0;
    }
  if (tid == 0) status[0] = bad;
}

// A^-1 from the banded factor, one wave per column c: L w = e_c forward, then
// L^T x = w backward.  Lane l holds the latest w_k (x_k) with k = l mod 64;
// with b <= 64 the band of row i contains at most one such k per lane, so a
// step is one product per lane and a DPP wave sum.  The four waves of a
// workgroup handle consecutive columns and walk the rows together: chunks of
// band rows are staged in LDS for all four.
constexpr int kBandChunk = 32;

__global__ void __launch_bounds__(256) k_band_inverse(const double* __restrict__ Lb, const double* __restrict__ Lt,
                                                      double* __restrict__ Ainv, int n, int b) {
  __shared__ double rows[kBandChunk][65];
  __shared__ double wbuf[4][MSCG_COARSE_CAP];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int W = b + 1;
  const int c0 = blockIdx.x * 4, c = c0 + wave;
  double* w = wbuf[wave];
  for (int k = lane; k < n; k += kWave) w[k] = 0.0;
  double reg = 0.0;
  // forward: w_i = (delta_ic - sum_{k in [max(c, i-b), i)} L[i][k] w_k) / L[i][i]
  for (int i0 = c0; i0 < n; i0 += kBandChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kBandChunk * W; e += blockDim.x) {
      const int r = e / W, t = e - r * W, i = i0 + r;
      rows[r][t] = i < n ? Lb[(long long)i * W + t] : 0.0;
    }
    __syncthreads();
    if (c >= n) continue;
    for (int r = 0; r < kBandChunk; ++r) {
      const int i = i0 + r;
      if (i >= n) break;
      if (i < c) continue;
      const int d = (lane - i) & (kWave - 1), k = i - kWave + d;
      const double term = (k >= c && k >= i - b) ? rows[r][k - i + b] * reg : 0.0;
      const double s = wave_total(term);
      const double wi = ((i == c ? 1.0 : 0.0) - s) / rows[r][b];
      if ((i & (kWave - 1)) == lane) {
        reg = wi;
        w[i] = wi;
      }
    }
  }
  // backward: x_i = (w_i - sum_{k in (i, min(n-1, i+b)]} L[k][i] x_k) / L[i][i]
  reg = 0.0;
  for (int i0 = n - 1; i0 >= 0; i0 -= kBandChunk) {
    __syncthreads();
    for (int e = threadIdx.x; e < kBandChunk * W; e += blockDim.x) {
      const int r = e / W, t = e - r * W, i = i0 - r;
      rows[r][t] = i >= 0 ? Lt[(long long)i * W + t] : 0.0;
    }
    __syncthreads();
    if (c >= n) continue;
    for (int r = 0; r < kBandChunk; ++r) {
      const int i = i0 - r;
      if (i < 0) break;
      const int k = i + 1 + ((lane - i - 1) & (kWave - 1));
      const double term = (k <= i + b && k < n) ? rows[r][k - i] * reg : 0.0;
      const double s = wave_total(term);
      const double xi = (w[i] - s) / rows[r][0];
      if ((i & (kWave - 1)) == lane) {
        reg = xi;
        w[i] = xi;
      }
    }
  }
  if (c < n)
    for (int k = lane; k < n; k += kWave) Ainv[(long long)c * n + k] = w[k];
}

// ---------------------------------------------------------------------------
// Solve-phase kernels (grid-wide).  Reductions write one partial per block;
// k_finish_* sums them in block order in one workgroup, so every result is
// independent of scheduling.
// ---------------------------------------------------------------------------

template <typename R>
__global__ void __launch_bounds__(kBlock) k_spmv_dot(Lv<R> L, const R* __restrict__ x, R* __restrict__ y,
                                                      double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  int c0, c1;
  block_cells(L.n, c0, c1);
  double acc = 0.0;
  for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    int i, j, k;
    cell_ijk(c, L.nx, L.ny, i, j, k);
    R d, o;
    stencil_at(L, x, i, j, k, c, d, o);
    const R v = d * x[c] - o;
    y[c] = v;
    acc += double(x[c]) * double(v);
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0 && part) part[blockIdx.x] = s;
}

// r = b - A x, partial |r|^2
template <typename R>
__global__ void __launch_bounds__(kBlock) k_residual(Lv<R> L, const R* __restrict__ b, const R* __restrict__ x,
                                                      R* __restrict__ r, double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < L.n; c += gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(c, L.nx, L.ny, i, j, k);
    R d, o;
    stencil_at(L, x, i, j, k, c, d, o);
    const R v = b[c] - (d * x[c] - o);
    r[c] = v;
    acc += (double)v * (double)v;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// res = b - A x without a reduction
template <typename R>
__global__ void __launch_bounds__(kBlock) k_residual_nodot(Lv<R> L, const R* __restrict__ b, const R* __restrict__ x,
                                                            R* __restrict__ res, const int* __restrict__ gate) {
  if (gate && *gate) return;
  for (int c = xcd_block() * blockDim.x + threadIdx.x; c < L.n; c += gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(c, L.nx, L.ny, i, j, k);
    R d, o;
    stencil_at(L, x, i, j, k, c, d, o);
    res[c] = b[c] - (d * x[c] - o);
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_dot(const R* __restrict__ a, const R* __restrict__ b, int n,
                                                 double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    acc += (double)a[c] * (double)b[c];
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z (first iteration) or p = z + beta p
template <typename R>
__global__ void __launch_bounds__(kBlock) k_update_p(const R* __restrict__ z, R* __restrict__ p, int n,
                                                      const Scal* __restrict__ sc) {
  const bool first = sc->it == 0;
  const R beta = (R)sc->beta;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    p[c] = first ? z[c] : z[c] + beta * p[c];
}

// x += alpha p, r -= alpha q, partial |r|^2
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cg_update(R* __restrict__ x, R* __restrict__ r, const R* __restrict__ p,
                                                       const R* __restrict__ q, int n, const Scal* __restrict__ sc,
                                                       double* __restrict__ part) {
  __shared__ double sm[kBlock / kWave];
  const R alpha = (R)sc->alpha;
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    x[c] += alpha * p[c];
    const R v = r[c] - alpha * q[c];
    r[c] = v;
    acc += (double)v * (double)v;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One step of the modified Jacobi splitting (P = 2D, Q = D - U - L, Section 3):
// xout = xin + (r - A xin) / (2 d) for every cell; first: xin = 0, so
// xout = r / (2 d).  xout must not alias xin.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_mjac_step(Lv<R> L, const R* __restrict__ r, const R* __restrict__ xin,
                                                       R* __restrict__ xout, int first, const int* __restrict__ gate) {
  if (gate && *gate) return;
  for (int c = xcd_block() * blockDim.x + threadIdx.x; c < L.n; c += gridDim.x * blockDim.x) {
    int i, j, k;
    cell_ijk(c, L.nx, L.ny, i, j, k);
    R d, o;
    if (first) {
      stencil_at(L, r, i, j, k, c, d, o);  // only d is used
      xout[c] = (r[c] - R(0)) / (R(2) * d);
    } else {
      stencil_at(L, xin, i, j, k, c, d, o);
      xout[c] = xin[c] + (r[c] - (d * xin[c] - o)) / (R(2) * d);
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_gs_half(Lv<R> L, const R* __restrict__ r, R* __restrict__ x, int colour,
                                                     int first, const int* __restrict__ gate) {
  if (gate && *gate) return;
  gs_half_range(L, r, x, colour, first != 0, xcd_block() * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_restrict(Lv<R> F, Xfer X, const R* __restrict__ r,
                                                      const R* __restrict__ x, R* __restrict__ g) {
  restrict_range(F, X, r, x, g, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_restrict_stored(Lv<R> F, Xfer X, const R* __restrict__ res,
                                                             R* __restrict__ g, const int* __restrict__ gate) {
  if (gate && *gate) return;
  restrict_stored_range(F, X, res, g, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_prolong(Lv<R> F, Xfer X, const R* __restrict__ y, R* __restrict__ x,
                                                     const int* __restrict__ gate) {
  if (gate && *gate) return;
  prolong_range(F, X, y, x, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// The same on a 2-D level, one workgroup per stretch of a fine row: the row's
// weights are the workgroup's, the column's the thread's, with no per-cell
// index division.  Same products in the same order as prolong_range (the z
// weight is 1 in 2-D), so the result is the same bit for bit.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_prolong_2d(Lv<R> F, Xfer X, const R* __restrict__ y, R* __restrict__ x,
                                                        const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= F.nx) return;
  int I[2], J[2];
  R wi[2], wj[2];
  ext_weights<R>(i, X.sx, X.cnx, X.interp, I[0], wi[0], I[1], wi[1]);
  ext_weights<R>(j, X.sy, X.cny, X.interp, J[0], wj[0], J[1], wj[1]);
  R v = R(0);
  for (int b = 0; b < 2; ++b) {
    if (wj[b] == R(0)) continue;
    for (int e = 0; e < 2; ++e) {
      if (wi[e] == R(0)) continue;
      v += (R(1) * wj[b] * wi[e]) * y[I[e] + X.cnx * J[b]];
    }
  }
  x[i + F.nx * j] += v;
}

// y = A^-1 g on the coarsest level (dense FP64 inverse; g, y in R).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_coarse_solve(const double* __restrict__ Ainv, const R* __restrict__ g,
                                                          R* __restrict__ y, int n, const int* __restrict__ gate) {
  // y = A^-1 g with one wave per output: A^-1 is symmetric, so output i is
  // the dot product of the stored row i (contiguous) with g.  Lane l sums the
  // columns l, l + 64, ..., then a fixed-order wave sum: the same bits on
  // every run.  A whole wave leaves together when it has no row.
  if (gate && *gate) return;
  const int lane = threadIdx.x % kWave, i = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  if (i >= n) return;
  const double* row = Ainv + (long long)i * n;
  double s = 0.0;
  for (int j = lane; j < n; j += kWave) s += row[j] * (double)g[j];
  s = wave_total(s);
  if (lane == 0) y[i] = (R)s;
}

// Keeps a loaded value live at this point, so that a load whose result is only
// needed after a gate's early return is still issued before it (the two
// round trips to memory then overlap).
template <typename T>
__device__ __forceinline__ void issue_before(const T& v) {
  asm volatile("" ::"s"(v));
}

// An ungated launch reads this instead of a flag: the gate's load then needs
// no branch on the pointer first.
__device__ const int g_no_gate = 0;
__device__ __forceinline__ const int* gate_or_zero(const int* gate) { return gate ? gate : &g_no_gate; }

// Scalar bookkeeping of one level's CG (Templates Figure 2.5) from the sum s
// of a reduction; one thread.
__device__ void apply_op(double s, Scal* __restrict__ sc, int op) {
  switch (op) {
    case kOpBB:
      sc->bb = s;
      break;
    case kOpEntry:  // entry check of the level criterion, with the mixed-precision floor
      sc->rr = s;
      sc->it = 0;
      sc->started = 0;
      sc->status = 0;
      if (sc->rel_floor2 > 0.0 && sc->rel_floor2 * s > sc->tol) sc->tol = sc->rel_floor2 * s;
      sc->converged = s < sc->tol ? 1 : 0;
      if (!(s == s) || s == INFINITY) { sc->status = -4; sc->converged = 1; }
      break;
    case kOpRho:
      sc->started += 1;
      // r.z <= 0 in finite precision: no further progress (status 1, the
      // caller decides); a non-finite value is a breakdown (-4)
      if (!(s == s) || s == INFINITY) { sc->status = -4; sc->converged = 1; }
      else if (!(s > 0.0)) { sc->status = 1; sc->converged = 1; }
      // r_new - r_old = -alpha q_old, so z.(r_new - r_old) = -alpha (z.q_old)
      sc->beta = sc->it == 0 ? 0.0 : (sc->flexible ? -sc->alpha * sc->zq / sc->rho : s / sc->rho);
      sc->rho = s;
      break;
    case kOpZq:
      sc->zq = s;
      break;
    case kOpPq:
      if (!(s == s) || s == INFINITY) { sc->status = -4; sc->converged = 1; sc->alpha = 0.0; }
      else if (!(s > 0.0) || sc->status != 0) { if (sc->status == 0) sc->status = 1; sc->converged = 1; sc->alpha = 0.0; }
      else sc->alpha = sc->rho / s;
      break;
    case kOpRr:
      sc->rr = s;
      sc->it += 1;
      if (s < sc->tol) sc->converged = 1;
      if (!(s == s) || s == INFINITY) { sc->status = -4; sc->converged = 1; }
      break;
  }
}

// Sum of the partials in block order (thread t takes partials t, t + blockDim,
// ..., then the deterministic workgroup sum).
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int nparts, double* sm) {
  double acc = 0.0;
  for (int q = threadIdx.x; q < nparts; q += blockDim.x) acc += part[q];
  return block_sum(acc, sm);
}

// Partials read in one batch (up to kPF per thread, issued together with
// whatever else the kernel needs first), then summed in the order of
// sum_partials: every workgroup that sums the same partials gets the same bits.
constexpr int kPF = 8;
__device__ __forceinline__ void load_partials(const double* __restrict__ part, int nparts, double (&pv)[kPF]) {
#pragma unroll
  for (int u = 0; u < kPF; ++u) {
    const int q = threadIdx.x + u * blockDim.x;
    pv[u] = q < nparts ? part[q] : 0.0;
  }
}
__device__ __forceinline__ double sum_loaded_partials(const double (&pv)[kPF], const double* __restrict__ part,
                                                      int nparts, double* sm) {
  double acc = pv[0];
#pragma unroll
  for (int u = 1; u < kPF; ++u) acc += pv[u];
  for (int q = threadIdx.x + kPF * blockDim.x; q < nparts; q += blockDim.x) acc += part[q];
  return block_sum(acc, sm);
}

__global__ void __launch_bounds__(kBlock) k_finish(const double* __restrict__ part, int nparts, Scal* __restrict__ sc,
                                                   int op, const int* __restrict__ gate) {
  // the gate, the scalars and the partials are read in one round trip
  const int gv = *gate_or_zero(gate);
  Scal loc = *sc;
  double pv[kPF];
  load_partials(part, nparts, pv);
  issue_before(gv);
  issue_before(loc.rho);
  if (gv) return;
  __shared__ double sm[kBlock / kWave];
  const double s = sum_loaded_partials(pv, part, nparts, sm);
  if (threadIdx.x == 0) {
    apply_op(s, &loc, op);
    *sc = loc;
  }
}

// partial sums of a . b (gated)
template <typename R>
__global__ void __launch_bounds__(kBlock) k_dot_g(const R* __restrict__ a, const R* __restrict__ b, int n,
                                                   double* __restrict__ part, const int* __restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double sm[kBlock / kWave];
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    acc += (double)a[c] * (double)b[c];
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p_new = z (first iteration) or z + beta p_old, q = A p_new over this
// thread's cells; returns its part of p_new . q.  The neighbours' p_new are
// formed from z and p_old on the fly (p_new and p_old are different buffers).
template <typename R>
__device__ __forceinline__ double pspmv_range(const Lv<R>& L, const R* __restrict__ z, const R* __restrict__ pold,
                                              R* __restrict__ pnew, R* __restrict__ q, bool first, R beta) {
  auto pv = [&](int c) { return first ? z[c] : z[c] + beta * pold[c]; };
  double acc = 0.0;
  const int nx = L.nx, ny = L.ny;
  int c0, c1;
  block_cells(L.n, c0, c1);
  for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    int i, j, k;
    cell_ijk(c, nx, ny, i, j, k);
    const int fx = i + (nx + 1) * (j + ny * k);
    const int fy = i + nx * (j + (ny + 1) * k);
    const R tw = L.tx[fx], te = L.tx[fx + 1], ts = L.ty[fy], tn = L.ty[fy + nx];
    R d = tw + te + ts + tn;
    R o = R(0);
    if (i > 0) o += tw * pv(c - 1);
    if (i < nx - 1) o += te * pv(c + 1);
    if (j > 0) o += ts * pv(c - nx);
    if (j < ny - 1) o += tn * pv(c + nx);
    if (L.tz) {
      const int plane = nx * ny;
      const int fz = i + nx * j + plane * k;
      const R tb = L.tz[fz], tt = L.tz[fz + plane];
      d += tb + tt;
      if (k > 0) o += tb * pv(c - plane);
      if (k < L.nz - 1) o += tt * pv(c + plane);
    }
    const R pc = pv(c);
    const R v = d * pc - o;
    pnew[c] = pc;
    q[c] = v;
    acc += (double)pc * (double)v;
  }
  return acc;
}

// The direction update and SpMV with partial sums of p.q (beta from sc).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_pspmv(Lv<R> L, const R* __restrict__ z, const R* __restrict__ pold,
                                                   R* __restrict__ pnew, R* __restrict__ q, double* __restrict__ part,
                                                   const Scal* __restrict__ sc, const int* __restrict__ gate) {
  const int gv = *gate_or_zero(gate);
  const int it = sc->it;
  const double beta_d = sc->beta;
  issue_before(gv);
  issue_before(it);
  issue_before(beta_d);
  if (gv) return;
  __shared__ double sm[kBlock / kWave];
  const double acc = pspmv_range(L, z, pold, pnew, q, it == 0, (R)beta_d);
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The same with the finish of r.z folded in: every workgroup sums the r.z
// partials itself (same order as k_finish, so the same rho and beta), and
// workgroup 0 does the bookkeeping of that finish once.  rho itself is stored
// by the update kernel that follows: the workgroups here still read the
// previous one.  On a breakdown every workgroup stops before writing.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_pspmv_rho(Lv<R> L, const R* __restrict__ z, const R* __restrict__ pold,
                                                       R* __restrict__ pnew, R* __restrict__ q,
                                                       const double* __restrict__ prho, int nrho,
                                                       double* __restrict__ ppq, Scal* __restrict__ sc,
                                                       const int* __restrict__ gate) {
  const int gv = *gate_or_zero(gate);
  const int it = sc->it;
  const double rho_prev = sc->rho;
  double pv[kPF];
  load_partials(prho, nrho, pv);
  issue_before(gv);
  issue_before(it);
  issue_before(rho_prev);
  if (gv) return;
  __shared__ double sm[kBlock / kWave];
  const double s = sum_loaded_partials(pv, prho, nrho, sm);
  const bool nonfinite = !(s == s) || s == INFINITY;
  const bool stop = nonfinite || !(s > 0.0);
  const double beta_d = it == 0 ? 0.0 : s / rho_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->started += 1;
    if (nonfinite) { sc->status = -4; sc->converged = 1; }
    else if (stop) { sc->status = 1; sc->converged = 1; }
    sc->beta = beta_d;
  }
  if (stop) return;
  const double acc = pspmv_range(L, z, pold, pnew, q, it == 0, (R)beta_d);
  const double t = block_sum(acc, sm);
  if (threadIdx.x == 0) ppq[blockIdx.x] = t;
}

// x += alpha p, r -= alpha q with partial sums of |r|^2 (gated)
template <typename R>
__global__ void __launch_bounds__(kBlock) k_cg_update_g(R* __restrict__ x, R* __restrict__ r,
                                                         const R* __restrict__ p, const R* __restrict__ q, int n,
                                                         double* __restrict__ part, const Scal* __restrict__ sc,
                                                         const int* __restrict__ gate) {
  const int gv = *gate_or_zero(gate);
  const double alpha_d = sc->alpha;
  issue_before(gv);
  issue_before(alpha_d);
  if (gv) return;
  __shared__ double sm[kBlock / kWave];
  const R alpha = (R)alpha_d;
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    x[c] += alpha * p[c];
    const R v = r[c] - alpha * q[c];
    r[c] = v;
    acc += (double)v * (double)v;
  }
  const double s = block_sum(acc, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p, r -= alpha q with partial sums of |r|^2, the finish of p.q
// folded in: every workgroup sums the r.z and p.q partials itself (same order
// as k_finish, so the same alpha = rho / p.q), workgroup 0 stores rho, alpha
// and the breakdown state once.  On a breakdown every workgroup stops before
// writing.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_update_pq(R* __restrict__ x, R* __restrict__ r, const R* __restrict__ p,
                                                       const R* __restrict__ q, int n, const double* __restrict__ prho,
                                                       int nrho, const double* __restrict__ ppq, int npq,
                                                       double* __restrict__ prr, Scal* __restrict__ sc,
                                                       const int* __restrict__ gate) {
  const int gv = *gate_or_zero(gate);
  const int status = sc->status;
  double pr[kPF], pp[kPF];
  load_partials(prho, nrho, pr);
  load_partials(ppq, npq, pp);
  issue_before(gv);
  issue_before(status);
  if (gv) return;
  __shared__ double sm[kBlock / kWave];
  const double rho = sum_loaded_partials(pr, prho, nrho, sm);
  const double pq = sum_loaded_partials(pp, ppq, npq, sm);
  const bool nonfinite = !(pq == pq) || pq == INFINITY;
  const bool stop = nonfinite || !(pq > 0.0) || status != 0;
  const double alpha_d = stop ? 0.0 : rho / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rho = rho;
    sc->alpha = alpha_d;
    if (nonfinite) { sc->status = -4; sc->converged = 1; }
    else if (stop) { if (status == 0) sc->status = 1; sc->converged = 1; }
  }
  if (stop) return;
  const R alpha = (R)alpha_d;
  double acc = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    x[c] += alpha * p[c];
    const R v = r[c] - alpha * q[c];
    r[c] = v;
    acc += (double)v * (double)v;
  }
  const double t = block_sum(acc, sm);
  if (threadIdx.x == 0) prr[blockIdx.x] = t;
}

__global__ void k_rhs(RhsArgs a) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  int i, j, k;
  cell_ijk(c, a.nx, a.ny, i, j, k);
  double v = a.f[c] * a.vol;
  if (i == 0 && a.bc_type[0] == 1) v += a.tx[(a.nx + 1) * (j + a.ny * k)] * a.bc_value[0];
  if (i == a.nx - 1 && a.bc_type[1] == 1) v += a.tx[a.nx + (a.nx + 1) * (j + a.ny * k)] * a.bc_value[1];
  if (j == 0 && a.bc_type[2] == 1) v += a.ty[i + a.nx * (a.ny + 1) * k] * a.bc_value[2];
  if (j == a.ny - 1 && a.bc_type[3] == 1) v += a.ty[i + a.nx * (a.ny + (a.ny + 1) * k)] * a.bc_value[3];
  if (a.dim == 3) {
    const int plane = a.nx * a.ny;
    if (k == 0 && a.bc_type[4] == 1) v += a.tz[i + a.nx * j] * a.bc_value[4];
    if (k == a.nz - 1 && a.bc_type[5] == 1) v += a.tz[i + a.nx * j + plane * a.nz] * a.bc_value[5];
  }
  a.b[c] = v;
}

// Initial guess: linear ramp between the x-face Dirichlet values (lifting by
// a smooth field matching the boundary data, Section 3) or zero.
__global__ void k_init_x(double* __restrict__ x, int n, int nx, double hx, double Lx, double p0, double p1, int ramp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = c % nx;
  x[c] = ramp ? p0 + (p1 - p0) * ((i + 0.5) * hx) / Lx : 0.0;
}

template <typename R>
__global__ void k_fill(R* __restrict__ a, long long n, R v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = t; c < n; c += stride) a[c] = v;
}

template <typename R>
__global__ void k_copy(const R* __restrict__ a, R* __restrict__ b, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long c = t; c < n; c += stride) b[c] = a[c];
}

// Mixed precision seam: out32 = in64 * scale and out64 = in32 * scale.
__global__ void k_scale_to_f32(const double* __restrict__ a, float* __restrict__ b, int n, const Scal* __restrict__ sc) {
  const double s = sc->rr > 0.0 ? 1.0 / sqrt(sc->rr) : 1.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) b[c] = (float)(a[c] * s);
}
__global__ void k_scale_to_f64(const float* __restrict__ a, double* __restrict__ b, int n, const Scal* __restrict__ sc) {
  const double s = sc->rr > 0.0 ? sqrt(sc->rr) : 1.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) b[c] = (double)a[c] * s;
}

// ---------------------------------------------------------------------------
// Small levels: the inner PCG of level ks and every level below it run in
// ONE workgroup, with the recursion unrolled into a loop over an explicit
// level stack.  No host round trip per iteration: the control flow that the
// paper's level tree describes (dynamic transitions, Section 4) happens on
// the device.
// ---------------------------------------------------------------------------

template <typename R>
struct SmallLevel {
  Lv<R> L;
  Xfer X;                 // to level + 1
  R *x, *r, *z, *p, *q;
  double tol;             // absolute criterion on |r|^2
  int lds_T, lds_z, lds_r, lds_x;  // byte offsets into dynamic LDS, -1 = stays in global memory
};

template <typename R>
struct SmallArgs {
  SmallLevel<R> lv[kMaxLevels];
  int ks, nlev;           // first small level, total levels
  int m, max_inner;
  double rel_floor2;      // (floor)^2 relative to |rhs|^2, 0 = off
  const double* Ainv;
  int ncoarse;
  long long* iters;       // per level, accumulated (device)
  long long* calls;
  int* status;
  const int* gate;
};

template <typename R>
__global__ void __launch_bounds__(1024, 1) k_small_pcg(SmallArgs<R> args) {
  if (args.gate && *args.gate) return;
  __shared__ double sm[1024 / kWave];
  __shared__ double sh_rho[kMaxLevels], sh_rr[kMaxLevels], sh_tol[kMaxLevels];
  __shared__ int sh_it[kMaxLevels];
  __shared__ double sh_g[1024], sh_part[1024];
  __shared__ SmallLevel<R> lv[kMaxLevels];  // level descriptors, LDS-resident for dynamic indexing
  __shared__ long long my_iters[kMaxLevels], my_calls[kMaxLevels];
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const SmallArgs<R>& a = args;
  const int L = a.nlev - 1;  // coarsest index
  if (tid < kMaxLevels) {
    lv[tid] = a.lv[tid];
    my_iters[tid] = 0;
    my_calls[tid] = 0;
  }
  __syncthreads();

  // Stage the face transmissibilities and the smoother's vectors of the
  // levels that fit into LDS: the 2(2m+1) half sweeps per iteration then read
  // LDS instead of L2.  The rhs of level ks arrives in global memory; x of
  // level ks is the result and stays there.
  for (int l = a.ks; l <= L; ++l) {
    const SmallLevel<R>& S = a.lv[l];
    if (S.lds_T >= 0) {
      R* t = reinterpret_cast<R*>(dyn_lds + S.lds_T);
      const int fx = (S.L.nx + 1) * S.L.ny * S.L.nz, fy = S.L.nx * (S.L.ny + 1) * S.L.nz;
      const int fz = S.L.tz ? S.L.nx * S.L.ny * (S.L.nz + 1) : 0;
      for (int e = tid; e < fx; e += nt) t[e] = S.L.tx[e];
      for (int e = tid; e < fy; e += nt) t[fx + e] = S.L.ty[e];
      for (int e = tid; e < fz; e += nt) t[fx + fy + e] = S.L.tz[e];
      if (tid == 0) {
        lv[l].L.tx = t;
        lv[l].L.ty = t + fx;
        if (fz) lv[l].L.tz = t + fx + fy;
      }
    }
    if (S.lds_z >= 0 && tid == 0) lv[l].z = reinterpret_cast<R*>(dyn_lds + S.lds_z);
    if (S.lds_r >= 0) {
      R* rr = reinterpret_cast<R*>(dyn_lds + S.lds_r);
      if (l == a.ks)
        for (int c = tid; c < S.L.n; c += nt) rr[c] = S.r[c];
      if (tid == 0) lv[l].r = rr;
    }
    if (S.lds_x >= 0 && l > a.ks && tid == 0) lv[l].x = reinterpret_cast<R*>(dyn_lds + S.lds_x);
  }
  __syncthreads();
  int status = 0;

  // start the PCG of level k: x = 0, r already holds the rhs.  Returns true if
  // the entry check is already satisfied.
  auto start = [&](int k) -> bool {
    SmallLevel<R>& S = lv[k];
    for (int c = tid; c < S.L.n; c += nt) S.x[c] = R(0);
    double acc = 0.0;
    for (int c = tid; c < S.L.n; c += nt) acc += (double)S.r[c] * (double)S.r[c];
    const double rr = block_sum(acc, sm);
    double tol = S.tol;
    if (a.rel_floor2 > 0.0 && a.rel_floor2 * rr > tol) tol = a.rel_floor2 * rr;
    if (tid == 0) { sh_rr[k] = rr; sh_tol[k] = tol; sh_it[k] = 0; }
    if (tid == 0) my_calls[k] += 1;
    __syncthreads();
    return rr < tol;
  };
  // pre-smoothing of level k from x = 0 (m SGS steps = R,B,R,...,R: 2m+1 half
  // sweeps, repeated colours being idempotent) and g_{k+1} = E^T (r - A z).
  auto pre = [&](int k) {
    SmallLevel<R>& S = lv[k];
    for (int h = 0; h <= 2 * a.m; ++h) {
      gs_half_range(S.L, S.r, S.z, h & 1, h == 0, tid, nt);
      __syncthreads();
    }
    // residual into q (free during the preconditioner), then g = E^T res
    for (int c = tid; c < S.L.n; c += nt) {
      int i, j, kk;
      cell_ijk(c, S.L.nx, S.L.ny, i, j, kk);
      R d, o;
      stencil_at(S.L, S.z, i, j, kk, c, d, o);
      S.q[c] = S.r[c] - (d * S.z[c] - o);
    }
    __syncthreads();
    if (S.X.frac) restrict_frac_range(S.L, S.X, (const R*)S.q, lv[k + 1].r, tid, nt);
    else restrict_stored_range(S.L, S.X, (const R*)S.q, lv[k + 1].r, tid, nt);
    __syncthreads();
  };
  // y = A^-1 g on the coarsest level: the columns of A^-1 are split into
  // nt / nc groups whose partial sums are added in group order.
  auto coarse = [&]() {
    SmallLevel<R>& C = lv[L];
    const int nc = a.ncoarse;
    for (int i = tid; i < nc; i += nt) sh_g[i] = (double)C.r[i];
    __syncthreads();
    const int groups = nc >= nt ? 1 : nt / nc;
    const int per = (nc + groups - 1) / groups;
    if (tid < groups * nc) {
      for (int i = tid % nc; i < nc; i += nt) {
        const int grp = tid / nc;
        const int j0 = grp * per, j1 = j0 + per < nc ? j0 + per : nc;
        double s = 0.0;
        for (int j = j0; j < j1; ++j) s += a.Ainv[(long long)j * nc + i] * sh_g[j];
        sh_part[grp * nc + i] = s;
      }
    }
    __syncthreads();
    for (int i = tid; i < nc; i += nt) {
      double s = 0.0;
      for (int grp = 0; grp < groups; ++grp) s += sh_part[grp * nc + i];
      C.x[i] = (R)s;
    }
    if (tid == 0) my_calls[L] += 1;
    __syncthreads();
  };
  // post-smoothing of level k and one CG step; returns true when level k is done
  auto post_step = [&](int k) -> bool {
    SmallLevel<R>& S = lv[k];
    if (S.X.frac) prolong_frac_range(S.L, S.X, lv[k + 1].x, S.z, tid, nt);
    else prolong_range(S.L, S.X, lv[k + 1].x, S.z, tid, nt);
    __syncthreads();
    for (int h = 0; h <= 2 * a.m; ++h) {
      gs_half_range(S.L, S.r, S.z, h & 1, false, tid, nt);
      __syncthreads();
    }
    // rho = r.z
    double acc = 0.0;
    for (int c = tid; c < S.L.n; c += nt) acc += (double)S.r[c] * (double)S.z[c];
    const double rho = block_sum(acc, sm);
    const int it = sh_it[k];
    if (!(rho == rho) || rho == INFINITY) { status = -4; return true; }
    if (!(rho > 0.0)) return true;  // no further progress in this precision: the level stops
    const R beta = it == 0 ? R(0) : (R)(rho / sh_rho[k]);
    for (int c = tid; c < S.L.n; c += nt) S.p[c] = it == 0 ? S.z[c] : S.z[c] + beta * S.p[c];
    __syncthreads();
    const double pq = block_sum(spmv_range<R, double>(S.L, S.p, S.q, tid, nt), sm);
    if (!(pq == pq) || pq == INFINITY) { status = -4; return true; }
    if (!(pq > 0.0)) return true;
    const R alpha = (R)(rho / pq);
    acc = 0.0;
    for (int c = tid; c < S.L.n; c += nt) {
      S.x[c] += alpha * S.p[c];
      const R v = S.r[c] - alpha * S.q[c];
      S.r[c] = v;
      acc += (double)v * (double)v;
    }
    const double rr = block_sum(acc, sm);
    if (tid == 0) { sh_rho[k] = rho; sh_rr[k] = rr; sh_it[k] = it + 1; my_iters[k] += 1; }
    __syncthreads();
    return rr < sh_tol[k] || it + 1 >= a.max_inner;
  };

  int k = a.ks;
  if (start(k)) goto done;
  for (;;) {
    // descend: begin an iteration at level k
    pre(k);
    if (k + 1 == L) {
      coarse();
    } else {
      ++k;
      if (!start(k)) continue;  // iterate on the deeper level
      --k;                      // deeper level already converged: y = 0
    }
    // ascend: finish iterations up the stack
    for (;;) {
      const bool fin = post_step(k);
      if (status) goto done;
      if (!fin) break;  // next iteration at level k
      if (k == a.ks) goto done;
      --k;
    }
  }
done:
  if (tid == 0) {
    for (int l = 0; l < kMaxLevels; ++l) {
      a.iters[l] += my_iters[l];
      a.calls[l] += my_calls[l];
    }
    if (status) a.status[0] = status;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_face_T(const FaceTArgs& a, hipStream_t s) {
  const long long tot = (long long)(a.nx + 1) * a.ny * a.nz + (long long)a.nx * (a.ny + 1) * a.nz +
                        (a.dim == 3 ? (long long)a.nx * a.ny * (a.nz + 1) : 0);
  hipLaunchKernelGGL(k_face_T, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_check_positive(const double* k, long long n, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_check_positive, dim3(grid_for(n, 2048)), dim3(256), 0, s, k, n, bad);
  return hipGetLastError();
}

hipError_t launch_coarsen(const CoarsenArgs& a, hipStream_t s) {
  int ce[3] = {a.cd[0], a.cd[1], a.cd[2]};
  ce[a.axis] += 1;
  const long long tot = (long long)ce[0] * ce[1] * ce[2];
  if (a.frac)
    hipLaunchKernelGGL(k_coarsen_frac, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_coarsen_axis, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* a, float* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 4096)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

// k_band_inverse with both bands of the factor in LDS for the whole launch
// (2 n (b + 1) doubles) and each wave's column in LDS: no barriers between
// rows.  Same operations, in the same order.
__global__ void __launch_bounds__(256) k_band_inverse_lds(const double* __restrict__ Lb, const double* __restrict__ Lt,
                                                          double* __restrict__ Ainv, int n, int b) {
  extern __shared__ double sh[];
  const int W = b + 1;
  double* lb = sh;
  double* lt = sh + (long long)n * W;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  double* w = sh + 2LL * n * W + (long long)wave * n;
  for (int e = threadIdx.x; e < n * W; e += blockDim.x) {
    lb[e] = Lb[e];
    lt[e] = Lt[e];
  }
  const int c = blockIdx.x * 4 + wave;
  for (int k = lane; k < n; k += kWave) w[k] = 0.0;
  __syncthreads();
  if (c >= n) return;
  double reg = 0.0;
  for (int i = c; i < n; ++i) {
    const int d = (lane - i) & (kWave - 1), k = i - kWave + d;
    const double term = (k >= c && k >= i - b) ? lb[i * W + (k - i + b)] * reg : 0.0;
    const double s = wave_total(term);
    const double wi = ((i == c ? 1.0 : 0.0) - s) / lb[i * W + b];
    if ((i & (kWave - 1)) == lane) {
      reg = wi;
      w[i] = wi;
    }
  }
  reg = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    const int k = i + 1 + ((lane - i - 1) & (kWave - 1));
    const double term = (k <= i + b && k < n) ? lt[i * W + (k - i)] * reg : 0.0;
    const double s = wave_total(term);
    const double xi = (w[i] - s) / lt[i * W];
    if ((i & (kWave - 1)) == lane) {
      reg = xi;
      w[i] = xi;
    }
  }
  for (int k = lane; k < n; k += kWave) Ainv[(long long)c * n + k] = w[k];
}

__global__ void k_pack_sym(const double* __restrict__ Ainv, int n, int NT, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= NT * (NT + 1) / 2 * 256) return;
  const int t = e >> 8, sl = (e >> 4) & 15, c = e & 15;
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int J = t - I * (I + 1) / 2;
  const int i = 16 * I + (sl ^ c), j = 16 * J + c;  // slot sl of column c holds row sl xor c
  out[e] = i < n && j < n ? Ainv[(long long)i * n + j] : 0.0;
}

hipError_t launch_pack_sym(const double* Ainv, int n, int ntile, double* out, hipStream_t s) {
  const int tot = ntile * (ntile + 1) / 2 * 256;
  hipLaunchKernelGGL(k_pack_sym, dim3((tot + 255) / 256), dim3(256), 0, s, Ainv, n, ntile, out);
  return hipGetLastError();
}

hipError_t launch_coarse_factor(const Lv<double>& L, double* A, double* Lrows, double* Ainv, int* status,
                                hipStream_t s) {
  if (L.n > MSCG_COARSE_CAP) return hipErrorInvalidValue;
  const long long nn = (long long)L.n * L.n;
  // bandwidth in natural order; the two band copies of the factor go to Lrows
  const int b = L.nz > 1 ? L.nx * L.ny : (L.ny > 1 ? L.nx : 1);
  if (b <= 64 && 2LL * (b + 1) * L.n <= nn) {
    // factor and inverse each with their band in LDS where it fits
    const int W = b + 1;
    const size_t f_lds = (size_t)L.n * W * sizeof(double);
    const size_t i_lds = (2 * (size_t)L.n * W + 4 * (size_t)L.n) * sizeof(double);
    static bool attr = false;
    if (!attr) {
      hipError_t e = hipFuncSetAttribute((const void*)k_chol_band_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)kBandLds);
      if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_band_inverse_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)kBandLds);
      if (e != hipSuccess) return e;
      attr = true;
    }
    double* Lb = Lrows;
    double* Lt = Lrows + (long long)L.n * W;
    if (f_lds <= kBandLds) {
      hipLaunchKernelGGL(k_chol_band_lds, dim3(1), dim3(256), f_lds, s, L, b, Lb, Lt, status);
    } else {
      hipLaunchKernelGGL(k_dense_assemble, dim3((L.n + 255) / 256), dim3(256), 0, s, L, A);
      hipLaunchKernelGGL(k_chol_band, dim3(1), dim3(1024), (size_t)W * W * sizeof(double), s, A, L.n, b, Lb, Lt,
                         status);
    }
    if (i_lds <= kBandLds)
      hipLaunchKernelGGL(k_band_inverse_lds, dim3((L.n + 3) / 4), dim3(256), i_lds, s, Lb, Lt, Ainv, L.n, b);
    else
      hipLaunchKernelGGL(k_band_inverse, dim3((L.n + 3) / 4), dim3(256), 0, s, Lb, Lt, Ainv, L.n, b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_dense_assemble, dim3((L.n + 255) / 256), dim3(256), 0, s, L, A);
  hipLaunchKernelGGL(k_chol_factor, dim3(1), dim3(1024), 0, s, A, L.n, status);
  hipLaunchKernelGGL(k_factor_rows, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, A, Lrows, L.n);
  hipLaunchKernelGGL(k_chol_inverse, dim3((L.n + 3) / 4), dim3(256), 0, s, A, Lrows, Ainv, L.n);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_spmv(const Lv<R>& L, const R* x, R* y, double* part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv_dot<R>, dim3(nparts), dim3(kBlock), 0, s, L, x, y, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_residual(const Lv<R>& L, const R* b, const R* x, R* r, double* part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_residual<R>, dim3(nparts), dim3(kBlock), 0, s, L, b, x, r, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_dot(const R* a, const R* b, int n, double* part, int nparts, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<R>, dim3(nparts), dim3(kBlock), 0, s, a, b, n, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_update_p(const R* z, R* p, int n, const Scal* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_update_p<R>, dim3(grid_for(n)), dim3(kBlock), 0, s, z, p, n, sc);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_update(R* x, R* r, const R* p, const R* q, int n, const Scal* sc, double* part, int nparts,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update<R>, dim3(nparts), dim3(kBlock), 0, s, x, r, p, q, n, sc, part);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gs_half(const Lv<R>& L, const R* r, R* x, int colour, int first, hipStream_t s, const int* gate) {
  const long long tot = (long long)((L.nx + 1) / 2) * L.ny * L.nz;
  hipLaunchKernelGGL(k_gs_half<R>, dim3(grid_for(tot, 1 << 20)), dim3(kBlock), 0, s, L, r, x, colour, first, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_mjac_step(const Lv<R>& L, const R* r, const R* xin, R* xout, int first, hipStream_t s,
                            const int* gate) {
  hipLaunchKernelGGL(k_mjac_step<R>, dim3(grid_for(L.n, 1 << 20)), dim3(kBlock), 0, s, L, r, xin, xout, first, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_restrict(const Lv<R>& F, const Xfer& X, const R* r, const R* x, R* g, hipStream_t s) {
  if (X.frac) return hipErrorNotSupported;  // the fractional path restricts a stored residual
  const long long nc = (long long)X.cnx * X.cny * X.cnz;
  hipLaunchKernelGGL(k_restrict<R>, dim3(grid_for(nc, 1 << 20)), dim3(kBlock), 0, s, F, X, r, x, g);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_residual_restrict(const Lv<R>& F, const Xfer& X, const R* r, const R* x, R* tmp, R* g,
                                    hipStream_t s, const int* gate) {
  const long long nc = (long long)X.cnx * X.cny * X.cnz;
  hipLaunchKernelGGL(k_residual_nodot<R>, dim3(grid_for(F.n, 1 << 20)), dim3(kBlock), 0, s, F, r, x, tmp, gate);
  if (X.frac) {
    hipLaunchKernelGGL(k_restrict_frac<R>, dim3((unsigned)((nc + 63) / 64)), dim3(64), 0, s, F, X, (const R*)tmp, g,
                       gate);
    return hipGetLastError();
  }
  // one thread per coarse cell; small coarse grids use 64-thread blocks to spread over more CUs
  if (nc < 65536)
    hipLaunchKernelGGL(k_restrict_stored<R>, dim3((unsigned)((nc + 63) / 64)), dim3(64), 0, s, F, X, (const R*)tmp, g,
                       gate);
  else
    hipLaunchKernelGGL(k_restrict_stored<R>, dim3(grid_for(nc, 1 << 20)), dim3(kBlock), 0, s, F, X,
                       (const R*)tmp, g, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_prolong(const Lv<R>& F, const Xfer& X, const R* y, R* x, hipStream_t s, const int* gate) {
  if (X.frac)
    hipLaunchKernelGGL(k_prolong_frac<R>, dim3(grid_for(F.n, 1 << 20)), dim3(kBlock), 0, s, F, X, y, x, gate);
  else
    if (F.nz == 1 && X.cnz == 1 && !F.tz && F.ny <= 65535)
      hipLaunchKernelGGL(k_prolong_2d<R>, dim3((F.nx + kBlock - 1) / kBlock, F.ny), dim3(kBlock), 0, s, F, X, y, x, gate);
    else
      hipLaunchKernelGGL(k_prolong<R>, dim3(grid_for(F.n, 1 << 20)), dim3(kBlock), 0, s, F, X, y, x, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_coarse_solve(const double* Ainv, const R* g, R* y, int n, hipStream_t s, const int* gate) {
  constexpr int kRowsPerBlock = kBlock / kWave;
  hipLaunchKernelGGL(k_coarse_solve<R>, dim3((n + kRowsPerBlock - 1) / kRowsPerBlock), dim3(kBlock), 0, s, Ainv, g, y,
                     n, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_dot_fin(const R* a, const R* b, int n, double* part, int nparts, Scal* sc, int op, hipStream_t s,
                          const int* gate) {
  hipLaunchKernelGGL(k_dot_g<R>, dim3(nparts), dim3(kBlock), 0, s, a, b, n, part, gate);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, (const double*)part, nparts, sc, op, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pspmv_fin(const Lv<R>& L, const R* z, const R* pold, R* pnew, R* q, double* part, int nparts,
                            Scal* sc, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_pspmv<R>, dim3(nparts), dim3(kBlock), 0, s, L, z, pold, pnew, q, part, (const Scal*)sc, gate);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, (const double*)part, nparts, sc, (int)kOpPq, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_cg_update_fin(R* x, R* r, const R* p, const R* q, int n, double* part, int nparts, Scal* sc,
                                hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_cg_update_g<R>, dim3(nparts), dim3(kBlock), 0, s, x, r, p, q, n, part, (const Scal*)sc, gate);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, (const double*)part, nparts, sc, (int)kOpRr, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_dot_part(const R* a, const R* b, int n, double* part, int nparts, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_dot_g<R>, dim3(nparts), dim3(kBlock), 0, s, a, b, n, part, gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pspmv_rho(const Lv<R>& L, const R* z, const R* pold, R* pnew, R* q, const double* prho, int nrho,
                            double* ppq, int nparts, Scal* sc, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_pspmv_rho<R>, dim3(nparts), dim3(kBlock), 0, s, L, z, pold, pnew, q, prho, nrho, ppq, sc,
                     gate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_update_pq_fin(R* x, R* r, const R* p, const R* q, int n, const double* prho, int nrho,
                                const double* ppq, double* prr, int nparts, Scal* sc, hipStream_t s,
                                const int* gate) {
  hipLaunchKernelGGL(k_update_pq<R>, dim3(nparts), dim3(kBlock), 0, s, x, r, p, q, n, prho, nrho, ppq, nparts, prr,
                     sc, gate);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, (const double*)prr, nparts, sc, (int)kOpRr, gate);
  return hipGetLastError();
}

hipError_t launch_finish(const double* part, int nparts, Scal* sc, int op, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kBlock), 0, s, part, nparts, sc, op, gate);
  return hipGetLastError();
}

hipError_t launch_rhs(const RhsArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_x(double* x, int n, int nx, double hx, double Lx, double p0, double p1, int ramp,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_init_x, dim3((n + 255) / 256), dim3(256), 0, s, x, n, nx, hx, Lx, p0, p1, ramp);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fill(R* a, long long n, R v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<R>, dim3(grid_for(n, 4096)), dim3(256), 0, s, a, n, v);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_copy(const R* a, R* b, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<R>, dim3(grid_for(n, 4096)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_scale_to_f32(const double* a, float* b, int n, const Scal* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, n, sc);
  return hipGetLastError();
}

hipError_t launch_scale_to_f64(const float* a, double* b, int n, const Scal* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_to_f64, dim3(grid_for(n)), dim3(kBlock), 0, s, a, b, n, sc);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_small_pcg(const SmallDesc<R>& d, hipStream_t s) {
  SmallArgs<R> a{};
  for (int l = 0; l < d.nlev; ++l) {
    a.lv[l].L = d.L[l];
    a.lv[l].X = d.X[l];
    a.lv[l].x = d.x[l];
    a.lv[l].r = d.r[l];
    a.lv[l].z = d.z[l];
    a.lv[l].p = d.p[l];
    a.lv[l].q = d.q[l];
    a.lv[l].tol = d.tol[l];
  }
  a.ks = d.ks;
  a.nlev = d.nlev;
  a.m = d.m;
  a.max_inner = d.max_inner;
  a.rel_floor2 = d.rel_floor2;
  a.Ainv = d.Ainv;
  a.ncoarse = d.ncoarse;
  a.iters = d.iters;
  a.calls = d.calls;
  a.status = d.status;
  a.gate = d.gate;
  // LDS plan: per level from the top small level down, faces then z then r;
  // then the coarsest level's rhs and solution; each array only if it fits.
  size_t off = 0;
  auto fit = [&](size_t bytes) -> int {
    bytes = (bytes + 15) & ~(size_t)15;
    if (off + bytes > kSmallLdsBytes) return -1;
    const int o = (int)off;
    off += bytes;
    return o;
  };
  for (int l = 0; l < kMaxLevels; ++l) a.lv[l].lds_T = a.lv[l].lds_z = a.lv[l].lds_r = a.lv[l].lds_x = -1;
  const int Lc = d.nlev - 1;
  for (int l = d.ks; l < Lc; ++l) {
    const Lv<R>& V = d.L[l];
    const size_t faces = (size_t)(V.nx + 1) * V.ny * V.nz + (size_t)V.nx * (V.ny + 1) * V.nz +
                         (V.tz ? (size_t)V.nx * V.ny * (V.nz + 1) : 0);
    a.lv[l].lds_T = fit(faces * sizeof(R));
    a.lv[l].lds_z = fit((size_t)V.n * sizeof(R));
    a.lv[l].lds_r = fit((size_t)V.n * sizeof(R));
  }
  a.lv[Lc].lds_r = fit((size_t)d.L[Lc].n * sizeof(R));
  a.lv[Lc].lds_x = fit((size_t)d.L[Lc].n * sizeof(R));
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_small_pcg<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kSmallLdsBytes);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_small_pcg<R>, dim3(1), dim3(1024), off, s, a);
  return hipGetLastError();
}

#define MSCG_INST(R)                                                                                              \
  template hipError_t launch_spmv<R>(const Lv<R>&, const R*, R*, double*, int, hipStream_t);                      \
  template hipError_t launch_residual<R>(const Lv<R>&, const R*, const R*, R*, double*, int, hipStream_t);        \
  template hipError_t launch_dot<R>(const R*, const R*, int, double*, int, hipStream_t);                          \
  template hipError_t launch_update_p<R>(const R*, R*, int, const Scal*, hipStream_t);                            \
  template hipError_t launch_cg_update<R>(R*, R*, const R*, const R*, int, const Scal*, double*, int, hipStream_t); \
  template hipError_t launch_gs_half<R>(const Lv<R>&, const R*, R*, int, int, hipStream_t, const int*);          \
  template hipError_t launch_mjac_step<R>(const Lv<R>&, const R*, const R*, R*, int, hipStream_t, const int*);    \
  template hipError_t launch_restrict<R>(const Lv<R>&, const Xfer&, const R*, const R*, R*, hipStream_t);         \
  template hipError_t launch_residual_restrict<R>(const Lv<R>&, const Xfer&, const R*, const R*, R*, R*, hipStream_t, \
                                                  const int*);                                                     \
  template hipError_t launch_prolong<R>(const Lv<R>&, const Xfer&, const R*, R*, hipStream_t, const int*);        \
  template hipError_t launch_coarse_solve<R>(const double*, const R*, R*, int, hipStream_t, const int*);          \
  template hipError_t launch_dot_fin<R>(const R*, const R*, int, double*, int, Scal*, int, hipStream_t,          \
                                        const int*);                                                               \
  template hipError_t launch_pspmv_fin<R>(const Lv<R>&, const R*, const R*, R*, R*, double*, int, Scal*,         \
                                          hipStream_t, const int*);                                                \
  template hipError_t launch_cg_update_fin<R>(R*, R*, const R*, const R*, int, double*, int, Scal*, hipStream_t, \
                                              const int*);                                                         \
  template hipError_t launch_dot_part<R>(const R*, const R*, int, double*, int, hipStream_t, const int*);       \
  template hipError_t launch_pspmv_rho<R>(const Lv<R>&, const R*, const R*, R*, R*, const double*, int, double*, \
                                          int, Scal*, hipStream_t, const int*);                                    \
  template hipError_t launch_update_pq_fin<R>(R*, R*, const R*, const R*, int, const double*, int, const double*, \
                                              double*, int, Scal*, hipStream_t, const int*);                      \
  template hipError_t launch_fill<R>(R*, long long, R, hipStream_t);                                              \
  template hipError_t launch_copy<R>(const R*, R*, long long, hipStream_t);                                       \
  template hipError_t launch_small_pcg<R>(const SmallDesc<R>&, hipStream_t);

MSCG_INST(double)
MSCG_INST(float)
template hipError_t launch_fill<int>(int*, long long, int, hipStream_t);
template hipError_t launch_fill<long long>(long long*, long long, long long, hipStream_t);

}  // namespace mscg
