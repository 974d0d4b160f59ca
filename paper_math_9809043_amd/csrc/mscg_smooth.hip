// mscg_smooth.hip -- temporally blocked red-black smoothing for 2-D levels.
//
// m symmetric Gauss-Seidel steps (eq. 2.3 splitting, Section 3) are 2m+1
// red-black half sweeps.  Instead of one grid-wide launch per half sweep, each
// workgroup loads a tile of TW x TH cells plus a halo of H = 2m+1 cells (r,
// the face transmissibilities and, after the coarse correction, z) into LDS,
// runs all 2m+1 half sweeps there, and writes back the tile.  A half sweep
// moves information by one cell, so after 2m+1 of them the tile's values are
// exactly those of the global sweeps; halo cells are scratch.  Neighbours
// outside the loaded region contribute nothing (their influence cannot reach
// the tile).  The post-smoothing variant also applies the prolongation
// z = z_pre + E y while loading.
#include <hip/hip_runtime.h>

#include "mscg_kernels.h"

namespace mscg {

namespace {

constexpr int kTW = 64, kTH = 32;       // tile
constexpr int kBX = 64, kBY = 8;        // threads: 64 x 8 = 512

template <typename R, bool POST>
__global__ void __launch_bounds__(kBX* kBY) k_smooth_tile(Lv<R> L, Xfer X, const R* __restrict__ r,
                                                           const R* __restrict__ zin, const R* __restrict__ y,
                                                           R* __restrict__ zout, int halo, int nsweep) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int nx = L.nx, ny = L.ny;
  const int x0 = blockIdx.x * kTW, y0 = blockIdx.y * kTH;
  const int rx0 = max(x0 - halo, 0), ry0 = max(y0 - halo, 0);
  const int rx1 = min(x0 + kTW + halo, nx), ry1 = min(y0 + kTH + halo, ny);
  const int RW = rx1 - rx0, RH = ry1 - ry0;
  const int MW = kTW + 2 * halo;  // LDS row pitch (cells)
  R* zs = reinterpret_cast<R*>(lds);
  R* rs = zs + (size_t)MW * (kTH + 2 * halo);
  R* txs = rs + (size_t)MW * (kTH + 2 * halo);         // (RH) rows of (RW + 1) faces, pitch MW + 1
  R* tys = txs + (size_t)(MW + 1) * (kTH + 2 * halo);  // (RH + 1) rows of RW faces, pitch MW
  const int tx = threadIdx.x % kBX, ty = threadIdx.x / kBX;

  // load the region
  for (int lj = ty; lj < RH; lj += kBY) {
    const int j = ry0 + lj;
    for (int li = tx; li < RW; li += kBX) {
      const int i = rx0 + li;
      const int c = i + nx * j;
      rs[lj * MW + li] = r[c];
      if (POST) {
        int I0, I1, J0, J1;
        R wi0, wi1, wj0, wj1;
        ext_weights<R>(i, X.sx, X.cnx, X.interp, I0, wi0, I1, wi1);
        ext_weights<R>(j, X.sy, X.cny, X.interp, J0, wj0, J1, wj1);
        // same products and order as the grid-wide prolongation
        R v = R(0);
        const int Js[2] = {J0, J1};
        const R wj[2] = {wj0, wj1};
        for (int b = 0; b < 2; ++b) {
          if (wj[b] == R(0)) continue;
          if (wi0 != R(0)) v += (R(1) * wj[b] * wi0) * y[I0 + X.cnx * Js[b]];
          if (wi1 != R(0)) v += (R(1) * wj[b] * wi1) * y[I1 + X.cnx * Js[b]];
        }
        zs[lj * MW + li] = zin[c] + v;
      }
    }
    for (int li = tx; li <= RW; li += kBX) txs[lj * (MW + 1) + li] = L.tx[(rx0 + li) + (nx + 1) * j];
  }
  for (int lj = ty; lj <= RH; lj += kBY)
    for (int li = tx; li < RW; li += kBX) tys[lj * MW + li] = L.ty[(rx0 + li) + nx * (ry0 + lj)];
  __syncthreads();

  // 2m+1 half sweeps: colour of cell (i, j) is (i + j) & 1, red first
  for (int h = 0; h < nsweep; ++h) {
    const int colour = h & 1;
    const bool first = !POST && h == 0;
    for (int lj = ty; lj < RH; lj += kBY) {
      const int j = ry0 + lj;
      // first local column of this colour in the row
      const int start = ((rx0 + j + colour) & 1);
      for (int li = start + 2 * tx; li < RW; li += 2 * kBX) {
        const int i = rx0 + li;
        const R tw = txs[lj * (MW + 1) + li], te = txs[lj * (MW + 1) + li + 1];
        const R ts = tys[lj * MW + li], tn = tys[(lj + 1) * MW + li];
        const R d = tw + te + ts + tn;
        R o = R(0);
        if (!first) {
          if (i > 0 && li > 0) o += tw * zs[lj * MW + li - 1];
          if (i < nx - 1 && li < RW - 1) o += te * zs[lj * MW + li + 1];
          if (j > 0 && lj > 0) o += ts * zs[(lj - 1) * MW + li];
          if (j < ny - 1 && lj < RH - 1) o += tn * zs[(lj + 1) * MW + li];
        }
        zs[lj * MW + li] = (rs[lj * MW + li] + o) / d;
      }
    }
    __syncthreads();
  }

  // write the tile
  for (int lj = ty; lj < kTH; lj += kBY) {
    const int j = y0 + lj;
    if (j >= ny) break;
    for (int li = tx; li < kTW; li += kBX) {
      const int i = x0 + li;
      if (i >= nx) break;
      zout[i + nx * j] = zs[(j - ry0) * MW + (i - rx0)];
    }
  }
}

}  // namespace

size_t smooth_tile_lds_bytes(int halo, size_t elem) {
  const size_t MW = kTW + 2 * halo, MH = kTH + 2 * halo;
  return elem * (MW * MH * 2 + (MW + 1) * MH + MW * (MH + 1));
}

template <typename R>
hipError_t launch_smooth_tile(const Lv<R>& L, const Xfer* X, const R* r, const R* zin, const R* y, R* zout,
                              int m, hipStream_t s) {
  if (L.tz || L.nz != 1) return hipErrorNotSupported;
  const int halo = 2 * m + 1;
  const size_t bytes = smooth_tile_lds_bytes(halo, sizeof(R));
  if (bytes > 156 * 1024) return hipErrorNotSupported;
  static bool attr[2][2] = {{false, false}, {false, false}};
  const int ri = sizeof(R) == 8 ? 1 : 0, pi = X ? 1 : 0;
  const void* fn = X ? (const void*)k_smooth_tile<R, true> : (const void*)k_smooth_tile<R, false>;
  if (!attr[ri][pi]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    if (e != hipSuccess) return e;
    attr[ri][pi] = true;
  }
  const dim3 grid((L.nx + kTW - 1) / kTW, (L.ny + kTH - 1) / kTH);
  const dim3 block(kBX * kBY);
  if (X)
    hipLaunchKernelGGL((k_smooth_tile<R, true>), grid, block, bytes, s, L, *X, r, zin, y, zout, halo, 2 * m + 1);
  else
    hipLaunchKernelGGL((k_smooth_tile<R, false>), grid, block, bytes, s, L, Xfer{}, r, zin, y, zout, halo, 2 * m + 1);
  return hipGetLastError();
}

template hipError_t launch_smooth_tile<double>(const Lv<double>&, const Xfer*, const double*, const double*,
                                               const double*, double*, int, hipStream_t);
template hipError_t launch_smooth_tile<float>(const Lv<float>&, const Xfer*, const float*, const float*,
                                              const float*, float*, int, hipStream_t);

}  // namespace mscg
