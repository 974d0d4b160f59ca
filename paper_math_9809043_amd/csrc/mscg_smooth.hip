// mscg_smooth.hip -- temporally blocked red-black smoothing for 2-D levels.
//
// m symmetric Gauss-Seidel steps (eq. 2.3 splitting, Section 3) are 2m+1
// red-black half sweeps.  Instead of one grid-wide launch per half sweep, each
// workgroup takes a tile of TW x TH cells plus a halo of H = 2m+1 cells, runs
// all 2m+1 half sweeps on it, and writes back the tile.  A half sweep moves
// information by one cell, so after 2m+1 of them the tile's values equal those
// of the grid-wide sweeps; halo cells are scratch.  Neighbours outside the
// loaded region contribute nothing (their influence cannot reach the tile).
//
// Layout: thread (k, row group) owns the k-th red and the k-th black cell of
// each of its rows and keeps their four neighbour coefficients (zero across
// the domain or region edge), inverse diagonal and r in registers, all loaded in one
// batch.  z lives in LDS split by colour, so the cells a half sweep updates
// are contiguous and their neighbours are contiguous in the other colour's
// array.  The update is z = (r + sum T z_nb) * (1 / d) with the terms in the
// same order as the grid-wide half sweep, so both give the same bits.  The
// post-smoothing variant also applies the prolongation z = z_pre + E y while
// loading.
#include <hip/hip_runtime.h>

#include "mscg_kernels.h"

namespace mscg {

namespace {

constexpr int kHalo = 9;  // 2m + 1 for m = 4

// Workgroups are handed to the chip's 8 XCDs (each with its own L2) in turn by
// linear workgroup id.  Renumbering the tiles so that XCD x gets the x-th
// contiguous run of tiles in row-major order keeps horizontally and
// vertically adjacent tiles, whose halos overlap, on one L2.  The map is a
// bijection of [0, T): the d-th workgroup sent to XCD x takes tile
// x * (T / 8) + min(x, T % 8) + d.
constexpr int kXcds = 8;
__device__ __forceinline__ void xcd_tile(int& bx, int& by) {
  const int gx = gridDim.x;
  const int T = gx * gridDim.y;
  const int lin = blockIdx.x + gx * blockIdx.y;
  const int x = lin % kXcds, d = lin / kXcds;
  const int t = x * (T / kXcds) + min(x, T % kXcds) + d;
  by = t / gx;
  bx = t - by * gx;
}

// POST: continue from zin (post-smoothing); PROL: apply the prolongation
// zin + E y while loading (else zin already holds it).
template <typename R, bool POST, int TW, int TH, int BX, int BY, bool PROL = POST>
__global__ void __launch_bounds__(BX* BY, (BX * BY == 256 && sizeof(R) == 8) ? 4 : 1) k_smooth_tile(Lv<R> L, Xfer X, const R* __restrict__ r,
                                                         const R* __restrict__ zin, const R* __restrict__ y,
                                                         R* __restrict__ zout, const int* __restrict__ gate,
                                                         double* __restrict__ part) {
  const int gv = gate ? *gate : 0;
  constexpr int MW = TW + 2 * kHalo, MH = TH + 2 * kHalo;
  constexpr int HW = (MW + 1) / 2;         // cells of one colour per region row, upper bound
  constexpr int NR = (MH + BY - 1) / BY;   // region rows per thread
  static_assert(HW <= BX, "tile too wide for the thread layout");
  __shared__ R zc[2][MH][HW];              // [colour][region row][index within the colour]
  const int nx = L.nx, ny = L.ny;
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int x0 = tbx * TW, y0 = tby * TH;
  const int rx0 = max(x0 - kHalo, 0), ry0 = max(y0 - kHalo, 0);
  const int RW = min(x0 + TW + kHalo, nx) - rx0, RH = min(y0 + TH + kHalo, ny) - ry0;
  const int k = threadIdx.x % BX, ty = threadIdx.x / BX;

  // Small tiles (latency-bound levels), the pre-smoother and tiles with at
  // most two region rows per thread issue every load before the first wait;
  // the post-smoother on the other large tiles, which runs at its register
  // limit, stages the coarse patch first (gate, patch, then the coefficients:
  // three round trips, fewer live registers).
  constexpr bool kEarly = !POST || TW * TH <= 196 || BY >= 16;
  static_assert(kEarly || PROL == POST, "the staged-patch path always applies the prolongation");
  R cw[NR][2], ce[NR][2], cs[NR][2], cn[NR][2], dg[NR][2], rr[NR][2];
  if constexpr (kEarly) {
    // Region cell (li, lj) has colour (rx0 + li + ry0 + lj) & 1 and index li >> 1
    // within its colour.  The thread's cell of colour c in row lj is
    // li = 2k + ((rx0 + ry0 + lj + c) & 1).
    R zp[NR][2];
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int lj = ty + BY * b;
      const int j = ry0 + lj;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int li = 2 * k + ((rx0 + ry0 + lj + c) & 1);
        cw[b][c] = ce[b][c] = cs[b][c] = cn[b][c] = rr[b][c] = zp[b][c] = R(0);
        if (lj < RH && li < RW) {
          const int i = rx0 + li;
          const int fx = i + (nx + 1) * j, fy = i + nx * j;
          cw[b][c] = L.tx[fx];
          ce[b][c] = L.tx[fx + 1];
          cs[b][c] = L.ty[fy];
          cn[b][c] = L.ty[fy + nx];
          rr[b][c] = r[i + nx * j];
          if (POST) zp[b][c] = zin[i + nx * j];
        }
      }
    }
    // post-smoothing: the coarse values the region's prolongation reads are
    // staged in LDS when the patch fits (factors >= 2 per axis)
    constexpr int kPW = MW / 2 + 2, kPH = MH / 2 + 2;
    constexpr int kYPer = PROL ? (kPW * kPH + BX * BY - 1) / (BX * BY) : 1;
    __shared__ R ys[PROL ? kPW * kPH : 1];
    int xI0[2], xI1[2];
    R xw0[2], xw1[2];
    int pI = 0, pJ = 0, PW = 0, PH = 0;
    bool staged = false;
    R yv_[kYPer];
    if (PROL) {
      int a0, a1, b0, b1;
      R u0, u1;
      ext_weights<R>(rx0, X.sx, X.cnx, X.interp, a0, u0, a1, u1);
      pI = a0;
      ext_weights<R>(rx0 + RW - 1, X.sx, X.cnx, X.interp, a0, u0, a1, u1);
      PW = a1 - pI + 1;
      ext_weights<R>(ry0, X.sy, X.cny, X.interp, b0, u0, b1, u1);
      pJ = b0;
      ext_weights<R>(ry0 + RH - 1, X.sy, X.cny, X.interp, b0, u0, b1, u1);
      PH = b1 - pJ + 1;
      staged = PW <= kPW && PH <= kPH;  // the same for every thread
#pragma unroll
      for (int u = 0; u < kYPer; ++u) {
        const int e = threadIdx.x + u * BX * BY;
        const int jj = staged ? e / PW : 0, ii = staged ? e - jj * PW : 0;
        yv_[u] = (staged && e < PW * PH) ? y[(pI + ii) + X.cnx * (pJ + jj)] : R(0);
      }
    }
    asm volatile("" ::"v"(gv));  // the gate's wait comes after every load is issued
    if (gv) return;
    if (PROL) {
#pragma unroll
      for (int q = 0; q < 2; ++q) ext_weights<R>(rx0 + 2 * k + q, X.sx, X.cnx, X.interp, xI0[q], xw0[q], xI1[q], xw1[q]);
      if (staged) {
#pragma unroll
        for (int u = 0; u < kYPer; ++u) {
          const int e = threadIdx.x + u * BX * BY;
          if (e < PW * PH) ys[e] = yv_[u];
        }
        __syncthreads();
      }
    }
    auto yv = [&](int I, int J) { return staged ? ys[(J - pJ) * PW + (I - pI)] : y[I + X.cnx * J]; };
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int lj = ty + BY * b;
      const int j = ry0 + lj;
      int J0 = 0, J1 = 0;
      R wj0 = R(0), wj1 = R(0);
      if (PROL && lj < RH) ext_weights<R>(j, X.sy, X.cny, X.interp, J0, wj0, J1, wj1);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q = (rx0 + ry0 + lj + c) & 1;
        const int li = 2 * k + q;
        dg[b][c] = R(1);  // inverse diagonal
        if (lj < RH && li < RW) {
          const int i = rx0 + li;
          const R tw = cw[b][c], te = ce[b][c], ts = cs[b][c], tn = cn[b][c];
          dg[b][c] = R(1) / (tw + te + ts + tn);
          if (!(i > 0 && li > 0)) cw[b][c] = R(0);
          if (!(i < nx - 1 && li < RW - 1)) ce[b][c] = R(0);
          if (!(j > 0 && lj > 0)) cs[b][c] = R(0);
          if (!(j < ny - 1 && lj < RH - 1)) cn[b][c] = R(0);
          if (PROL) {
            // same products, in the same order, as the grid-wide prolongation
            R v = R(0);
            if (wj0 != R(0)) {
              if (xw0[q] != R(0)) v += (R(1) * wj0 * xw0[q]) * yv(xI0[q], J0);
              if (xw1[q] != R(0)) v += (R(1) * wj0 * xw1[q]) * yv(xI1[q], J0);
            }
            if (wj1 != R(0)) {
              if (xw0[q] != R(0)) v += (R(1) * wj1 * xw0[q]) * yv(xI0[q], J1);
              if (xw1[q] != R(0)) v += (R(1) * wj1 * xw1[q]) * yv(xI1[q], J1);
            }
            zc[c][lj][k] = zp[b][c] + v;
          } else if (POST) {
            zc[c][lj][k] = zp[b][c];
          }
        }
      }
    }
    __syncthreads();
  } else {
    if (gv) return;
    // Region cell (li, lj) has colour (rx0 + li + ry0 + lj) & 1 and index li >> 1
    // within its colour.  The thread's cell of colour c in row lj is
    // li = 2k + ((rx0 + ry0 + lj + c) & 1).
    int xI0[2], xI1[2];
    R xw0[2], xw1[2];
    // post-smoothing: the coarse values the region's prolongation reads are
    // staged in LDS when the patch fits (factors >= 2 per axis)
    constexpr int kPW = MW / 2 + 2, kPH = MH / 2 + 2;
    __shared__ R ys[POST ? kPW * kPH : 1];
    int pI = 0, pJ = 0, PW = 0;
    bool staged = false;
    if (POST) {
#pragma unroll
      for (int q = 0; q < 2; ++q) ext_weights<R>(rx0 + 2 * k + q, X.sx, X.cnx, X.interp, xI0[q], xw0[q], xI1[q], xw1[q]);
      int a0, a1, b0, b1;
      R u0, u1;
      ext_weights<R>(rx0, X.sx, X.cnx, X.interp, a0, u0, a1, u1);
      pI = a0;
      ext_weights<R>(rx0 + RW - 1, X.sx, X.cnx, X.interp, a0, u0, a1, u1);
      PW = a1 - pI + 1;
      ext_weights<R>(ry0, X.sy, X.cny, X.interp, b0, u0, b1, u1);
      pJ = b0;
      ext_weights<R>(ry0 + RH - 1, X.sy, X.cny, X.interp, b0, u0, b1, u1);
      const int PH = b1 - pJ + 1;
      staged = PW <= kPW && PH <= kPH;  // the same for every thread
      if (staged) {
        for (int e = threadIdx.x; e < PW * PH; e += BX * BY) {
          const int jj = e / PW, ii = e - jj * PW;
          ys[e] = y[(pI + ii) + X.cnx * (pJ + jj)];
        }
        __syncthreads();
      }
    }
    auto yv = [&](int I, int J) { return staged ? ys[(J - pJ) * PW + (I - pI)] : y[I + X.cnx * J]; };
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int lj = ty + BY * b;
      const int j = ry0 + lj;
      int J0 = 0, J1 = 0;
      R wj0 = R(0), wj1 = R(0);
      if (POST && lj < RH) ext_weights<R>(j, X.sy, X.cny, X.interp, J0, wj0, J1, wj1);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q = (rx0 + ry0 + lj + c) & 1;
        const int li = 2 * k + q;
        cw[b][c] = ce[b][c] = cs[b][c] = cn[b][c] = R(0);
        dg[b][c] = R(1);  // inverse diagonal
        rr[b][c] = R(0);
        if (lj < RH && li < RW) {
          const int i = rx0 + li;
          const int fx = i + (nx + 1) * j, fy = i + nx * j;
          const R tw = L.tx[fx], te = L.tx[fx + 1], ts = L.ty[fy], tn = L.ty[fy + nx];
          dg[b][c] = R(1) / (tw + te + ts + tn);
          if (i > 0 && li > 0) cw[b][c] = tw;
          if (i < nx - 1 && li < RW - 1) ce[b][c] = te;
          if (j > 0 && lj > 0) cs[b][c] = ts;
          if (j < ny - 1 && lj < RH - 1) cn[b][c] = tn;
          rr[b][c] = r[i + nx * j];
          if (POST) {
            // same products, in the same order, as the grid-wide prolongation
            R v = R(0);
            if (wj0 != R(0)) {
              if (xw0[q] != R(0)) v += (R(1) * wj0 * xw0[q]) * yv(xI0[q], J0);
              if (xw1[q] != R(0)) v += (R(1) * wj0 * xw1[q]) * yv(xI1[q], J0);
            }
            if (wj1 != R(0)) {
              if (xw0[q] != R(0)) v += (R(1) * wj1 * xw0[q]) * yv(xI0[q], J1);
              if (xw1[q] != R(0)) v += (R(1) * wj1 * xw1[q]) * yv(xI1[q], J1);
            }
            zc[c][lj][k] = zin[i + nx * j] + v;
          }
        }
      }
    }
    __syncthreads();
  }
  // 2m+1 half sweeps, red (colour 0) first; neighbours are of the other
  // colour: (li - 1, li + 1) in the row, li in the rows above and below
  for (int h = 0; h < kHalo; ++h) {
    const int c = h & 1, oc = c ^ 1;
    const bool first = !POST && h == 0;
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int lj = ty + BY * b;
      const int li = 2 * k + ((rx0 + ry0 + lj + c) & 1);
      if (lj < RH && li < RW) {
        R o = R(0);
        if (!first) {
          const int w = li > 0 ? (li - 1) >> 1 : 0;
          const int e = min((li + 1) >> 1, HW - 1);
          const int s = lj > 0 ? lj - 1 : 0, n = min(lj + 1, MH - 1);
          if (cw[b][c] != R(0)) o += cw[b][c] * zc[oc][lj][w];
          if (ce[b][c] != R(0)) o += ce[b][c] * zc[oc][lj][e];
          if (cs[b][c] != R(0)) o += cs[b][c] * zc[oc][s][k];
          if (cn[b][c] != R(0)) o += cn[b][c] * zc[oc][n][k];
        }
        zc[c][lj][k] = (rr[b][c] + o) * dg[b][c];
      }
    }
    __syncthreads();
  }

  // write back the tile's own cells
#pragma unroll
  for (int b = 0; b < NR; ++b) {
    const int lj = ty + BY * b;
    const int j = ry0 + lj;
    if (lj >= RH || j < y0 || j >= y0 + TH) continue;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int li = 2 * k + ((rx0 + ry0 + lj + c) & 1);
      const int i = rx0 + li;
      if (li < RW && i >= x0 && i < x0 + TW) zout[i + nx * j] = zc[c][lj][k];
    }
  }
  if (POST && part) {
    // this tile's part of r . zout (the CG's rho), tile cells in thread
    // order, then the waves in order: one partial per tile
    double acc = 0.0;
#pragma unroll
    for (int b = 0; b < NR; ++b) {
      const int lj = ty + BY * b;
      const int j = ry0 + lj;
      if (lj >= RH || j < y0 || j >= y0 + TH) continue;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int li = 2 * k + ((rx0 + ry0 + lj + c) & 1);
        const int i = rx0 + li;
        if (li < RW && i >= x0 && i < x0 + TW) acc += (double)rr[b][c] * (double)zc[c][lj][k];
      }
    }
    __shared__ double wsum[BX * BY / kWave];
    acc = wave_sum_dpp(acc);
    const int tid = threadIdx.x;
    if ((tid & (kWave - 1)) == kWave - 1) wsum[tid / kWave] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < BX * BY / kWave; ++w) t += wsum[w];
      part[tbx + gridDim.x * tby] = t;
    }
  }
}

// FUSED = false: the post-smoother continues from zin, which already holds
// the prolongation
template <typename R, int TW, int TH, int BX, int BY, bool FUSED = true>
hipError_t launch_tiles(const Lv<R>& L, const Xfer* X, const R* r, const R* zin, const R* y, R* zout, hipStream_t s,
                        const int* gate, double* part) {
  const dim3 grid((L.nx + TW - 1) / TW, (L.ny + TH - 1) / TH);
  const dim3 block(BX * BY);
  if constexpr (!FUSED) {
    hipLaunchKernelGGL((k_smooth_tile<R, true, TW, TH, BX, BY, false>), grid, block, 0, s, L, *X, r, zin, y, zout,
                       gate, part);
    return hipGetLastError();
  }
  if (X)
    hipLaunchKernelGGL((k_smooth_tile<R, true, TW, TH, BX, BY>), grid, block, 0, s, L, *X, r, zin, y, zout, gate,
                       part);
  else
    hipLaunchKernelGGL((k_smooth_tile<R, false, TW, TH, BX, BY>), grid, block, 0, s, L, Xfer{}, r, zin, y, zout,
                       gate, (double*)nullptr);
  return hipGetLastError();
}

constexpr int kShapeTW[4] = {64, 110, 46, 14}, kShapeTH[4] = {32, 38, 14, 14};

// Tile shapes: 0 = 64 x 32 (512 threads), 1 = 110 x 38 (512 threads, region
// rows of exactly 128 cells), 2 = 46 x 14 (1024 threads for the pre-smoother,
// 512 for the post-smoother), 3 = 14 x 14 (512 threads, one region row per
// thread).  Larger tiles re-read less halo but hold more registers per
// thread, which caps the waves per CU; measured on MI355X (1024^2 and 256^2
// levels), the small-register shapes win: 46 x 14 on the largest levels,
// 14 x 14 below.  Per 1024^2 launch, shape 2 ran pre / post in 27 / 48 us
// with 256 threads (four region rows per thread; the post-smoother spilled),
// 23 / 44 us with 512 and 20 / 59 us with 1024.  Shape 3 on a 256^2 level:
// 7.3 / 11.4 us with 256 threads, 5.2 / 9.2 us with 512.
int auto_shape(int nx, int ny) {
  const long long cells = (long long)nx * ny;
  return cells >= (1LL << 19) ? 2 : 3;
}

// Residual and restriction in one pass (2-D): g = E^T (r - A z), Section 3.
// A workgroup owns kCTx x kCTy coarse cells.  It loads the fine cells of their
// footprint (plus a one-cell halo of z) into LDS, forms the residual there,
// then sums each fine row against the x weights of each coarse column and
// those row sums against the y weights.  Terms and order are those of the
// two-kernel path (residual stored, then the stored-residual restriction), so
// the result is the same bit for bit.
constexpr int kCTx = 8, kCTy = 4;          // coarse cells per workgroup
constexpr int kFootMax = 4 * 1 + 2 * 2 + 2;  // fine cells in one coarse cell's footprint for s <= 4
constexpr int kRegW = 4 * (kCTx - 1) + kFootMax, kRegH = 4 * (kCTy - 1) + kFootMax;

template <typename R>
__global__ void __launch_bounds__(256) k_resid_restrict_tile(Lv<R> L, Xfer X, const R* __restrict__ r,
                                                             const R* __restrict__ z, R* __restrict__ g,
                                                             const int* __restrict__ gate) {
  constexpr int kZ = (kRegH + 2) * (kRegW + 2), kC = kRegH * kRegW;
  constexpr int kZPer = (kZ + 255) / 256, kCPer = (kC + 255) / 256;
  __shared__ R zs[kRegH + 2][kRegW + 2];
  __shared__ R res[kRegH][kRegW];
  __shared__ R tmp[kRegH][kCTx];
  __shared__ R wxt[kCTx][kFootMax], wyt[kCTy][kFootMax];  // footprint weights of the block's coarse columns, rows
  const int nx = L.nx, ny = L.ny, tid = threadIdx.x;
  int tbx, tby;
  xcd_tile(tbx, tby);
  const int I0 = tbx * kCTx, J0 = tby * kCTy;
  const int I1 = min(I0 + kCTx, X.cnx) - 1, J1 = min(J0 + kCTy, X.cny) - 1;
  int lox, hix, loy, hiy, t0, t1;
  ext_support(I0, X.sx, nx, X.interp, lox, t0);
  ext_support(I1, X.sx, nx, X.interp, t1, hix);
  ext_support(J0, X.sy, ny, X.interp, loy, t0);
  ext_support(J1, X.sy, ny, X.interp, t1, hiy);
  const int RW = hix - lox + 1, RH = hiy - loy + 1;
  // every load of the block first, with the gate: one round trip to memory.
  // z on the region and a one-cell ring (zero outside the grid: those terms
  // are skipped); T and r of the region's cells
  const int gv = gate ? *gate : 0;
  R zv[kZPer];
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int e = tid + 256 * u;
    const int lj = e / (RW + 2), li = e - lj * (RW + 2);
    const int i = lox - 1 + li, j = loy - 1 + lj;
    zv[u] = (e < (RH + 2) * (RW + 2) && i >= 0 && i < nx && j >= 0 && j < ny) ? z[i + nx * j] : R(0);
  }
  R cw[kCPer], ce[kCPer], cs[kCPer], cn[kCPer], rv[kCPer];
#pragma unroll
  for (int u = 0; u < kCPer; ++u) {
    const int e = tid + 256 * u;
    const bool in = e < RH * RW;
    const int lj = in ? e / RW : 0, li = in ? e - lj * RW : 0;
    const int i = lox + li, j = loy + lj;
    const int fx = i + (nx + 1) * j, fy = i + nx * j;
    cw[u] = in ? L.tx[fx] : R(0);
    ce[u] = in ? L.tx[fx + 1] : R(0);
    cs[u] = in ? L.ty[fy] : R(0);
    cn[u] = in ? L.ty[fy + nx] : R(0);
    rv[u] = in ? r[fy] : R(0);
  }
  asm volatile("" ::"v"(gv));  // the gate's wait comes after every load is issued
  if (gv) return;
#pragma unroll
  for (int u = 0; u < kZPer; ++u) {
    const int e = tid + 256 * u;
    if (e < (RH + 2) * (RW + 2)) zs[e / (RW + 2)][e % (RW + 2)] = zv[u];
  }
  if (tid < kCTx * kFootMax) {
    const int c = tid / kFootMax, b = tid - c * kFootMax, I = I0 + c;
    int ilo, ihi;
    ext_support(I, X.sx, nx, X.interp, ilo, ihi);
    wxt[c][b] = (I <= I1 && ilo + b <= ihi) ? ext_weight_of<R>(ilo + b, I, X.sx, X.cnx, X.interp) : R(0);
  } else if (tid < kCTx * kFootMax + kCTy * kFootMax) {
    const int t = tid - kCTx * kFootMax, c = t / kFootMax, b = t - c * kFootMax, J = J0 + c;
    int jlo, jhi;
    ext_support(J, X.sy, ny, X.interp, jlo, jhi);
    wyt[c][b] = (J <= J1 && jlo + b <= jhi) ? ext_weight_of<R>(jlo + b, J, X.sy, X.cny, X.interp) : R(0);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kCPer; ++u) {
    const int e = tid + 256 * u;
    if (e >= RH * RW) continue;
    const int lj = e / RW, li = e - lj * RW;
    const int i = lox + li, j = loy + lj;
    const R tw = cw[u], te = ce[u], ts = cs[u], tn = cn[u];
    const R d = tw + te + ts + tn;
    R o = R(0);
    if (i > 0) o += tw * zs[lj + 1][li];
    if (i < nx - 1) o += te * zs[lj + 1][li + 2];
    if (j > 0) o += ts * zs[lj][li + 1];
    if (j < ny - 1) o += tn * zs[lj + 2][li + 1];
    res[lj][li] = rv[u] - (d * zs[lj + 1][li + 1] - o);
  }
  __syncthreads();
  // x pass: row lj against the weights of coarse column I over its footprint
  for (int e = tid; e < RH * kCTx; e += blockDim.x) {
    const int lj = e / kCTx, c = e - lj * kCTx, I = I0 + c;
    if (I > I1) continue;
    int ilo, ihi;
    ext_support(I, X.sx, nx, X.interp, ilo, ihi);
    R racc = R(0);
    for (int i = ilo; i <= ihi; ++i) racc += wxt[c][i - ilo] * res[lj][i - lox];
    tmp[lj][c] = racc;
  }
  __syncthreads();
  // y pass
  for (int e = tid; e < kCTy * kCTx; e += blockDim.x) {
    const int cj = e / kCTx, c = e % kCTx, J = J0 + cj, I = I0 + c;
    if (J > J1 || I > I1) continue;
    int jlo, jhi;
    ext_support(J, X.sy, ny, X.interp, jlo, jhi);
    R acc = R(0);
    for (int j = jlo; j <= jhi; ++j) {
      const R wj = wyt[cj][j - jlo];
      if (wj == R(0)) continue;
      acc += (R(1) * wj) * tmp[j - loy][c];
    }
    g[I + X.cnx * J] = acc;
  }
}

}  // namespace

bool smooth_tile_supported(int nz, bool has_tz, int m) { return nz == 1 && !has_tz && 2 * m + 1 == kHalo; }

int smooth_tile_count(int nx, int ny, int shape) {
  if (shape < 0 || shape > 3) shape = auto_shape(nx, ny);
  return ((nx + kShapeTW[shape] - 1) / kShapeTW[shape]) * ((ny + kShapeTH[shape] - 1) / kShapeTH[shape]);
}

template <typename R>
hipError_t launch_smooth_tile(const Lv<R>& L, const Xfer* X, const R* r, const R* zin, const R* y, R* zout,
                              int m, int shape, hipStream_t s, const int* gate, double* part) {
  if (!smooth_tile_supported(L.nz, L.tz != nullptr, m)) return hipErrorNotSupported;
  if (shape < 0 || shape > 3) shape = auto_shape(L.nx, L.ny);
  switch (shape) {
    case 0: return launch_tiles<R, 64, 32, 64, 8>(L, X, r, zin, y, zout, s, gate, part);
    case 1: return launch_tiles<R, 110, 38, 64, 8>(L, X, r, zin, y, zout, s, gate, part);
    case 2:  // one region row per thread for the pre-smoother, two for the post-smoother
      if (X) {
        // the prolongation as a grid-wide pass in place on zin, then the
        // sweeps from zin: fused into the tiles it held more registers (fewer
        // waves) than it saved in traffic
        const hipError_t e = launch_prolong<R>(L, *X, y, const_cast<R*>(zin), s, gate);
        if (e != hipSuccess) return e;
        return launch_tiles<R, 46, 14, 32, 16, false>(L, X, r, zin, y, zout, s, gate, part);
      }
      return launch_tiles<R, 46, 14, 32, 32>(L, X, r, zin, y, zout, s, gate, part);
    default: return launch_tiles<R, 14, 14, 16, 32>(L, X, r, zin, y, zout, s, gate, part);
  }
}

bool resid_restrict_tile_supported(const Lv<double>& L, const Xfer& X) {
  auto ok = [&](int f) { return f >= 1 && f <= 4; };
  return !X.frac && !L.tz && L.nz == 1 && X.cnz == 1 && ok(X.sx) && ok(X.sy);
}

template <typename R>
hipError_t launch_resid_restrict_tile(const Lv<R>& L, const Xfer& X, const R* r, const R* z, R* g, hipStream_t s,
                                      const int* gate) {
  const Lv<double> shape{L.nx, L.ny, L.nz, L.n, nullptr, nullptr, L.tz ? (const double*)1 : nullptr};
  if (!resid_restrict_tile_supported(shape, X)) return hipErrorNotSupported;
  const dim3 grid((X.cnx + kCTx - 1) / kCTx, (X.cny + kCTy - 1) / kCTy);
  hipLaunchKernelGGL(k_resid_restrict_tile<R>, grid, dim3(256), 0, s, L, X, r, z, g, gate);
  return hipGetLastError();
}

template hipError_t launch_resid_restrict_tile<double>(const Lv<double>&, const Xfer&, const double*, const double*,
                                                      double*, hipStream_t, const int*);
template hipError_t launch_resid_restrict_tile<float>(const Lv<float>&, const Xfer&, const float*, const float*,
                                                     float*, hipStream_t, const int*);

template hipError_t launch_smooth_tile<double>(const Lv<double>&, const Xfer*, const double*, const double*,
                                               const double*, double*, int, int, hipStream_t, const int*, double*);
template hipError_t launch_smooth_tile<float>(const Lv<float>&, const Xfer*, const float*, const float*,
                                              const float*, float*, int, int, hipStream_t, const int*, double*);

}  // namespace mscg
