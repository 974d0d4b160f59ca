// mscg_small2x2.hip -- one-workgroup solver for a 2-D last inner level of at
// most 64 x 64 cells, each thread owning a 2 x 2 block of cells.
//
// Same algorithm as the colour-split kernel (the level's inner PCG with all
// its iterations in one launch, Section 2.3; the two-grid cycle of eq. 2.10
// with red-black symmetric Gauss-Seidel, Section 3; the level criterion
// |r|^2 / N_k < f^k eps^2), with a layout that keeps the smoother's iterate
// and the CG direction in registers.
//
// Thread t (wave w, lane l) owns block (bp, bq) = (l mod 32, 2 w + l / 32),
// the cells (2 bp + a, 2 bq + b), a, b in {0, 1}, numbered u = a + 2 b.  Cells
// 0 and 3 are red ((i + j) even), 1 and 2 black, so every thread updates
// exactly two cells in each half sweep and each of them has two of its four
// neighbours in the same block: only one horizontal and one vertical
// neighbour come from another thread.  Those go through four LDS exchange
// arrays, one per position u, indexed by block with a zero border: after a
// half sweep each thread publishes its two new values.  Cells past the grid
// (nx or ny odd, or below 64) are ghosts with zero coefficients, zero
// right-hand side and unit diagonal: they stay zero.
//
// The residual for the restriction goes to a natural-layout LDS array; the
// restriction and the prolongation follow the colour-split kernel.  The
// coarsest solve applies the FP64 inverse from its lower triangle alone (the
// inverse is symmetric), stored in 16 x 16 tiles: half the bytes the dense
// product reads from L2 each iteration.  Reductions: the four owned cells in
// order, DPP within each wave, then the 16 wave sums in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "mscg_kernels.h"

namespace mscg {

namespace {

constexpr int kT = 1024;               // threads
constexpr int kBW = 32, kBH = 32;      // blocks per block row, block rows
constexpr int kEP = kBW + 2;           // exchange array pitch (zero border)
constexpr int kEA = (kBH + 2) * kEP;   // entries per exchange array
constexpr int kRP = 2 * kBW + 1;       // residual array pitch (odd: a column read is conflict-free)
constexpr int kFoot2 = 12;             // >= footprint of one coarse cell along an axis (linear, s <= 4)

struct Small2x2Args {
  int nx, ny;
  int sx, sy, cnx, cny, nc;
  int interp, m, max_inner;
  double tol, rel_floor2;
  const void *tx, *ty, *rhs;
  void* x;
  const double* Asym;  // lower triangle of the coarsest inverse in 16 x 16 tiles
  int ntile;           // tiles per side
  long long *iters, *calls;
  int level;
  int* status;
  const int* gate;
  int off_ex, off_res, off_xs, off_ps, off_tx1, off_g, off_y, off_wx, off_wy, off_ci, off_cw, off_ri, off_rw;
};

template <typename R>
__global__ void __launch_bounds__(kT, 1) k_small_2x2(Small2x2Args a) {
  if (a.gate && *a.gate) return;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ __align__(16) double sm[2][kT / kWave];
  R* ex = reinterpret_cast<R*>(lds + a.off_ex);     // [u][bq + 1][bp + 1]
  R* res = reinterpret_cast<R*>(lds + a.off_res);   // [j][i], pitch kRP
  R* tx1 = reinterpret_cast<R*>(lds + a.off_tx1);  // x-pass sums, [I][row], pitch ny + 1
  double* g = reinterpret_cast<double*>(lds + a.off_g);  // padded with zeros to 16 ntile
  double* y = reinterpret_cast<double*>(lds + a.off_y);
  double* part = reinterpret_cast<double*>(lds + a.off_res);  // coarsest partials, after the restriction
  R* xs = reinterpret_cast<R*>(lds + a.off_xs);    // iterate x, [u][tid]
  R* ps = reinterpret_cast<R*>(lds + a.off_ps);    // CG direction p, [u][tid]
  R* wx = reinterpret_cast<R*>(lds + a.off_wx);
  R* wy = reinterpret_cast<R*>(lds + a.off_wy);
  int* ci = reinterpret_cast<int*>(lds + a.off_ci);
  R* cw = reinterpret_cast<R*>(lds + a.off_cw);
  int* ri = reinterpret_cast<int*>(lds + a.off_ri);
  R* rw = reinterpret_cast<R*>(lds + a.off_rw);
  const R* TX = static_cast<const R*>(a.tx);
  const R* TY = static_cast<const R*>(a.ty);
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
  const int bp = lane & (kBW - 1), bq = 2 * wid + lane / kBW;
  const int nx = a.nx, ny = a.ny;
  const int ncx = a.cnx, ncy = a.cny, nc = a.nc;

  int red = 0;
  auto block_sum = [&](double v) {
    v = wave_sum_dpp(v);
    if (lane == kWave - 1) sm[red][wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kT / kWave; ++w) s += sm[red][w];
    red ^= 1;
    return s;
  };
  // exchange entry of position u of block (bp + dp, bq + dq)
  auto xe = [&](int u, int dp, int dq) { return u * kEA + (bq + 1 + dq) * kEP + (bp + 1 + dp); };

  // ---- set-up: zero the exchange arrays (their border stays zero), tables
  for (int e = tid; e < 4 * kEA; e += kT) ex[e] = R(0);
  for (int e = nc + tid; e < 16 * a.ntile; e += kT) g[e] = 0.0;
  for (int i = tid; i < nx; i += kT) {
    int I0, I1;
    R w0, w1;
    ext_weights<R>(i, a.sx, ncx, a.interp, I0, w0, I1, w1);
    ci[i] = I0 | (I1 << 16);
    cw[2 * i] = w0;
    cw[2 * i + 1] = w1;
  }
  for (int j = tid; j < ny; j += kT) {
    int J0, J1;
    R w0, w1;
    ext_weights<R>(j, a.sy, ncy, a.interp, J0, w0, J1, w1);
    ri[j] = J0 | (J1 << 16);
    rw[2 * j] = w0;
    rw[2 * j + 1] = w1;
  }
  for (int e = tid; e < ncx * kFoot2; e += kT) {
    const int I = e / kFoot2, b = e - I * kFoot2;
    int lo, hi;
    ext_support(I, a.sx, nx, a.interp, lo, hi);
    wx[e] = lo + b <= hi ? ext_weight_of<R>(lo + b, I, a.sx, ncx, a.interp) : R(0);
  }
  for (int e = tid; e < ncy * kFoot2; e += kT) {
    const int J = e / kFoot2, b = e - J * kFoot2;
    int lo, hi;
    ext_support(J, a.sy, ny, a.interp, lo, hi);
    wy[e] = lo + b <= hi ? ext_weight_of<R>(lo + b, J, a.sy, ncy, a.interp) : R(0);
  }

  // ---- owned cells
  // Coefficients: the four faces inside the block are shared by two owned
  // cells (zero on both sides when one of them is a ghost).
  R tW0, tS0, tE01, tN02, tE1, tS1, tN13, tW2, tN2, tE23, tE3, tN3;
  R dg[4], di[4], r[4], z[4];
  bool ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = 2 * bp + (u & 1), j = 2 * bq + (u >> 1);
    ok[u] = i < nx && j < ny;
    const int ii = ok[u] ? i : 0, jj = ok[u] ? j : 0;
    const int fx = ii + (nx + 1) * jj, fy = ii + nx * jj;
    const R tw = TX[fx], te = TX[fx + 1], ts = TY[fy], tn = TY[fy + nx];
    dg[u] = ok[u] ? tw + te + ts + tn : R(1);
    di[u] = R(1) / dg[u];
    const R cw_ = ok[u] && ii > 0 ? tw : R(0);
    const R ce_ = ok[u] && ii < nx - 1 ? te : R(0);
    const R cs_ = ok[u] && jj > 0 ? ts : R(0);
    const R cn_ = ok[u] && jj < ny - 1 ? tn : R(0);
    if (u == 0) { tW0 = cw_; tE01 = ce_; tS0 = cs_; tN02 = cn_; }
    if (u == 1) { tE1 = ce_; tS1 = cs_; tN13 = cn_; }
    if (u == 2) { tW2 = cw_; tE23 = ce_; tN2 = cn_; }
    if (u == 3) { tE3 = ce_; tN3 = cn_; }
    r[u] = ok[u] ? static_cast<const R*>(a.rhs)[ii + nx * jj] : R(0);
    xs[u * kT + tid] = R(0);
    z[u] = R(0);
  }
  // sum of T_f v_nb for cell u of vector v: own block from registers, the
  // rest from the exchange arrays (which hold v of the other cells)
  auto offsum = [&](const R* v, int u) -> R {
    if (u == 0) return tW0 * ex[xe(1, -1, 0)] + tE01 * v[1] + tS0 * ex[xe(2, 0, -1)] + tN02 * v[2];
    if (u == 1) return tE01 * v[0] + tE1 * ex[xe(0, 1, 0)] + tS1 * ex[xe(3, 0, -1)] + tN13 * v[3];
    if (u == 2) return tW2 * ex[xe(3, -1, 0)] + tE23 * v[3] + tN02 * v[0] + tN2 * ex[xe(0, 0, 1)];
    return tE23 * v[2] + tE3 * ex[xe(2, 1, 0)] + tN13 * v[1] + tN3 * ex[xe(1, 0, 1)];
  };
  auto publish = [&](const R* v, int u) { ex[xe(u, 0, 0)] = v[u]; };
  // half sweep of the Section 3 splitting over cells u0 and u1 (red: 0, 3;
  // black: 1, 2), compile-time positions so that z stays in registers
  auto half_sweep = [&](auto u0c, auto u1c, bool first) {
    constexpr int u0 = decltype(u0c)::value, u1 = decltype(u1c)::value;
    if (first) {
      z[u0] = r[u0] * di[u0];
      z[u1] = r[u1] * di[u1];
    } else {
      const R n0 = (r[u0] + offsum(z, u0)) * di[u0];
      const R n1 = (r[u1] + offsum(z, u1)) * di[u1];
      z[u0] = n0;
      z[u1] = n1;
    }
    publish(z, u0);
    publish(z, u1);
    __syncthreads();
  };
  using C0 = std::integral_constant<int, 0>;
  using C1 = std::integral_constant<int, 1>;
  using C2 = std::integral_constant<int, 2>;
  using C3 = std::integral_constant<int, 3>;
  // 2m + 1 half sweeps: red, then m (black, red) pairs
  auto sweeps = [&](bool from_zero) {
    half_sweep(C0{}, C3{}, from_zero);
    for (int h = 0; h < a.m; ++h) {
      half_sweep(C1{}, C2{}, false);
      half_sweep(C0{}, C3{}, false);
    }
  };

  double rr = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) rr += (double)r[u] * (double)r[u];
  rr = block_sum(rr);  // its barrier also orders the set-up writes before their use
  double tol = a.tol;
  if (a.rel_floor2 > 0.0 && a.rel_floor2 * rr > tol) tol = a.rel_floor2 * rr;
  long long iters = 0, coarse_calls = 0;
  int status = 0;
  double rho_old = 0.0;

  if (!(rr < tol)) {
    for (int it = 0; it < a.max_inner; ++it) {
      // -- pre-smoothing from zero (z of the black cells is overwritten before
      // it is read), then the residual for the restriction.  The last half
      // sweep is red, so the exchange arrays hold the current z of every cell.
      sweeps(true);
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ok[u]) res[(2 * bq + (u >> 1)) * kRP + 2 * bp + (u & 1)] = r[u] - (dg[u] * z[u] - offsum(z, u));
      __syncthreads();
      // -- g = E^T res: x pass over (I, fine row), rows along the lanes, then
      // y pass over (J, I), I along the lanes; odd pitches keep both passes'
      // LDS reads free of bank conflicts
      const int p1 = ny + 1;
      for (int e = tid; e < ny * ncx; e += kT) {
        const int I = e / ny, row = e - I * ny;
        int lo, hi;
        ext_support(I, a.sx, nx, a.interp, lo, hi);
        R s = R(0);
#pragma unroll
        for (int b = 0; b < kFoot2; ++b) {
          const int i = min(lo + b, hi);
          s += wx[I * kFoot2 + b] * res[row * kRP + i];
        }
        tx1[I * p1 + row] = s;
      }
      __syncthreads();
      for (int e = tid; e < nc; e += kT) {
        const int J = e / ncx, I = e - J * ncx;
        int lo, hi;
        ext_support(J, a.sy, ny, a.interp, lo, hi);
        R s = R(0);
#pragma unroll
        for (int b = 0; b < kFoot2; ++b) {
          const int j = min(lo + b, hi);
          s += wy[J * kFoot2 + b] * tx1[I * p1 + j];
        }
        g[e] = (double)s;
      }
      __syncthreads();
      {
        // -- coarsest: y = A^-1 g from the lower triangle in 16 x 16 tiles.
        // A 16-lane group (one DPP row) takes tile (I, J), I >= J, lane c
        // its column c: y_J[c] += sum_r T[r][c] g_I[r] stays in the lane,
        // y_I[r] += sum_c T[r][c] g_J[c] is a sum across the lanes, formed
        // by a four-stage exchange that leaves row c's total in lane c.
        // Each output block gets one 16-vector per tile of its block row or
        // column (slot = the other tile index), summed in slot order.
        const int NT = a.ntile, ntiles = NT * (NT + 1) / 2;
        const int grp = tid >> 4, c = tid & 15;
        auto gat = [&](int e) { return g[e]; };
        for (int t = grp; t < ntiles; t += kT / 16) {
          int I = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
          while (I * (I + 1) / 2 > t) --I;
          while ((I + 1) * (I + 2) / 2 <= t) ++I;
          const int J = t - I * (I + 1) / 2;
          const double* T = a.Asym + (long long)t * 256;
          const double gJc = gat(16 * J + c);
          // The tile is stored skewed: slot s of lane c holds row s xor c
          // (column c).  Each exchange stage then pairs slot s with slot
          // s xor m, m = 15, 7, 3, 1 for the mirror, half-row mirror and the
          // two quad permutations: the partner lane's slot holds the same row,
          // so no lane has to choose what to keep or send.  Slots arrive in
          // quads that close one second-stage value each.
          const double* Tl = T + c;
          double acc_c = 0.0;
          auto quad = [&](auto s0c, const double (&v)[4]) {
            constexpr int s0 = decltype(s0c)::value;  // slots s0, s0 ^ 15, s0 ^ 7, s0 ^ 8
            constexpr int sl[4] = {s0, s0 ^ 15, s0 ^ 7, s0 ^ 8};
#pragma unroll
            for (int k = 0; k < 4; ++k) acc_c += v[k] * gat(16 * I + (sl[k] ^ c));
            const double u_a = v[0] * gJc + dpp_full<0x140>(v[1] * gJc);  // slot s0 (mirror)
            const double u_b = v[2] * gJc + dpp_full<0x140>(v[3] * gJc);  // slot s0 ^ 7
            return u_a + dpp_full<0x141>(u_b);                            // half-row mirror
          };
          auto load = [&](int s0, double (&v)[4]) {
            v[0] = Tl[s0 * 16];
            v[1] = Tl[(s0 ^ 15) * 16];
            v[2] = Tl[(s0 ^ 7) * 16];
            v[3] = Tl[(s0 ^ 8) * 16];
          };
          // quads for the second-stage slots 0, 3 (-> third-stage slot 0) and 1, 2 (-> 1);
          // the next quad's loads go out before this quad's arithmetic
          double qa[4], qb[4];
          load(0, qa);
          load(3, qb);
          asm volatile("" ::: "memory");
          const double w0 = quad(std::integral_constant<int, 0>{}, qa);
          load(1, qa);
          asm volatile("" ::: "memory");
          const double w3 = quad(std::integral_constant<int, 3>{}, qb);
          load(2, qb);
          asm volatile("" ::: "memory");
          const double v0 = w0 + dpp_full<0x1B>(w3);  // quad permutation 3 - (c mod 4)
          const double w1 = quad(std::integral_constant<int, 1>{}, qa);
          const double w2 = quad(std::integral_constant<int, 2>{}, qb);
          const double v1 = w1 + dpp_full<0x1B>(w2);
          part[(J * NT + I) * 16 + c] = acc_c;
          if (I != J) {  // the same for all 16 lanes of the group
            // partner c xor 1: lane c ends with the total of row c
            const double row = v0 + dpp_full<0xB1>(v1);
            part[(I * NT + J) * 16 + c] = row;
          }
        }
        __syncthreads();
        for (int i = tid; i < nc; i += kT) {
          const int X = i >> 4, r_ = i & 15;
          double s = 0.0;
          for (int Y = 0; Y < NT; ++Y) s += part[(X * NT + Y) * 16 + r_];
          y[i] = s;
        }
      }
      coarse_calls++;
      __syncthreads();
      // -- prolongation z += E y, then publish the black cells (the first
      // post half sweep is red and reads them)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!ok[u]) continue;
        const int i = 2 * bp + (u & 1), j = 2 * bq + (u >> 1);
        const int pi = ci[i], pj = ri[j];
        const int I0 = pi & 0xffff, I1 = pi >> 16, b0 = ncx * (pj & 0xffff), b1 = ncx * (pj >> 16);
        const R wi0 = cw[2 * i], wi1 = cw[2 * i + 1], wj0 = rw[2 * j], wj1 = rw[2 * j + 1];
        z[u] += wj0 * (wi0 * (R)y[I0 + b0] + wi1 * (R)y[I1 + b0]) + wj1 * (wi0 * (R)y[I0 + b1] + wi1 * (R)y[I1 + b1]);
      }
      publish(z, 1);
      publish(z, 2);
      __syncthreads();
      // -- post-smoothing
      sweeps(false);
      // -- CG step (Templates Figure 2.5)
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += (double)r[u] * (double)z[u];
      const double rho = block_sum(acc);
      if (!(rho == rho) || rho == INFINITY) { status = -4; break; }
      if (!(rho > 0.0)) break;  // no further progress in this precision: the level stops
      const R beta = it == 0 ? R(0) : (R)(rho / rho_old);
      R pv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pv[u] = it == 0 ? z[u] : z[u] + beta * ps[u * kT + tid];
        ps[u * kT + tid] = pv[u];
        publish(pv, u);
      }
      __syncthreads();
      R q[4];
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        q[u] = dg[u] * pv[u] - offsum(pv, u);
        acc += (double)pv[u] * (double)q[u];
      }
      const double pq = block_sum(acc);
      if (!(pq == pq) || pq == INFINITY) { status = -4; break; }
      if (!(pq > 0.0)) break;
      const R alpha = (R)(rho / pq);
      acc = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xs[u * kT + tid] += alpha * pv[u];
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
  for (int u = 0; u < 4; ++u)
    if (ok[u]) xo[2 * bp + (u & 1) + nx * (2 * bq + (u >> 1))] = xs[u * kT + tid];
  if (tid == 0) {
    a.iters[a.level] += iters;
    a.calls[a.level] += 1;
    a.calls[a.level + 1] += coarse_calls;
    if (status) a.status[0] = status;
  }
}

}  // namespace

template <typename R>
hipError_t launch_small_2x2(const SmallDesc<R>& d, hipStream_t s) {
  const int ks = d.ks;
  if (ks + 1 != d.nlev - 1) return hipErrorNotSupported;
  const Lv<R>& V = d.L[ks];
  const Xfer& X = d.X[ks];
  if (V.tz || V.nz != 1 || V.nx > 2 * kBW || V.ny > 2 * kBH) return hipErrorNotSupported;
  const int nc = X.cnx * X.cny;
  // the coarsest product needs the tiled lower triangle, at most 16 x 16 tiles
  if (nc > kT || !d.Asym || d.ntile > 16 || d.ntile * 16 < nc) return hipErrorNotSupported;
  auto foot = [&](int f) { return f == 1 ? 1 : X.interp == 1 ? f : f + 2 * (f / 2) + 2; };
  if (foot(X.sx) > kFoot2 || foot(X.sy) > kFoot2) return hipErrorNotSupported;
  Small2x2Args a{};
  a.nx = V.nx; a.ny = V.ny;
  a.sx = X.sx; a.sy = X.sy; a.cnx = X.cnx; a.cny = X.cny; a.nc = nc;
  a.interp = X.interp; a.m = d.m; a.max_inner = d.max_inner;
  a.tol = d.tol[ks]; a.rel_floor2 = d.rel_floor2;
  a.tx = V.tx; a.ty = V.ty; a.rhs = d.r[ks]; a.x = d.x[ks];
  a.Asym = d.Asym;
  a.ntile = d.ntile;
  a.iters = d.iters; a.calls = d.calls; a.level = ks; a.status = d.status;
  a.gate = d.gate;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const int o = (int)off;
    off += (bytes + 15) & ~(size_t)15;
    return o;
  };
  a.off_ex = take((size_t)4 * kEA * sizeof(R));
  // the residual array also holds the coarsest partials (2 kT doubles, or
  // ntile^2 slots of 16 for the tiled product)
  a.off_res = take(std::max({(size_t)2 * kBH * kRP * sizeof(R), (size_t)2 * kT * sizeof(double),
                             (size_t)a.ntile * a.ntile * 16 * sizeof(double)}));
  a.off_xs = take((size_t)4 * kT * sizeof(R));
  a.off_ps = take((size_t)4 * kT * sizeof(R));
  a.off_tx1 = take((size_t)(V.ny + 1) * X.cnx * sizeof(R));
  a.off_g = take((size_t)16 * d.ntile * sizeof(double));
  a.off_y = take((size_t)nc * sizeof(double));
  a.off_wx = take((size_t)X.cnx * kFoot2 * sizeof(R));
  a.off_wy = take((size_t)X.cny * kFoot2 * sizeof(R));
  a.off_ci = take((size_t)V.nx * sizeof(int));
  a.off_cw = take((size_t)2 * V.nx * sizeof(R));
  a.off_ri = take((size_t)V.ny * sizeof(int));
  a.off_rw = take((size_t)2 * V.ny * sizeof(R));
  if (off > 156 * 1024) return hipErrorNotSupported;
  static bool attr[2] = {false, false};
  const int ri = sizeof(R) == 8 ? 1 : 0;
  if (!attr[ri]) {
    hipError_t e = hipFuncSetAttribute((const void*)k_small_2x2<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       156 * 1024);
    if (e != hipSuccess) return e;
    attr[ri] = true;
  }
  hipLaunchKernelGGL((k_small_2x2<R>), dim3(1), dim3(kT), off, s, a);
  return hipGetLastError();
}

template hipError_t launch_small_2x2<double>(const SmallDesc<double>&, hipStream_t);
template hipError_t launch_small_2x2<float>(const SmallDesc<float>&, hipStream_t);

}  // namespace mscg
