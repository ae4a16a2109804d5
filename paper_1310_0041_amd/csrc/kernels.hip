// gfx950 kernels of the multigrid solver for the screened anisotropic Poisson
// systems of Kazhdan et al., "Gradient-Domain Processing for Large EM Image
// Stacks" (Sec. 4 operator, Sec. 4.1 multigrid steps, Sec. 4.2 7-point
// stencil).  Every level operator is alpha*Id + sum_a w_a L_a, L_a the
// 3-point Neumann second difference along axis a (no faces outside the grid).
//
// All stencils are evaluated in difference form, sum_nb w (x_nb - x_c), which
// keeps the rounding error proportional to the local variation instead of
// the magnitude of x.
#include "gd_launch.h"

namespace gd {

// ---------------------------------------------------------------- helpers

// Deterministic block sum of a double (wave shuffles, then the waves in
// order).  Result valid on thread 0.  `red` must hold blockDim/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

struct Tile {
  int g, x0, y0, z0, z1;
};

// Decode blockIdx.x into (grid, tile, z-range) for TX x TY tiles over the
// grid's own size (coarse = false) or its child's size (coarse = true).
template <int TX, int TY>
__device__ __forceinline__ Tile decode_tile(const GridDesc* __restrict__ grids,
                                            const int64_t* __restrict__ block0, int ngrids,
                                            int zlen, bool coarse) {
  Tile t;
  const int64_t bid = blockIdx.x;
  t.g = find_grid(block0, ngrids, bid);
  const GridDesc& G = grids[t.g];
  const int nx = coarse ? G.cnx : G.nx, ny = coarse ? G.cny : G.ny, nz = coarse ? G.cnz : G.nz;
  const int64_t local = bid - block0[t.g];
  const int tx = (nx + TX - 1) / TX, ty = (ny + TY - 1) / TY;
  const int64_t txy = (int64_t)tx * ty;
  const int zc = (int)(local / txy);
  const int r = (int)(local - (int64_t)zc * txy);
  t.x0 = (r % tx) * TX;
  t.y0 = (r / tx) * TY;
  t.z0 = zc * zlen;
  t.z1 = min(t.z0 + zlen, nz);
  return t;
}

// Cell-centred linear up-sampling weights along one axis: the fine cell i of
// a halved axis takes 3/4 of its parent i/2 and 1/4 of the nearer coarse
// neighbour, the parent itself standing in for a neighbour outside the grid;
// a kept axis (f == 1) maps i to i.
__device__ __forceinline__ void lin_idx(int i, int f, int nc, int& a, int& b) {
  if (f == 1) { a = b = i; return; }
  a = i >> 1;
  b = (i & 1) ? a + 1 : a - 1;
  if (b < 0 || b >= nc) b = a;
}

// Value of the up-sampled coarse correction at fine cell (i, j, k) of grid G.
template <typename S>
__device__ __forceinline__ typename Ty<S>::C prolong_value(const S* __restrict__ ec, const GridDesc& G,
                                                          int i, int j, int k, int mode) {
  using C = typename Ty<S>::C;
  const S* e = ec + G.coff;
  const int64_t cpl = (int64_t)G.cnx * G.cny;
  if (mode == 1) {
    return Ty<S>::ld(e + (int64_t)(k / G.fz) * cpl + (int64_t)(j / G.fy) * G.cnx + (i / G.fx));
  }
  int ia, ib, ja, jb, ka, kb;
  lin_idx(i, G.fx, G.cnx, ia, ib);
  lin_idx(j, G.fy, G.cny, ja, jb);
  lin_idx(k, G.fz, G.cnz, ka, kb);
  const C wa = (C)0.75, wb = (C)0.25;
  const S* pa = e + (int64_t)ka * cpl;
  const S* pb = e + (int64_t)kb * cpl;
  auto row = [&](const S* p, int jj) {
    const S* q = p + (int64_t)jj * G.cnx;
    return wa * Ty<S>::ld(q + ia) + wb * Ty<S>::ld(q + ib);
  };
  const C za = wa * row(pa, ja) + wb * row(pa, jb);
  const C zb = wa * row(pb, ja) + wb * row(pb, jb);
  return wa * za + wb * zb;
}

// ------------------------------------------------------- red-black sweep
//
// One complete red-black Gauss-Seidel sweep (Sec. 4.1, multi-coloured GS),
// out of place: reads x_in, writes x_out.  A block owns a TX x TY column of
// the grid and marches along z, keeping four planes of x (with a 2-cell
// in-plane halo) and four planes of b (1-cell halo) in LDS:
//   step p:  red voxels of plane p on the tile plus a 1-cell ring (from
//            old black values), then black voxels of plane p - 1 on the tile
//            (from the new red values of planes p-2..p), then plane p - 1 is
//            written and plane p + 2 enters the ring.
// Recomputing the red ring makes every tile independent of its neighbours,
// so blocks never exchange data and the sweep equals the sequential
// definition exactly.  When e_coarse != NULL the prolongated coarse
// correction is added to x while it is loaded (fused up-sampling).

template <typename S>
__global__ void __launch_bounds__(256)
k_rb_sweep(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids,
           int zlen, const S* __restrict__ xin, S* __restrict__ xout, const S* __restrict__ bin,
           const S* __restrict__ ec, int pmode) {
  using C = typename Ty<S>::C;
  constexpr int TX = SW_TX, TY = SW_TY;
  constexpr int HX = TX + 4, HY = TY + 4;   // x tile with 2-cell halo
  constexpr int BX = TX + 2, BY = TY + 2;   // b tile with 1-cell halo
  constexpr int NXL = (HX * HY + 255) / 256;
  constexpr int NBL = (BX * BY + 255) / 256;
  __shared__ C X[4][HY][HX];
  __shared__ C B[4][BY][BX];

  const Tile t = decode_tile<TX, TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const C alpha = (C)G.alpha, wx = (C)G.wx, wy = (C)G.wy, wz = (C)G.wz;
  const int64_t pl = (int64_t)nx * ny;
  const S* xg = xin + G.off;
  const S* bg = bin + G.off;
  S* xo = xout + G.off;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;

  C rx[NXL], rb[NBL];
  auto fetch = [&](int q) {  // global -> registers, plane q (x) and q - 1 (b)
#pragma unroll
    for (int k = 0; k < NXL; ++k) {
      const int i = tid + 256 * k;
      const int hy = i / HX, hx = i - hy * HX;
      const int gx = x0 - 2 + hx, gy = y0 - 2 + hy;
      C v = (C)0;
      if (i < HX * HY && q >= 0 && q < nz && gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
        v = Ty<S>::ld(xg + q * pl + (int64_t)gy * nx + gx);
        if (ec) v += prolong_value<S>(ec, G, gx, gy, q, pmode);
      }
      rx[k] = v;
    }
    const int qb = q - 1;
#pragma unroll
    for (int k = 0; k < NBL; ++k) {
      const int i = tid + 256 * k;
      const int by = i / BX, bx = i - by * BX;
      const int gx = x0 - 1 + bx, gy = y0 - 1 + by;
      C v = (C)0;
      if (i < BX * BY && qb >= 0 && qb < nz && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
        v = Ty<S>::ld(bg + qb * pl + (int64_t)gy * nx + gx);
      rb[k] = v;
    }
  };
  auto stash = [&](int q) {  // registers -> LDS slots of planes q (x), q - 1 (b)
    const int sx = q & 3, sb = (q - 1) & 3;
#pragma unroll
    for (int k = 0; k < NXL; ++k) {
      const int i = tid + 256 * k;
      if (i < HX * HY) (&X[sx][0][0])[i] = rx[k];
    }
#pragma unroll
    for (int k = 0; k < NBL; ++k) {
      const int i = tid + 256 * k;
      if (i < BX * BY) (&B[sb][0][0])[i] = rb[k];
    }
  };
  // zero-residual update of the voxel at LDS x coords (hy, hx), plane p
  auto relax = [&](int p, int hy, int hx, int by, int bx, int gx, int gy) {
    const int s0 = p & 3;
    const C xc = X[s0][hy][hx];
    C r = B[s0][by][bx] - alpha * xc;
    C d = alpha;
    if (gx > 0) { r += wx * (X[s0][hy][hx - 1] - xc); d += wx; }
    if (gx < nx - 1) { r += wx * (X[s0][hy][hx + 1] - xc); d += wx; }
    if (gy > 0) { r += wy * (X[s0][hy - 1][hx] - xc); d += wy; }
    if (gy < ny - 1) { r += wy * (X[s0][hy + 1][hx] - xc); d += wy; }
    if (p > 0) { r += wz * (X[(p - 1) & 3][hy][hx] - xc); d += wz; }
    if (p < nz - 1) { r += wz * (X[(p + 1) & 3][hy][hx] - xc); d += wz; }
    X[s0][hy][hx] = d > (C)0 ? xc + r / d : (C)0;
  };

  const int pfirst = max(q0 - 1, 0);
  const int plast = (q1 < nz) ? q1 : nz;  // p == nz: black of the last plane only
  // prologue: x planes pfirst-1 .. pfirst+1 and b plane pfirst
  fetch(pfirst - 1); stash(pfirst - 1);
  fetch(pfirst);     stash(pfirst);
  fetch(pfirst + 1); stash(pfirst + 1);
  fetch(pfirst + 2);  // in flight: x plane pfirst+2, b plane pfirst+1

  for (int p = pfirst; p <= plast; ++p) {
    __syncthreads();
    if (p < nz) {  // red voxels of plane p on the tile and its 1-cell ring
      for (int i = tid; i < BY * (BX / 2); i += 256) {
        const int ry = i / (BX / 2), m = i - ry * (BX / 2);
        const int gy = y0 - 1 + ry;
        const int rxx = 2 * m + ((x0 - 1 + gy + p) & 1);
        const int gx = x0 - 1 + rxx;
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) relax(p, ry + 1, rxx + 1, ry, rxx, gx, gy);
      }
    }
    __syncthreads();
    const int q = p - 1;  // black voxels of plane q on the tile
    const bool outq = q >= q0 && q < q1;
    if (outq) {
      for (int i = tid; i < TY * (TX / 2); i += 256) {
        const int ty = i / (TX / 2), m = i - ty * (TX / 2);
        const int gy = y0 + ty;
        const int txx = 2 * m + ((x0 + gy + q + 1) & 1);
        const int gx = x0 + txx;
        if (gx < nx && gy < ny) relax(q, ty + 2, txx + 2, ty + 1, txx + 1, gx, gy);
      }
    }
    __syncthreads();
    if (outq) {
      for (int i = tid; i < TY * TX; i += 256) {
        const int ty = i / TX, tx = i - ty * TX;
        const int gx = x0 + tx, gy = y0 + ty;
        if (gx < nx && gy < ny) Ty<S>::st(xo + q * pl + (int64_t)gy * nx + gx, X[q & 3][ty + 2][tx + 2]);
      }
    }
    stash(p + 2);
    if (p + 1 <= plast) fetch(p + 3);
  }
}

// ------------------------------------------- residual + restriction (gather)
//
// One thread per coarse cell: the residual of each of its (up to 8) children
// is evaluated and summed into the coarse right-hand side (the transpose of
// piecewise-constant up-sampling), and the coarse unknown is zeroed.  The
// per-block FP64 sum of r^2 over the fine cells feeds the residual norm.
template <typename S>
__global__ void __launch_bounds__(256)
k_residual_restrict(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids,
                    int zlen, const S* __restrict__ xin, const S* __restrict__ bin, S* __restrict__ bc,
                    S* __restrict__ xc, double* __restrict__ partials) {
  using C = typename Ty<S>::C;
  __shared__ double red[4];
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, true);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const C alpha = (C)G.alpha, wx = (C)G.wx, wy = (C)G.wy, wz = (C)G.wz;
  const int64_t pl = (int64_t)nx * ny;
  const int64_t cpl = (int64_t)G.cnx * G.cny;
  const S* x = xin + G.off;
  const S* b = bin + G.off;
  const int I = t.x0 + (threadIdx.x & 63), J = t.y0 + (threadIdx.x >> 6);
  double nrm = 0.0;
  if (I < G.cnx && J < G.cny) {
    for (int K = t.z0; K < t.z1; ++K) {
      C sum = (C)0;
      for (int dz = 0; dz < G.fz; ++dz) {
        const int k = K * G.fz + dz;
        if (k >= nz) break;
        for (int dy = 0; dy < G.fy; ++dy) {
          const int j = J * G.fy + dy;
          if (j >= ny) break;
          for (int dx = 0; dx < G.fx; ++dx) {
            const int i = I * G.fx + dx;
            if (i >= nx) break;
            const int64_t v = k * pl + (int64_t)j * nx + i;
            const C xv = Ty<S>::ld(x + v);
            C r = Ty<S>::ld(b + v) - alpha * xv;
            if (i > 0) r += wx * (Ty<S>::ld(x + v - 1) - xv);
            if (i < nx - 1) r += wx * (Ty<S>::ld(x + v + 1) - xv);
            if (j > 0) r += wy * (Ty<S>::ld(x + v - nx) - xv);
            if (j < ny - 1) r += wy * (Ty<S>::ld(x + v + nx) - xv);
            if (k > 0) r += wz * (Ty<S>::ld(x + v - pl) - xv);
            if (k < nz - 1) r += wz * (Ty<S>::ld(x + v + pl) - xv);
            sum += r;
            nrm += (double)r * (double)r;
          }
        }
      }
      const int64_t cv = G.coff + K * cpl + (int64_t)J * G.cnx + I;
      Ty<S>::st(bc + cv, sum);
      if (xc) Ty<S>::st(xc + cv, (C)0);
    }
  }
  if (partials) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// ------------------------------------------------------ prolongation (+=)
template <typename S>
__global__ void __launch_bounds__(256)
k_prolong_add(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
              const S* __restrict__ ec, S* __restrict__ xio, int mode) {
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.nx * G.ny;
  S* x = xio + G.off;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = k * pl + (int64_t)j * G.nx + i;
    Ty<S>::st(x + v, Ty<S>::ld(x + v) + prolong_value<S>(ec, G, i, j, k, mode));
  }
}

// ------------------------------------------- finest level of AD / SP (Eq. 1, 2)
//
// Canonical system of both phases: A = alpha + w_x L_x + w_y L_y + w_z L_z,
// b = alpha I1 + (w_x L_x + w_y L_y) I0 (AD: alpha = 0; SP: w_z = 0).  The
// plain solver iterates on the correction E = x - I0, whose right-hand side
// is b - A I0 = alpha (I1 - I0) - w_z L_z I0.

template <typename Tin>
__device__ __forceinline__ double in_at(const Tin* p, int64_t v) { return ld64(p + v); }

template <typename Tin, typename S>
__global__ void __launch_bounds__(256)
k_rhs_corr(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
           const Tin* __restrict__ I0, const Tin* __restrict__ I1, S* __restrict__ bout,
           S* __restrict__ xout, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  double nrm = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = (int64_t)nx * ny;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
      const double c = in_at(I0, u);
      double lxy = 0.0, lz = 0.0;
      if (i > 0) lxy += G.wx * (c - in_at(I0, u - 1));
      if (i < nx - 1) lxy += G.wx * (c - in_at(I0, u + 1));
      if (j > 0) lxy += G.wy * (c - in_at(I0, u - G.ipy));
      if (j < ny - 1) lxy += G.wy * (c - in_at(I0, u + G.ipy));
      if (G.wz != 0.0) {
        if (k > 0) lz += in_at(I0, u - G.ipz) - c;
        if (k < nz - 1) lz += in_at(I0, u + G.ipz) - c;
      }
      double bcan = lxy, bcorr = G.wz * lz;
      if (G.alpha != 0.0) {
        const double v1 = in_at(I1, u);
        bcan += G.alpha * v1;
        bcorr += G.alpha * (v1 - c);
      }
      nrm += bcan * bcan;
      const int64_t v = G.off + k * pl + (int64_t)j * nx + i;
      if (bout) st64(bout + v, bcorr);
      if (xout) st64(xout + v, 0.0);
    }
  }
  if (partials) {
    const double s = block_sum(nrm, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// x at packed index v / caller index u: I0 + E (mode 0) or x64 (mode 1)
template <typename Tin, typename S, int MODE>
__device__ __forceinline__ double xval(const Tin* I0, const S* E, const double* x64, int64_t u, int64_t v) {
  if (MODE == 0) return in_at(I0, u) + ld64(E + v);
  return x64[v];
}

template <typename Tin, typename S, int MODE>
__global__ void __launch_bounds__(256)
k_canon_residual(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids,
                 int zlen, const Tin* __restrict__ I0, const Tin* __restrict__ I1, const S* __restrict__ E,
                 const double* __restrict__ x64, S* __restrict__ rout, const double* __restrict__ inv_scale,
                 double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  const S* Eg = (MODE == 0) ? E + G.off : E;
  const double* xg = (MODE == 1) ? x64 + G.off : x64;
  double nrm = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = (int64_t)nx * ny;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
      const int64_t v = k * pl + (int64_t)j * nx + i;
      const double c0 = in_at(I0, u);
      const double xc = xval<Tin, S, MODE>(I0, Eg, xg, u, v);
      double r = -G.alpha * xc;  // b - A x, difference form
      if (G.alpha != 0.0) r += G.alpha * in_at(I1, u);
      if (i > 0) r += G.wx * ((c0 - in_at(I0, u - 1)) + (xval<Tin, S, MODE>(I0, Eg, xg, u - 1, v - 1) - xc));
      if (i < nx - 1) r += G.wx * ((c0 - in_at(I0, u + 1)) + (xval<Tin, S, MODE>(I0, Eg, xg, u + 1, v + 1) - xc));
      if (j > 0) r += G.wy * ((c0 - in_at(I0, u - G.ipy)) + (xval<Tin, S, MODE>(I0, Eg, xg, u - G.ipy, v - nx) - xc));
      if (j < ny - 1) r += G.wy * ((c0 - in_at(I0, u + G.ipy)) + (xval<Tin, S, MODE>(I0, Eg, xg, u + G.ipy, v + nx) - xc));
      if (G.wz != 0.0) {
        if (k > 0) r += G.wz * (xval<Tin, S, MODE>(I0, Eg, xg, u - G.ipz, v - pl) - xc);
        if (k < nz - 1) r += G.wz * (xval<Tin, S, MODE>(I0, Eg, xg, u + G.ipz, v + pl) - xc);
      }
      nrm += r * r;
      if (rout) st64(rout + G.off + v, r * inv_scale[t.g]);
    }
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename Tin, typename S, int MODE>
__global__ void __launch_bounds__(256)
k_sum_shift(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
            const Tin* __restrict__ I0, const S* __restrict__ E, const double* __restrict__ x64,
            double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  double s = 0.0;
  if (i < G.nx && j < G.ny) {
    const int64_t pl = (int64_t)G.nx * G.ny;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = G.off + k * pl + (int64_t)j * G.nx + i;
      if (MODE == 0) {
        s += ld64(E + v);
      } else {
        const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
        s += x64[v] - in_at(I0, u);
      }
    }
  }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

template <typename Tin, typename S, typename Tout, int MODE>
__global__ void __launch_bounds__(256)
k_finalize(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
           const Tin* __restrict__ I0, const S* __restrict__ E, const double* __restrict__ x64,
           const double* __restrict__ shift, Tout* __restrict__ out) {
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.nx * G.ny;
  const double sh = shift ? shift[t.g] : 0.0;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
    const int64_t v = G.off + k * pl + (int64_t)j * G.nx + i;
    const double x = (MODE == 0) ? in_at(I0, u) + ld64(E + v) : x64[v];
    st64(out + u, x - sh);
  }
}

template <typename Tin>
__global__ void __launch_bounds__(256)
k_refine_init(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
              const Tin* __restrict__ I0, double* __restrict__ x64) {
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.nx * G.ny;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
    x64[G.off + k * pl + (int64_t)j * G.nx + i] = in_at(I0, u);
  }
}

template <typename S>
__global__ void __launch_bounds__(256)
k_refine_update(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
                double* __restrict__ x64, const S* __restrict__ e, const double* __restrict__ scale) {
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.nx * G.ny;
  const double s = scale[t.g];
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = G.off + k * pl + (int64_t)j * G.nx + i;
    x64[v] += s * ld64(e + v);
  }
}

// -------------------------------------------------- general system (Sec. 4)
template <typename S>
__global__ void __launch_bounds__(256)
k_rhs_general(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
              const S* __restrict__ V, const S* __restrict__ Gx, const S* __restrict__ Gy,
              const S* __restrict__ Gz, S* __restrict__ bout) {
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  const int64_t pl = (int64_t)nx * ny;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = G.off + k * pl + (int64_t)j * nx + i;
    double b = 0.0;
    if (G.alpha != 0.0) b += G.alpha * ld64(V + v);
    // (D_a^T g)_v = g[v - e_a] - g[v]; faces outside the grid carry nothing
    if (Gx && G.wx != 0.0) {
      double d = 0.0;
      if (i > 0) d += ld64(Gx + v - 1);
      if (i < nx - 1) d -= ld64(Gx + v);
      b += G.wx * d;
    }
    if (Gy && G.wy != 0.0) {
      double d = 0.0;
      if (j > 0) d += ld64(Gy + v - nx);
      if (j < ny - 1) d -= ld64(Gy + v);
      b += G.wy * d;
    }
    if (Gz && G.wz != 0.0) {
      double d = 0.0;
      if (k > 0) d += ld64(Gz + v - pl);
      if (k < nz - 1) d -= ld64(Gz + v);
      b += G.wz * d;
    }
    st64(bout + v, b);
  }
}

template <typename S>
__global__ void __launch_bounds__(256)
k_general_residual(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids,
                   int zlen, const S* __restrict__ xin, const S* __restrict__ bin, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile<EW_TX, EW_TY>(grids, block0, ngrids, zlen, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x & 63), j = t.y0 + (threadIdx.x >> 6);
  double rr = 0.0, bb = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = (int64_t)nx * ny;
    const S* x = xin + G.off;
    const S* b = bin + G.off;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = k * pl + (int64_t)j * nx + i;
      const double xc = ld64(x + v), bv = ld64(b + v);
      double r = bv - G.alpha * xc;
      if (i > 0) r += G.wx * (ld64(x + v - 1) - xc);
      if (i < nx - 1) r += G.wx * (ld64(x + v + 1) - xc);
      if (j > 0) r += G.wy * (ld64(x + v - nx) - xc);
      if (j < ny - 1) r += G.wy * (ld64(x + v + nx) - xc);
      if (k > 0) r += G.wz * (ld64(x + v - pl) - xc);
      if (k < nz - 1) r += G.wz * (ld64(x + v + pl) - xc);
      rr += r * r;
      bb += bv * bv;
    }
  }
  const double s1 = block_sum(rr, red);
  const double s2 = block_sum(bb, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s1;
    partials[2 * blockIdx.x + 1] = s2;
  }
}

// ------------------------------------------------------------ reduction
// One block per grid sums that grid's block partials in a fixed order.
__global__ void __launch_bounds__(256)
k_reduce(const double* __restrict__ partials, const int64_t* __restrict__ block0, int ncomp,
         double* __restrict__ out) {
  __shared__ double red[4];
  const int g = blockIdx.x;
  const int64_t b0 = block0[g], b1 = block0[g + 1];
  for (int c = 0; c < ncomp; ++c) {
    double s = 0.0;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) s += partials[b * ncomp + c];
    const double tot = block_sum(s, red);
    if (threadIdx.x == 0) out[g * ncomp + c] = tot;
  }
}

// ============================================================ launchers

#define GD_ARGS(geom) dim3((unsigned)(geom).nblocks), dim3(256), 0, st, (geom).grids, (geom).block0, (geom).ngrids, (geom).zlen

#define GD_DISPATCH_S(s, MACRO)                        \
  switch (s) {                                         \
    case GD_F64: MACRO(double); break;                 \
    case GD_F32: MACRO(float); break;                  \
    case GD_F16: MACRO(__half); break;                 \
    case GD_BF16: MACRO(__hip_bfloat16); break;        \
    default: return hipErrorInvalidValue;              \
  }

#define GD_DISPATCH_S2(s, T1, MACRO)                   \
  switch (s) {                                         \
    case GD_F64: MACRO(T1, double); break;             \
    case GD_F32: MACRO(T1, float); break;              \
    case GD_F16: MACRO(T1, __half); break;             \
    case GD_BF16: MACRO(T1, __hip_bfloat16); break;    \
    default: return hipErrorInvalidValue;              \
  }

static hipError_t last() { return hipGetLastError(); }

hipError_t launch_rb_sweep(gd_dtype s, const Geom& g, const void* xin, void* xout, const void* b,
                           const void* ec, int pmode, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_rb_sweep<T>, GD_ARGS(g), (const T*)xin, (T*)xout, (const T*)b, (const T*)ec, pmode)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_residual_restrict(gd_dtype s, const Geom& g, const void* x, const void* b, void* bc,
                                    void* xc, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_residual_restrict<T>, GD_ARGS(g), (const T*)x, (const T*)b, (T*)bc, (T*)xc, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_prolong_add(gd_dtype s, const Geom& g, const void* ec, void* x, int mode, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_prolong_add<T>, GD_ARGS(g), (const T*)ec, (T*)x, mode)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_rhs_corr(gd_dtype tin, gd_dtype s, const Geom& g, const void* I0, const void* I1, void* b,
                           void* x, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T) hipLaunchKernelGGL((k_rhs_corr<TI, T>), GD_ARGS(g), (const TI*)I0, (const TI*)I1, (T*)b, (T*)x, partials)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  return last();
}

hipError_t launch_canon_residual(gd_dtype tin, gd_dtype s, int mode, const Geom& g, const void* I0,
                                 const void* I1, const void* E, const double* x64, void* r_out,
                                 const double* inv_scale, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T)                                                                                          \
  if (mode == 0)                                                                                           \
    hipLaunchKernelGGL((k_canon_residual<TI, T, 0>), GD_ARGS(g), (const TI*)I0, (const TI*)I1, (const T*)E, \
                       x64, (T*)r_out, inv_scale, partials);                                               \
  else                                                                                                     \
    hipLaunchKernelGGL((k_canon_residual<TI, T, 1>), GD_ARGS(g), (const TI*)I0, (const TI*)I1, (const T*)E, \
                       x64, (T*)r_out, inv_scale, partials)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  return last();
}

hipError_t launch_sum_shift(gd_dtype tin, gd_dtype s, int mode, const Geom& g, const void* I0, const void* E,
                            const double* x64, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T)                                                                                             \
  if (mode == 0)                                                                                              \
    hipLaunchKernelGGL((k_sum_shift<TI, T, 0>), GD_ARGS(g), (const TI*)I0, (const T*)E, x64, partials);        \
  else                                                                                                        \
    hipLaunchKernelGGL((k_sum_shift<TI, T, 1>), GD_ARGS(g), (const TI*)I0, (const T*)E, x64, partials)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  return last();
}

template <typename TI, typename T>
static hipError_t finalize_out(gd_dtype tout, int mode, const Geom& g, const void* I0, const void* E,
                               const double* x64, const double* shift, void* out, hipStream_t st) {
#define L(TO)                                                                                                \
  if (mode == 0)                                                                                             \
    hipLaunchKernelGGL((k_finalize<TI, T, TO, 0>), GD_ARGS(g), (const TI*)I0, (const T*)E, x64, shift, (TO*)out); \
  else                                                                                                       \
    hipLaunchKernelGGL((k_finalize<TI, T, TO, 1>), GD_ARGS(g), (const TI*)I0, (const T*)E, x64, shift, (TO*)out)
  GD_DISPATCH_S(tout, L)
#undef L
  return hipSuccess;
}

hipError_t launch_finalize(gd_dtype tin, gd_dtype s, gd_dtype tout, int mode, const Geom& g, const void* I0,
                           const void* E, const double* x64, const double* shift, void* out, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define L2(TI, T) e = finalize_out<TI, T>(tout, mode, g, I0, E, x64, shift, out, st)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  if (e != hipSuccess) return e;
  return last();
}

hipError_t launch_refine_init(gd_dtype tin, const Geom& g, const void* I0, double* x64, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_refine_init<T>, GD_ARGS(g), (const T*)I0, x64)
  GD_DISPATCH_S(tin, L)
#undef L
  return last();
}

hipError_t launch_refine_update(gd_dtype s, const Geom& g, double* x64, const void* e, const double* scale,
                                hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_refine_update<T>, GD_ARGS(g), x64, (const T*)e, scale)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_rhs_general(gd_dtype s, const Geom& g, const void* V, const void* Gx, const void* Gy,
                              const void* Gz, void* b, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_rhs_general<T>, GD_ARGS(g), (const T*)V, (const T*)Gx, (const T*)Gy, (const T*)Gz, (T*)b)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_general_residual(gd_dtype s, const Geom& g, const void* x, const void* b, double* partials,
                                   hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_general_residual<T>, GD_ARGS(g), (const T*)x, (const T*)b, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_reduce(const double* partials, const int64_t* block0, int ngrids, int ncomp, double* out,
                         hipStream_t st) {
  if (ngrids == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3(ngrids), dim3(256), 0, st, partials, block0, ncomp, out);
  return last();
}

}  // namespace gd
