// gfx950 kernels of the multigrid solver for the screened anisotropic Poisson
// systems of Kazhdan et al., "Gradient-Domain Processing for Large EM Image
// Stacks" (Sec. 4 operator, Sec. 4.1 multigrid steps, Sec. 4.2 7-point
// stencil).  Every level operator is alpha*Id + sum_a w_a L_a, L_a the
// 3-point Neumann second difference along axis a (no faces outside the grid).
//
// Layout: a grid's array is [nz][ny][px] with x pitch px >= nx (the library's
// own arrays pad px to a multiple of 4 so that x pairs are aligned; arrays
// given by a caller use px = nx).  A 2-D slice is described as nz = its rows,
// ny = 1, so that every kernel marches along the slowest axis.
//
// All stencils are evaluated in difference form, sum_nb w (x_nb - x_c), which
// keeps the rounding error proportional to the local variation instead of
// the magnitude of x.
#include <cstdlib>
#include <type_traits>
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
  int64_t bid;  // logical block index (per-block partial sums go here)
};

// Logical block index.  Work-groups go to the 8 XCDs round-robin and each
// XCD has its own L2.  Order 1 hands XCD x a contiguous run of tiles, so
// that the halos of neighbouring tiles are fetched into one L2 (used by the
// relaxation of slice batches); order 0 is the plain order.
__device__ __forceinline__ int64_t xcd_block(int order = 0) {
  if (order != 1) return blockIdx.x;
  // XCD x = b mod 8 takes the contiguous run [x q + min(x, r), ...) of
  // logical blocks (q = n / 8, r = n mod 8): a bijection of [0, n)
  const int64_t b = blockIdx.x, n = gridDim.x;
  const int64_t q = n >> 3, r = n & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Decode blockIdx.x into (grid, tile, z-range) for tx x ty tiles over the
// grid's own size (coarse = false) or its child's size (coarse = true).
__device__ __forceinline__ Tile decode_tile(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0,
                                            int ngrids, int zlen, int tx_, int ty_, bool coarse,
                                            int order = 0) {
  Tile t;
  const int64_t bid = xcd_block(order);
  t.bid = bid;
  t.g = find_grid(block0, ngrids, bid);
  const GridDesc& G = grids[t.g];
  const int nx = coarse ? G.cnx : G.nx, ny = coarse ? G.cny : G.ny, nz = coarse ? G.cnz : G.nz;
  const int64_t local = bid - block0[t.g];
  const int tx = (nx + tx_ - 1) / tx_, ty = (ny + ty_ - 1) / ty_;
  const int64_t txy = (int64_t)tx * ty;
  const int zc = (int)(local / txy);
  const int r = (int)(local - (int64_t)zc * txy);
  t.x0 = (r % tx) * tx_;
  t.y0 = (r / tx) * ty_;
  t.z0 = zc * zlen;
  t.z1 = min(t.z0 + zlen, nz);
  return t;
}

// Cell-centred linear up-sampling along one axis: the fine cell i of a
// halved axis takes 3/4 of its parent i/2 and 1/4 of the nearer coarse
// neighbour; where that neighbour is outside the grid the parent takes weight
// 1 (mirror boundary).  A kept axis (f == 1) maps i to i with weight 1.
// two == false means the single index a carries weight 1.
__device__ __forceinline__ bool lin_idx(int i, int f, int nc, int& a, int& b) {
  if (f == 1) { a = b = i; return false; }
  a = i >> 1;
  b = (i & 1) ? a + 1 : a - 1;
  if (b < 0 || b >= nc) { b = a; return false; }
  return true;
}

template <typename C>
__device__ __forceinline__ C lin_mix(bool two, C va, C vb) {
  return two ? (C)0.75 * va + (C)0.25 * vb : va;
}

// Value of the up-sampled coarse correction at fine cell (i, j, k) of grid G:
// x first, then y, then z (prolong_pair evaluates the same expression).
template <typename S>
__device__ __forceinline__ typename Ty<S>::C prolong_value(const S* __restrict__ ec, const GridDesc& G,
                                                          int i, int j, int k, int mode) {
  using C = typename Ty<S>::C;
  const S* e = ec + G.coff;
  const int64_t cpl = (int64_t)G.cpx * G.cny;
  if (mode == 1) {
    return Ty<S>::ld(e + (int64_t)(k / G.fz) * cpl + (int64_t)(j / G.fy) * G.cpx + (i / G.fx));
  }
  int ia, ib, ja, jb, ka, kb;
  const bool tx = lin_idx(i, G.fx, G.cnx, ia, ib);
  const bool ty = lin_idx(j, G.fy, G.cny, ja, jb);
  const bool tz = lin_idx(k, G.fz, G.cnz, ka, kb);
  auto row = [&](int kk, int jj) {
    const S* q = e + (int64_t)kk * cpl + (int64_t)jj * G.cpx;
    return lin_mix<C>(tx, Ty<S>::ld(q + ia), tx ? Ty<S>::ld(q + ib) : (C)0);
  };
  auto plane = [&](int kk) { return lin_mix<C>(ty, row(kk, ja), ty ? row(kk, jb) : (C)0); };
  return lin_mix<C>(tz, plane(ka), tz ? plane(kb) : (C)0);
}

// The same for the x-pair (i, i + 1), i even, of the library's arrays (child
// pitch a multiple of 4): the pair shares its coarse rows.
template <typename S>
__device__ __forceinline__ void prolong_pair(const S* __restrict__ ec, const GridDesc& G, int i, int j, int k,
                                             int mode, typename Ty<S>::C& va, typename Ty<S>::C& vb) {
  using C = typename Ty<S>::C;
  const S* e = ec + G.coff;
  const int64_t cpl = (int64_t)G.cpx * G.cny;
  if (mode == 1) {
    const S* r = e + (int64_t)(k / G.fz) * cpl + (int64_t)(j / G.fy) * G.cpx;
    va = Ty<S>::ld(r + i / G.fx);
    vb = Ty<S>::ld(r + (i + 1) / G.fx);
    return;
  }
  int ja, jb, ka, kb;
  const bool ty = lin_idx(j, G.fy, G.cny, ja, jb);
  const bool tz = lin_idx(k, G.fz, G.cnz, ka, kb);
  int iaA, ibA, iaB, ibB;
  const bool txA = lin_idx(i, G.fx, G.cnx, iaA, ibA);
  const bool txB = lin_idx(i + 1, G.fx, G.cnx, iaB, ibB);
  auto rows = [&](int kk, int jj, C& ra, C& rb) {
    const S* q = e + (int64_t)kk * cpl + (int64_t)jj * G.cpx;
    if (G.fx == 1) {
      ld2(q + i, true, true, ra, rb);  // kept axis: weight 1 on i and i + 1
    } else {
      const C c0 = Ty<S>::ld(q + iaA);  // the pair's common parent
      ra = lin_mix<C>(txA, c0, txA ? Ty<S>::ld(q + ibA) : (C)0);
      rb = lin_mix<C>(txB, c0, txB ? Ty<S>::ld(q + ibB) : (C)0);
    }
  };
  auto planes = [&](int kk, C& pa, C& pb) {
    C a0, b0, a1 = 0, b1 = 0;
    rows(kk, ja, a0, b0);
    if (ty) rows(kk, jb, a1, b1);
    pa = lin_mix<C>(ty, a0, a1);
    pb = lin_mix<C>(ty, b0, b1);
  };
  C a0, b0, a1 = 0, b1 = 0;
  planes(ka, a0, b0);
  if (tz) planes(kb, a1, b1);
  va = lin_mix<C>(tz, a0, a1);
  vb = lin_mix<C>(tz, b0, b1);
}

// ------------------------------------------------------- red-black sweep
//
// One complete red-black Gauss-Seidel sweep (Sec. 4.1, multi-coloured GS),
// out of place: reads x_in, writes x_out.  A block owns a TX x TY column of
// the grid and marches along z.  Thread t owns the x-pair (x0 + 2 (t mod
// TX/2), y0 + t / (TX/2)) and its two neighbours along x: in every plane one
// of the pair is red and the other black, and the z-neighbours of a cell are
// cells of the same column, so each thread keeps its column of planes
// p-2 .. p+2 in registers and only the in-plane neighbours go through LDS
// (four planes, with a 2-cell halo ring loaded by the threads in turn).
//   step p:  barrier | red cells of plane p (own pair and the 1-cell ring
//            around the tile, from old black values), written to plane p's
//            LDS buffer | black cells of plane p - 1 (from the new red values
//            of planes p-2..p: in-plane ones from plane p - 1's buffer,
//            written in the previous step), plane p - 1 written to memory,
//            plane p + 2 enters LDS (the buffer plane p - 2 used)
// One barrier per plane suffices: within a step no buffer is both written
// and read (red cells of plane p are written, only black cells of plane p
// and planes p +- 1 are read; plane p - 1 is read; plane p + 2 is written).
// Recomputing the red ring makes every tile independent of its neighbours,
// so blocks never exchange data and the sweep equals the sequential
// definition exactly.  Every thread relaxes its red cell and a ring cell in
// each plane (a thread without a ring cell relaxes a stand-in and writes it
// to a slot of its own), so that the LDS reads of both issue together, and
// the plane parity is a compile-time argument of the unrolled step: the
// per-parity weights and inverse diagonals stay in registers.  When
// e_coarse != NULL the up-sampled coarse correction is added to x while it
// is loaded (fused prolongation).
// TY == 1 is the row form for grids with ny == 1 (2-D slices).

template <int TX, int TY>
struct SweepShape {
  static constexpr bool ROW = (TY == 1);
  static constexpr int NT = TX * TY / 2;                 // threads: one x-pair each
  static constexpr int YO = ROW ? 0 : 2;                 // tile row 0 inside the LDS plane
  static constexpr int HX = TX + 4, HY = ROW ? 1 : TY + 4;
  static constexpr int NHALO = HX * HY - TX * TY;        // halo cells per plane
  static constexpr int NHR = (NHALO + NT - 1) / NT;      // halo cells per thread
  static constexpr int NRING = ROW ? 1 : (TX + 2) + TY;  // red ring-1 cells per plane
};

// LDS coordinates of halo cell h (everything of the HY x HX plane outside the tile)
template <int TX, int TY>
__device__ __forceinline__ void halo_cell(int h, int& hy, int& hx) {
  using SS = SweepShape<TX, TY>;
  if constexpr (SS::ROW) {
    hy = 0;
    hx = (h < 2) ? h : TX + h;  // 0, 1, TX + 2, TX + 3
  } else {
    constexpr int HX = SS::HX;
    if (h < 2 * HX) { hy = h / HX; hx = h - hy * HX; return; }
    h -= 2 * HX;
    if (h < 2 * HX) { hy = TY + 2 + h / HX; hx = h - (h / HX) * HX; return; }
    h -= 2 * HX;
    hy = 2 + (h >> 2);
    const int c = h & 3;
    hx = (c < 2) ? c : TX + c;  // 0, 1, TX + 2, TX + 3
  }
}

// LDS coordinates of the m-th red cell of the 1-cell ring at plane p
template <int TX, int TY>
__device__ __forceinline__ void ring_red_cell(int m, int x0, int y0, int p, int& hy, int& hx) {
  using SS = SweepShape<TX, TY>;
  if constexpr (SS::ROW) {
    // cells x0 - 1 and x0 + TX of the single row; exactly one is red
    hy = 0;
    hx = ((x0 - 1 + p) & 1) == 0 ? 1 : TX + 2;
    (void)m; (void)y0;
  } else {
    constexpr int HALF = (TX + 2) / 2;
    if (m < 2 * HALF) {  // top (hy = 1) or bottom (hy = TY + 2) row, hx in 1 .. TX + 2
      hy = (m < HALF) ? 1 : TY + 2;
      const int k = (m < HALF) ? m : m - HALF;
      const int s = (x0 + y0 - 2 + hy + p) & 1;  // parity hx must have
      hx = (s ? 1 : 2) + 2 * k;
    } else {  // left (hx = 1) or right (hx = TX + 2) column, hy in 2 .. TY + 1
      const int k = m - 2 * HALF;
      const int HC = TY / 2;
      hx = (k < HC) ? 1 : TX + 2;
      const int kk = (k < HC) ? k : k - HC;
      const int s = (x0 - 2 + hx + y0 - 2 + p) & 1;
      hy = 2 + s + 2 * kk;
    }
  }
}

// Work split of the 1-cell ring and the halo over the waves of a block, so
// that every wave gets the same share.
template <int N, int NT>
struct WaveSplit {
  static constexpr int NW = NT / 64;
  static constexpr int PER = (N + NW - 1) / NW;  // items per wave (<= 64 by construction)
  static __device__ __forceinline__ int item(int tid) {  // -1: none
    const int w = tid >> 6, l = tid & 63;
    const int m = w * PER + l;
    return (l < PER && m < N) ? m : -1;
  }
};

// Gauss-Seidel value of one cell in correction form, x + (b - A x) / d:
// the residual is accumulated from neighbour differences (exact for close
// values), which keeps the FP32 rounding floor low when x is much larger
// than b (small alpha).  Neighbours are taken left, right, up, down, z-1,
// z+1 with explicit fused multiply-adds, so that a ring cell and its owner
// compute it alike.  inv == 0 (no diagonal) gives 0.
template <typename C>
__device__ __forceinline__ C fmac(C a, C b, C c) {
  if constexpr (sizeof(C) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}
template <typename C, bool ROW>
__device__ __forceinline__ C relax(C x, C b, C alpha, C wl, C nl, C wr, C nr, C wu, C nu, C wd, C nd, C wzm, C nzm,
                                   C wzp, C nzp, C inv) {
  C r = fmac(-alpha, x, b);
  r = fmac(wl, nl - x, r);
  r = fmac(wr, nr - x, r);
  if (!ROW) {
    r = fmac(wu, nu - x, r);
    r = fmac(wd, nd - x, r);
  }
  r = fmac(wzm, nzm - x, r);
  r = fmac(wzp, nzp - x, r);
  return inv != (C)0 ? fmac(r, inv, x) : (C)0;
}

template <typename S, int TX, int TY, bool FP, bool VEC>
__global__ void __launch_bounds__(TX * TY / 2)
k_rb_sweep(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
           const S* __restrict__ xin, S* __restrict__ xout, const S* __restrict__ bin,
           const S* __restrict__ ec, int pmode, int order) {
  using C = typename Ty<S>::C;
  using SS = SweepShape<TX, TY>;
  constexpr int NT = SS::NT, YO = SS::YO, HX = SS::HX, HY = SS::HY, NHR = SS::NHR;
  constexpr int PLANE = HX * HY;
  constexpr bool ROW = SS::ROW;
  using Ring = WaveSplit<SS::NRING, NT>;
  static_assert(Ring::PER <= 64, "ring share per wave");
  // four planes, then one slot per thread that takes the masked writes of
  // threads without a ring cell
  __shared__ C X[4 * PLANE + NT];

  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false, order);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const C alpha = (C)G.alpha, wx = (C)G.wx, wy = (C)G.wy, wz = (C)G.wz;
  const int64_t pl = (int64_t)px * ny;
  const S* xg = xin + G.off;
  const S* bg = bin + G.off;
  S* xo = xout + G.off;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;

  // ---- own pair (gx, gx + 1) of row gy
  const int tyl = tid / (TX / 2), pxl = tid - tyl * (TX / 2);
  const int gx = x0 + 2 * pxl, gy = y0 + tyl;
  const bool rowok = gy < ny;
  const bool vA = rowok && gx < nx, vB = rowok && gx + 1 < nx;
  const int lo = (YO + tyl) * HX + 2 + 2 * pxl;  // LDS index of gx inside a plane
  const int own = gy * px + gx;                 // element offset inside a plane (< 2^28)
  const C wU = (gy > 0) ? wy : (C)0, wD = (gy + 1 < ny) ? wy : (C)0;
  // per plane parity par = p & 1 the red cell of the pair is at position cp = (gy + par) & 1
  int offO[2], offY[2];
  C wO[2], wP[2], wL[2], wR[2], invI[2], invE[2];
  bool vR[2];
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    const int cp = (gy + par) & 1;
    offO[par] = cp ? lo + 2 : lo - 1;
    offY[par] = lo + cp;
    wO[par] = (cp ? (gx + 2 < nx) : (gx > 0)) ? wx : (C)0;
    wP[par] = (cp ? true : vB) ? wx : (C)0;
    vR[par] = cp ? vB : vA;  // the red cell of plane p (and black cell of plane p - 1) exists
    // left, right, up, down, then z: the order the 1-cell ring uses too, so
    // that a ring cell and its owner round alike and every tile shape gives
    // the same values
    wL[par] = cp ? wP[par] : wO[par];  // left neighbour: the pair partner when the cell is gx + 1
    wR[par] = cp ? wO[par] : wP[par];
    const C dxy = alpha + wL[par] + wR[par] + wU + wD;
    // diagonal inside the z-range and on its first or last plane
    const C wz1 = nz > 1 ? wz : (C)0;
    const C di = (dxy + wz1) + wz1, de = dxy + wz1;
    invI[par] = di > (C)0 ? (C)1 / di : (C)0;
    invE[par] = de > (C)0 ? (C)1 / de : (C)0;
  }

  // ---- halo cells of this thread (loaded every plane)
  int hoff[NHR], hg[NHR];
  bool hv[NHR], hs[NHR];
#pragma unroll
  for (int k = 0; k < NHR; ++k) {
    int h;
    if (k < NHR - 1) {
      h = tid + NT * k;
    } else {  // last round: spread the remainder over the waves
      const int m = WaveSplit<SS::NHALO - NT * (NHR - 1), NT>::item(tid);
      h = m < 0 ? -1 : NT * k + m;
    }
    int hy = 0, hx = 0;
    if (h >= 0) halo_cell<TX, TY>(h, hy, hx);
    const int cx = x0 - 2 + hx, cy = y0 - YO + hy;
    hs[k] = h >= 0;
    hv[k] = h >= 0 && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    hoff[k] = hy * HX + hx;
    hg[k] = hv[k] ? cy * px + cx : 0;
  }

  // ---- ring red cell of this thread, for each plane parity
  const int rm = Ring::item(tid);
  int ro[2], rg[2];
  bool rv[2];
  C rwl[2], rwr[2], rwu[2], rwd[2], rinvI[2], rinvE[2];
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    int hy = 0, hx = 0;
    if (rm >= 0) ring_red_cell<TX, TY>(rm, x0, y0, par, hy, hx);
    const int cx = x0 - 2 + hx, cy = y0 - YO + hy;
    rv[par] = rm >= 0 && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    // a thread without a ring cell relaxes its own cell's position as a
    // stand-in (in-plane neighbours inside the LDS plane) and writes the
    // result to its dummy slot
    ro[par] = rm >= 0 ? hy * HX + hx : lo;
    rg[par] = rv[par] ? cy * px + cx : 0;
    rwl[par] = cx > 0 ? wx : (C)0;
    rwr[par] = cx < nx - 1 ? wx : (C)0;
    rwu[par] = cy > 0 ? wy : (C)0;
    rwd[par] = cy < ny - 1 ? wy : (C)0;
    const C dxy = alpha + rwl[par] + rwr[par] + rwu[par] + rwd[par];
    const C wz1 = nz > 1 ? wz : (C)0;
    const C di = (dxy + wz1) + wz1, de = dxy + wz1;
    rinvI[par] = di > (C)0 ? (C)1 / di : (C)0;
    rinvE[par] = de > (C)0 ? (C)1 / de : (C)0;
  }

  // ---- plane loads: x pair + halo (registers), b pair, ring b.  Two planes
  // of x and b are in flight while a plane is relaxed; a loaded value is
  // first touched one or two planes later, so the loads overlap the updates.
  // Values are kept raw (storage format) until stash / split: converting a
  // 16-bit value right after its load would make the wave wait for it there.
  // The plain loads are issued unconditionally from clamped, always valid
  // addresses and masked when used: with no branch around them the compiler
  // can wait for the oldest plane only, keeping the next one in flight.
  struct XSet {
    Raw2<S> p;                      // own pair
    Raw<S> h[NHR];                  // halo cells
    C ea = 0, eb = 0, eh[NHR] = {};  // fused prolongation (FP)
  };
  auto plane_ptr = [&](const S* base, int q) { return base + (int64_t)min(max(q, 0), nz - 1) * pl; };
  auto fetch_x = [&](int q, XSet& o) {
    const S* P = plane_ptr(xg, q);
    if (VEC) {
      ld_raw2(P + (vA ? own : 0), true, true, o.p);
    } else {
      o.p = Raw2<S>();
      if (vA) ld_raw2(P + own, false, vB, o.p);
    }
#pragma unroll
    for (int k = 0; k < NHR; ++k) ld_raw(P + hg[k], o.h[k]);
    if (FP) {
      o.ea = o.eb = (C)0;
#pragma unroll
      for (int k = 0; k < NHR; ++k) o.eh[k] = (C)0;
      if (q >= 0 && q < nz) {
        if (vA) prolong_pair<S>(ec, G, gx, gy, q, pmode, o.ea, o.eb);
#pragma unroll
        for (int k = 0; k < NHR; ++k)
          if (hv[k]) o.eh[k] = prolong_value<S>(ec, G, x0 - 2 + hoff[k] % HX, y0 - YO + hoff[k] / HX, q, pmode);
      }
    }
  };
  auto xa = [&](const XSet& o, int q) -> C {
    const C v = FP ? raw_ca(o.p) + o.ea : raw_ca(o.p);
    return (q >= 0 && q < nz && vA) ? v : (C)0;
  };
  auto xb = [&](const XSet& o, int q) -> C {
    const C v = FP ? raw_cb(o.p) + o.eb : raw_cb(o.p);
    return (q >= 0 && q < nz && vB) ? v : (C)0;
  };
  auto stash = [&](int q, const XSet& o) {
    C* P = X + (q & 3) * PLANE;
    const bool okq = q >= 0 && q < nz;
    P[lo] = xa(o, q);
    P[lo + 1] = xb(o, q);
#pragma unroll
    for (int k = 0; k < NHR; ++k)
      if (hs[k]) P[hoff[k]] = (okq && hv[k]) ? (FP ? raw_c(o.h[k]) + o.eh[k] : raw_c(o.h[k])) : (C)0;
  };
  // b pair of plane q (memory order, raw; masked by bA / bB)
  auto fetch_b = [&](int q, Raw2<S>& r) {
    const S* P = plane_ptr(bg, q);
    if (VEC) {
      ld_raw2(P + (vA ? own : 0), true, true, r);
    } else {
      r = Raw2<S>();
      if (vA) ld_raw2(P + own, false, vB, r);
    }
  };
  auto bA = [&](const Raw2<S>& r, int q) -> C { return (q >= 0 && q < nz && vA) ? raw_ca(r) : (C)0; };
  auto bB = [&](const Raw2<S>& r, int q) -> C { return (q >= 0 && q < nz && vB) ? raw_cb(r) : (C)0; };
  auto ring_b = [&](int q) -> Raw<S> {
    Raw<S> r;
    ld_raw(plane_ptr(bg, q) + rg[q & 1], r);
    return r;
  };
  // pair (in memory order) -> (red, black) of plane q
  auto split = [&](int q, C a, C b, C& r, C& k) {
    const bool cp = ((gy + q) & 1) != 0;
    b = vB ? b : (C)0;
    r = cp ? b : a;
    k = cp ? a : b;
  };

  // column registers (red R / black K of planes p-2 .. p+1), b of planes p-1, p
  C Rm2 = 0, Km2 = 0, Rm1, Km1, R0, K0, Rp1, Kp1;
  C bRm1, bKm1, bR0, bK0;
  // Loads in flight sit in two slots each (plane r in slot (r - pfirst) & 1)
  // and the loop is unrolled by two, so that no in-flight register is ever
  // copied: a copy would make the wave wait for the newest loads.
  XSet S0, S1;
  Raw2<S> B0, B1;
  Raw<S> RB0, RB1;
  const int pfirst = max(q0 - 1, 0);
  const int plast = (q1 < nz) ? q1 : nz;  // p == nz: black of the last plane only
  {
    XSet t0;
    Raw2<S> tb;
    fetch_x(pfirst - 1, t0); stash(pfirst - 1, t0); split(pfirst - 1, xa(t0, pfirst - 1), xb(t0, pfirst - 1), Rm1, Km1);
    fetch_x(pfirst, t0);     stash(pfirst, t0);     split(pfirst, xa(t0, pfirst), xb(t0, pfirst), R0, K0);
    fetch_x(pfirst + 1, t0); stash(pfirst + 1, t0); split(pfirst + 1, xa(t0, pfirst + 1), xb(t0, pfirst + 1), Rp1, Kp1);
    fetch_b(pfirst - 1, tb); split(pfirst - 1, bA(tb, pfirst - 1), bB(tb, pfirst - 1), bRm1, bKm1);
    fetch_b(pfirst, tb);     split(pfirst, bA(tb, pfirst), bB(tb, pfirst), bR0, bK0);
  }
  RB0 = ring_b(pfirst);
  RB1 = ring_b(pfirst + 1);
  fetch_x(pfirst + 2, S0);
  fetch_x(pfirst + 3, S1);
  fetch_b(pfirst + 1, B1);
  fetch_b(pfirst + 2, B0);

  // one plane step: red of plane p, black of plane p - 1, then plane p + 2
  // enters LDS and the loads of planes p + 4 (x), p + 3 (b), p + 2 (ring b)
  // go out into the slots just consumed
  auto step = [&](auto PC, int p, XSet& XS, Raw2<S>& BS, Raw<S>& RBS) {
    constexpr int par = decltype(PC)::value;  // p & 1, fixed per unrolled step
    __syncthreads();
    if (p < nz) {
      // ---- red cells of plane p: the pair's red cell and the ring cell,
      // both computed by every thread (masked), so that their LDS reads
      // issue together
      C* P = X + (p & 3) * PLANE;
      const C* Pm = X + ((p - 1) & 3) * PLANE;
      const C* Pp = X + ((p + 1) & 3) * PLANE;
      const C wzm = p > 0 ? wz : (C)0, wzp = p < nz - 1 ? wz : (C)0;
      const bool edge = p == 0 || p == nz - 1;
      const bool cp = ((gy + p) & 1) != 0;  // red cell on the pair's right
      const C vo = P[offO[par]];
      const C up = ROW ? (C)0 : P[offY[par] - HX], dn = ROW ? (C)0 : P[offY[par] + HX];
      const int o = ro[par];
      const C rx = P[o], rl = P[o - 1], rr = P[o + 1];
      const C ru = ROW ? (C)0 : P[o - HX], rd = ROW ? (C)0 : P[o + HX];
      const C rzm = Pm[o], rzp = Pp[o];
      const C nv = relax<C, ROW>(R0, bR0, alpha, wL[par], cp ? K0 : vo, wR[par], cp ? vo : K0, wU, up, wD, dn, wzm, Km1,
                                 wzp, Kp1, edge ? invE[par] : invI[par]);
      R0 = vR[par] ? nv : (C)0;
      P[offY[par]] = R0;
      const C rb = (p >= 0 && rv[par]) ? raw_c(RBS) : (C)0;
      const C rn = relax<C, ROW>(rx, rb, alpha, rwl[par], rl, rwr[par], rr, rwu[par], ru, rwd[par], rd, wzm, rzm,
                                 wzp, rzp, edge ? rinvE[par] : rinvI[par]);
      *(rv[par] ? P + o : X + 4 * PLANE + tid) = rn;
    }
    // no barrier here: the black cells of plane p - 1 read only plane
    // p - 1's buffer, whose red cells were written in the previous step
    const int q = p - 1;
    if (q >= q0 && q < q1) {
      // ---- black cells of plane q = p - 1 (same position as the red cell of plane p)
      const C* P = X + (q & 3) * PLANE;
      const C wzm = q > 0 ? wz : (C)0, wzp = q < nz - 1 ? wz : (C)0;
      const bool edge = q == 0 || q == nz - 1;
      const bool cq = ((gy + q) & 1) != 0;  // red position of plane q
      // the black cell sits on the pair's right when the red one is on its left
      const C vo = P[offO[par]];
      const C up = ROW ? (C)0 : P[offY[par] - HX], dn = ROW ? (C)0 : P[offY[par] + HX];
      const C nv = relax<C, ROW>(Km1, bKm1, alpha, wL[par], cq ? vo : Rm1, wR[par], cq ? Rm1 : vo, wU, up, wD, dn, wzm,
                                 Rm2, wzp, R0, edge ? invE[par] : invI[par]);
      Km1 = vR[par] ? nv : (C)0;
      if (vA) st2(xo + (int64_t)q * pl + own, VEC, vB, cq ? Km1 : Rm1, cq ? Rm1 : Km1);
    }
    stash(p + 2, XS);
    Rm2 = Rm1; Km2 = Km1; Rm1 = R0; Km1 = K0; R0 = Rp1; K0 = Kp1;
    split(p + 2, xa(XS, p + 2), xb(XS, p + 2), Rp1, Kp1);
    bRm1 = bR0; bKm1 = bK0;
    split(p + 1, bA(BS, p + 1), bB(BS, p + 1), bR0, bK0);
    // next planes (clamped reads past the chunk's end are harmless and keep
    // the loop free of a branch around the loads)
    fetch_x(p + 4, XS);
    fetch_b(p + 3, BS);
    ld_raw(plane_ptr(bg, p + 2) + rg[par], RBS);  // ring b of plane p + 2 (same parity)
  };
  using E0 = std::integral_constant<int, 0>;
  using E1 = std::integral_constant<int, 1>;
  int p = pfirst;
  if ((pfirst & 1) == 0) {
    for (; p + 1 <= plast; p += 2) {
      step(E0{}, p, S0, B1, RB0);
      step(E1{}, p + 1, S1, B0, RB1);
    }
    if (p <= plast) step(E0{}, p, S0, B1, RB0);
  } else {
    for (; p + 1 <= plast; p += 2) {
      step(E1{}, p, S0, B1, RB0);
      step(E0{}, p + 1, S1, B0, RB1);
    }
    if (p <= plast) step(E1{}, p, S0, B1, RB0);
  }
}

// ------------------------------------------------ residual + restriction
//
// r = b - A x on the fine grid, summed into the coarse right-hand side (each
// coarse cell the sum of its children: the transpose of piecewise-constant
// up-sampling), the coarse unknown zeroed, and the per-block FP64 sum of r^2
// over the fine cells for the residual norm.
// A block owns a TX x TY fine tile and marches along z; thread t owns an
// x-pair.  The pair's column (planes k-1, k, k+1) stays in registers and the
// in-plane neighbours come from LDS (three planes, 1-cell halo ring).  The
// residuals of the children are summed in the pair (f_x = 2), across the two
// rows of a wave (f_y = 2, lanes l and l + 32) and over two planes (f_z = 2)
// before the owner of the coarse cell writes it.  zlen is even.
template <typename S, int TX, int TY>
__global__ void __launch_bounds__(TX * TY / 2)
k_restrict_z(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
             const S* __restrict__ xin, const S* __restrict__ bin, S* __restrict__ bc, S* __restrict__ xc,
             double* __restrict__ partials) {
  using C = typename Ty<S>::C;
  constexpr bool ROW = (TY == 1);
  constexpr int NT = TX * TY / 2;
  constexpr int YO = ROW ? 0 : 1;
  constexpr int HX = TX + 2, HY = ROW ? 1 : TY + 2;
  constexpr int NHALO = HX * HY - TX * TY;
  constexpr int NHR = (NHALO + NT - 1) / NT;
  static_assert(ROW || TX == 64, "row pairs of a wave: TX/2 == 32 lanes per row");
  __shared__ C X[3][HY][HX];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];

  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const C alpha = (C)G.alpha, wx = (C)G.wx, wy = (C)G.wy, wz = (C)G.wz;
  const int64_t pl = (int64_t)px * ny;
  const int64_t cpl = (int64_t)G.cpx * G.cny;
  const S* xg = xin + G.off;
  const S* bg = bin + G.off;
  const bool vec = ((px | G.off) & 1) == 0, cvec = ((G.cpx | G.coff) & 1) == 0;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;
  const int tyl = tid / (TX / 2), pxl = tid - tyl * (TX / 2);
  const int gx = x0 + 2 * pxl, gy = y0 + tyl;
  const bool rowok = gy < ny;
  const bool vA = rowok && gx < nx, vB = rowok && gx + 1 < nx;
  const int lx = 1 + 2 * pxl, ly = YO + tyl;
  const int64_t own = (int64_t)gy * px + gx;
  const bool up = gy > 0, dn = gy + 1 < ny, o0 = gx > 0, o1 = gx + 2 < nx;

  int hoff[NHR];
  int64_t hg[NHR];
  bool hv[NHR];
#pragma unroll
  for (int k = 0; k < NHR; ++k) {
    const int h = tid + NT * k;
    int hy = 0, hx = 0;
    if (ROW) {
      hx = (h == 0) ? 0 : HX - 1;
    } else if (h < HX) {
      hy = 0; hx = h;
    } else if (h < 2 * HX) {
      hy = HY - 1; hx = h - HX;
    } else {
      const int m = h - 2 * HX;
      hy = 1 + (m >> 1);
      hx = (m & 1) ? HX - 1 : 0;
    }
    const int cx = x0 - 1 + hx, cy = y0 - YO + hy;
    hv[k] = h < NHALO && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    hoff[k] = hy * HX + hx;
    hg[k] = hv[k] ? (int64_t)cy * px + cx : 0;
  }
  // x of plane q: raw loads from clamped addresses (no branch around them),
  // converted and masked in stash(); b pairs likewise, one plane ahead
  Raw2<S> rx;
  Raw<S> rh[NHR];
  C na = 0, nb = 0;
  auto plane_off = [&](int q) { return (int64_t)min(max(q, 0), nz - 1) * pl; };
  auto fetch = [&](int q) {
    const S* P = xg + plane_off(q);
    ld_raw2(P + (vA ? own : 0), vec, true, rx);
#pragma unroll
    for (int k = 0; k < NHR; ++k) ld_raw(P + hg[k], rh[k]);
  };
  auto stash = [&](int q) {  // converts the last fetch into na, nb and LDS
    const bool okq = q >= 0 && q < nz;
    na = (okq && vA) ? raw_ca(rx) : (C)0;
    nb = (okq && vB) ? raw_cb(rx) : (C)0;
    C* P = &X[((q % 3) + 3) % 3][0][0];
    P[ly * HX + lx] = na;
    P[ly * HX + lx + 1] = nb;
#pragma unroll
    for (int k = 0; k < NHR; ++k)
      if (tid + NT * k < NHALO) P[hoff[k]] = (okq && hv[k]) ? raw_c(rh[k]) : (C)0;
  };
  Raw2<S> rbn;
  auto fetch_b = [&](int q) { ld_raw2(bg + plane_off(q) + (vA ? own : 0), vec, true, rbn); };
  auto conv_b = [&](int q, C& a, C& b) {
    const bool okq = q >= 0 && q < nz;
    a = (okq && vA) ? raw_ca(rbn) : (C)0;
    b = (okq && vB) ? raw_cb(rbn) : (C)0;
  };

  C ma, mb, ca, cb, pa, pb, ba, bb;
  fetch(q0 - 1); stash(q0 - 1); ma = na; mb = nb;  // (the ring slot of q0 - 1 is rewritten before it is read)
  fetch(q0); stash(q0); ca = na; cb = nb;
  fetch_b(q0); conv_b(q0, ba, bb);
  fetch(q0 + 1);
  fetch_b(q0 + 1);
  double nrm = 0.0;
  C s0 = 0, s1 = 0;
  for (int k = q0; k < q1; ++k) {
    stash(k + 1);
    pa = na; pb = nb;
    fetch(k + 2);
    __syncthreads();
    const C* P = &X[k % 3][0][0];
    const bool zm = k > 0, zp = k < nz - 1;
    C ra = 0, rb = 0;
    if (vA) {
      const C xa = ca;
      C r = ba - alpha * xa;
      r += vB ? wx * (cb - xa) : (C)0;
      r += o0 ? wx * (P[ly * HX + lx - 1] - xa) : (C)0;
      r += up ? wy * (P[(ly - 1 + (ROW ? 1 : 0)) * HX + lx] - xa) : (C)0;
      r += dn ? wy * (P[(ly + 1 - (ROW ? 1 : 0)) * HX + lx] - xa) : (C)0;
      r += zm ? wz * (ma - xa) : (C)0;
      r += zp ? wz * (pa - xa) : (C)0;
      ra = r;
    }
    if (vB) {
      const C xb = cb;
      C r = bb - alpha * xb;
      r += wx * (ca - xb);
      r += o1 ? wx * (P[ly * HX + lx + 2] - xb) : (C)0;
      r += up ? wy * (P[(ly - 1 + (ROW ? 1 : 0)) * HX + lx + 1] - xb) : (C)0;
      r += dn ? wy * (P[(ly + 1 - (ROW ? 1 : 0)) * HX + lx + 1] - xb) : (C)0;
      r += zm ? wz * (mb - xb) : (C)0;
      r += zp ? wz * (pb - xb) : (C)0;
      rb = r;
    }
    nrm += (double)ra * (double)ra + (double)rb * (double)rb;
    if (G.fx == 2) s0 += ra + rb; else { s0 += ra; s1 += rb; }
    if (G.fz == 1 || (k & 1) || k == nz - 1) {
      // rows 2J and 2J + 1 sit in lanes l and l + 32 of one wave
      if (!ROW && G.fy == 2) {
        s0 += __shfl_down(s0, 32, 64);
        s1 += __shfl_down(s1, 32, 64);
      }
      const bool owner = ROW || G.fy == 1 || (tyl & 1) == 0;
      if (owner && vA) {
        const int I = gx / G.fx, J = gy / G.fy, K = k / G.fz;
        const int64_t cv = G.coff + K * cpl + (int64_t)J * G.cpx + I;
        if (G.fx == 2) {
          Ty<S>::st(bc + cv, s0);
          if (xc) Ty<S>::st(xc + cv, (C)0);
        } else {
          st2(bc + cv, cvec, vB, s0, s1);
          if (xc) st2(xc + cv, cvec, vB, (C)0, (C)0);
        }
      }
      s0 = s1 = (C)0;
    }
    ma = ca; mb = cb; ca = pa; cb = pb;
    conv_b(k + 1, ba, bb);
    fetch_b(k + 2);
  }
  if (partials) {
    const double sm = block_sum(nrm, red);
    if (threadIdx.x == 0) partials[t.bid] = sm;
  }
}

// ------------------------------------------------------ prolongation (+=)
template <typename S>
__global__ void __launch_bounds__(256)
k_prolong_add(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
              int etx, const S* __restrict__ ec, S* __restrict__ xio, int mode) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  S* x = xio + G.off;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = k * pl + (int64_t)j * G.px + i;
    Ty<S>::st(x + v, Ty<S>::ld(x + v) + prolong_value<S>(ec, G, i, j, k, mode));
  }
}

// Pair form for the library's arrays (tiles of the relaxation, one x-pair per
// thread), marching along z.  The x and y interpolation of a thread is the
// same on every plane: each coarse plane reduces to one value per fine cell
// of the pair, kept in a window of three coarse planes (K - 1, K, K + 1)
// that advances with the fine plane's parent K, so a coarse plane is loaded
// once per block column.  Fine values are read raw two planes ahead and
// coarse planes one advance ahead, from clamped addresses without branches.
// Every weight and index is that of prolong_value (cell-centred trilinear,
// weight 1 on kept axes and at mirror edges; mode 1 piecewise constant).
template <typename S, int TX, int TY, bool KEEPX>
__global__ void __launch_bounds__(TX * TY / 2)
k_prolong_pair(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
               const S* __restrict__ ec, S* __restrict__ xio, int mode) {
  // KEEPX: the level keeps x (f_x == 1), so a coarse row holds the pair itself
  using C = typename Ty<S>::C;
  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false);
  const GridDesc& G = grids[t.g];
  const int tid = threadIdx.x;
  const int tyl = tid / (TX / 2), pxl = tid - tyl * (TX / 2);
  const int gx = t.x0 + 2 * pxl, gy = t.y0 + tyl;
  const bool ok = gy < G.ny && gx < G.nx;
  const bool vB = gx + 1 < G.nx;
  const int64_t pl = (int64_t)G.px * G.ny;
  S* x = xio + G.off + (ok ? (int64_t)gy * G.px + gx : 0);
  const int nz = G.nz, cnz = G.cnz, fz = G.fz;
  const S* e = ec + G.coff;
  const int64_t cpl = (int64_t)G.cpx * G.cny;

  // x: vA = a0 v(i0) + a1 v(i1), vB = b0 v(i0) + b2 v(i2) on a coarse row
  int i0 = 0, i1 = 0, i2 = 0;
  C a0 = 1, a1 = 0, b0 = 0, b2 = 0;
  // y: rows ja (weight ya) and jb (weight yb)
  int ja = 0, jb = 0;
  C ya = 1, yb = 0;
  if (ok) {
    if (G.fx == 1) {  // the pair (gx, gx + 1) of the coarse row (KEEPX loads it from i0 at once)
      i0 = i1 = gx;
      i2 = vB ? gx + 1 : gx;
      b2 = 1;
    } else if (mode == 1) {
      i0 = i1 = i2 = gx / 2;
      b0 = 1;
    } else {
      int pa, qa, pb, qb;
      const bool tA = lin_idx(gx, 2, G.cnx, pa, qa);
      const bool tB = lin_idx(gx + 1, 2, G.cnx, pb, qb);
      i0 = pa;  // the pair's common parent
      i1 = tA ? qa : pa;
      i2 = tB ? qb : pa;
      a0 = tA ? (C)0.75 : (C)1; a1 = tA ? (C)0.25 : (C)0;
      b0 = tB ? (C)0.75 : (C)1; b2 = tB ? (C)0.25 : (C)0;
    }
    if (G.fy == 1) {
      ja = jb = gy;
    } else if (mode == 1) {
      ja = jb = gy / 2;
    } else {
      const bool ty = lin_idx(gy, 2, G.cny, ja, jb);
      if (ty) { ya = (C)0.75; yb = (C)0.25; } else { jb = ja; }
    }
  }
  const S* ra = e + (int64_t)ja * G.cpx;
  const S* rb = e + (int64_t)jb * G.cpx;
  struct CRaw { Raw<S> v[6]; Raw2<S> p[2]; };
  auto cload = [&](int K, CRaw& r) {  // coarse plane K (clamped)
    const int64_t o = (int64_t)min(max(K, 0), cnz - 1) * cpl;
    if (KEEPX) {
      ld_raw2(ra + o + i0, true, true, r.p[0]);
      ld_raw2(rb + o + i0, true, true, r.p[1]);
    } else {
      ld_raw(ra + o + i0, r.v[0]); ld_raw(ra + o + i1, r.v[1]); ld_raw(ra + o + i2, r.v[2]);
      ld_raw(rb + o + i0, r.v[3]); ld_raw(rb + o + i1, r.v[4]); ld_raw(rb + o + i2, r.v[5]);
    }
  };
  // explicit fused multiply-adds in one order: the window set-up and its
  // advance compute a coarse plane's value alike, so a fine plane gets the
  // same value whichever z-chunk it falls in
  auto cval = [&](const CRaw& r, C& va, C& vb) {
    if (KEEPX) {
      va = fmac(yb, raw_ca(r.p[1]), ya * raw_ca(r.p[0]));
      vb = fmac(yb, raw_cb(r.p[1]), ya * raw_cb(r.p[0]));
    } else {
      const C u0 = raw_c(r.v[0]), u1 = raw_c(r.v[1]), u2 = raw_c(r.v[2]);
      const C w0 = raw_c(r.v[3]), w1 = raw_c(r.v[4]), w2 = raw_c(r.v[5]);
      va = fmac(yb, fmac(a1, w1, a0 * w0), ya * fmac(a1, u1, a0 * u0));
      vb = fmac(yb, fmac(b2, w2, b0 * w0), ya * fmac(b2, u2, b0 * u0));
    }
  };
  auto fplane = [&](int k) { return x + (int64_t)min(max(k, 0), nz - 1) * pl; };

  const int k0 = t.z0, k1 = t.z1;
  int Kc = k0 / fz;
  C vma, vmb, v0a, v0b, vpa, vpb;
  CRaw cr;
  cload(Kc - 1, cr); cval(cr, vma, vmb);
  cload(Kc, cr);     cval(cr, v0a, v0b);
  cload(Kc + 1, cr); cval(cr, vpa, vpb);
  cload(Kc + 2, cr);
  Raw2<S> f0, f1, fn;
  ld_raw2(fplane(k0), true, true, f0);
  ld_raw2(fplane(k0 + 1), true, true, f1);
  for (int k = k0; k < k1; ++k) {
    ld_raw2(fplane(k + 2), true, true, fn);
    const int K = k / fz;
    if (K > Kc) {  // advance the window (uniform over the block)
      vma = v0a; vmb = v0b; v0a = vpa; v0b = vpb;
      cval(cr, vpa, vpb);
      Kc = K;
    }
    cload(Kc + 2, cr);
    // z weights: parent K and its neighbour on the fine cell's side
    C za, zb;
    if (mode == 0 && fz == 2) {
      const int Kn = (k & 1) ? K + 1 : K - 1;
      const bool two = Kn >= 0 && Kn < cnz;
      const C w1 = two ? (C)0.75 : (C)1, w2 = two ? (C)0.25 : (C)0;
      za = fmac(w2, (k & 1) ? vpa : vma, w1 * v0a);
      zb = fmac(w2, (k & 1) ? vpb : vmb, w1 * v0b);
    } else {
      za = v0a;
      zb = v0b;
    }
    if (ok) st2(x + (int64_t)k * pl, true, vB, raw_ca(f0) + za, raw_cb(f0) + zb);
    f0 = f1;
    f1 = fn;
  }
}

// ------------------------------------------- finest level of AD / SP (Eq. 1, 2)
//
// Canonical system of both phases: A = alpha + w_x L_x + w_y L_y + w_z L_z,
// b = alpha I1 + (w_x L_x + w_y L_y) I0 (AD: alpha = 0; SP: w_z = 0).  In
// the grid description the caller's y axis is the grid's y axis for a stack
// and its z axis for a slice (ny = 1); the in-slice weights are then w_x and
// w_z.  GridDesc::zin flags the slice form.
// The plain solver iterates on the correction E = x - I0, whose right-hand
// side is b - A I0 = alpha (I1 - I0) - (cross-slice part of A) I0.

template <typename Tin>
__device__ __forceinline__ double in_at(const Tin* p, int64_t v) { return ld64(p + v); }

// ------------------------------------- correction-form stencil passes
//
// Both passes on the finest grid use one z-marching structure (pairs of x
// per thread, the three planes of one field in an LDS ring for the in-plane
// neighbours, z neighbours in registers; FP64 arithmetic):
//
// KIND 0, right-hand side of the correction E = x - I0.  With F = I0:
//   b_corr = alpha (I1 - I0) - [stack] w_z L_z I0
//   ||b||^2 of the canonical system b = alpha I1 + (w_x L_x + w_y L_y) I0
//   (+ w_z L_z I0 for a slice, whose "z" is its own second axis); the stack
//   form's cross-slice target is zero (Eq. (1)).  Writes b_corr and a zero
//   correction.
// KIND 1, canonical residual b - A x in FP64.  With F = x - I0 (E in MODE 0,
// x64 - I0 in MODE 1, x64 + s e - I0 in MODE 2, where the refinement's
// update x64 + s e is also written to x64_out, s = e_scale[grid]) the I0
// terms of b and A x cancel except across slices:
//   r = alpha (I1 - I0 - F) - (w_x L_x + w_y L_y + w_z L_z) F - [stack] w_z L_z I0
//   ||r||^2 per block; r * inv_scale stored when rout is set.
// L_a v is the Neumann second difference sum over existing neighbours of
// (v_c - v_n).  Row tiles (TY == 1) serve grids with ny == 1.
template <typename Tin, typename S, int TX, int TY, int KIND, int MODE>
__global__ void __launch_bounds__(TX * TY / 2)
k_corr_stencil(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
               const Tin* __restrict__ I0, const Tin* __restrict__ I1, const S* __restrict__ E,
               const double* __restrict__ x64, S* __restrict__ out0, S* __restrict__ out1,
               const double* __restrict__ inv_scale, double* __restrict__ partials,
               double* __restrict__ x64_out, const double* __restrict__ e_scale) {
  constexpr bool ROW = (TY == 1);
  constexpr int NT = TX * TY / 2;
  constexpr int YO = ROW ? 0 : 1;
  constexpr int HX = TX + 2, HY = ROW ? 1 : TY + 2;
  constexpr int NHALO = HX * HY - TX * TY;
  constexpr int NHR = (NHALO + NT - 1) / NT;
  static_assert(MODE < 2 || KIND == 1, "the refinement update belongs to the residual pass");
  __shared__ double X[3][HY][HX];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];

  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const bool slice = G.zin != 0;
  const double alpha = G.alpha, wx = G.wx, wy = ROW ? 0.0 : G.wy, wz = G.wz;
  const bool cross = !slice && wz != 0.0;  // the stack's cross-slice term of I0
  const int64_t pl = (int64_t)px * ny;
  const Tin* I0g = I0 + G.ioff;
  const Tin* I1g = (I1 && alpha != 0.0) ? I1 + G.ioff : nullptr;
  const S* Eg = E + G.off;
  const double* xg = x64 + G.off;
  const bool ivec = ((G.ioff | G.ipy | G.ipz) & 1) == 0, vec = ((px | G.off) & 1) == 0;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;
  const int tyl = tid / (TX / 2), pxl = tid - tyl * (TX / 2);
  const int gx = x0 + 2 * pxl, gy = y0 + tyl;
  const bool rowok = gy < ny;
  const bool vA = rowok && gx < nx, vB = rowok && gx + 1 < nx;
  const int lx = 1 + 2 * pxl, ly = YO + tyl;
  const int64_t own = (int64_t)gy * px + gx, ownu = (int64_t)gy * G.ipy + gx;
  const bool up = !ROW && gy > 0, dn = !ROW && gy + 1 < ny, o0 = gx > 0, o1 = gx + 2 < nx;

  int hoff[NHR];
  int64_t hg[NHR], hu[NHR];
  bool hv[NHR];
#pragma unroll
  for (int k = 0; k < NHR; ++k) {
    const int h = tid + NT * k;
    int hy = 0, hx = 0;
    if (ROW) {
      hx = (h == 0) ? 0 : HX - 1;
    } else if (h < HX) {
      hy = 0; hx = h;
    } else if (h < 2 * HX) {
      hy = HY - 1; hx = h - HX;
    } else {
      const int m = h - 2 * HX;
      hy = 1 + (m >> 1);
      hx = (m & 1) ? HX - 1 : 0;
    }
    const int cx = x0 - 1 + hx, cy = y0 - YO + hy;
    hv[k] = h < NHALO && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    hoff[k] = hy * HX + hx;
    hg[k] = hv[k] ? (int64_t)cy * px + cx : 0;
    hu[k] = hv[k] ? (int64_t)cy * G.ipy + cx : 0;
  }
  // Raw loads of plane q: F's own pair and halo values and (KIND 1) I0's
  // pair; converted to FP64 only in stash(), after other work has run.
  using FS = std::conditional_t<KIND == 0, Tin, std::conditional_t<MODE == 0, S, double>>;
  Raw2<FS> rf;
  Raw2<Tin> ri;
  Raw2<S> re;  // MODE 2: the correction e
  Raw<FS> rh[NHR];
  Raw<Tin> rhi[NHR];
  Raw<S> rhe[NHR];
  const double es = (MODE == 2) ? e_scale[t.g] : 0.0;
  // loads from clamped addresses without branches around them (masked in stash)
  auto fetch = [&](int q) {
    const int qc = min(max(q, 0), nz - 1);
    const Tin* I0q = I0g + qc * G.ipz;
    const int64_t po = qc * pl;
    const int64_t oo = vA ? own : 0, ou = vA ? ownu : 0;
    if (KIND == 0) {
      ld_raw2(reinterpret_cast<const FS*>(I0q) + ou, ivec, vB, rf);
    } else {
      ld_raw2(I0q + ou, ivec, vB, ri);
      if (MODE == 0) {
        ld_raw2(reinterpret_cast<const FS*>(Eg) + po + oo, true, true, rf);
      } else {
        ld_raw2(reinterpret_cast<const FS*>(xg) + po + oo, true, true, rf);
        if (MODE == 2) ld_raw2(Eg + po + oo, true, true, re);
      }
    }
#pragma unroll
    for (int k = 0; k < NHR; ++k) {
      if (KIND == 0) ld_raw(reinterpret_cast<const FS*>(I0q) + hu[k], rh[k]);
      else if (MODE == 0) ld_raw(reinterpret_cast<const FS*>(Eg) + po + hg[k], rh[k]);
      else {
        ld_raw(reinterpret_cast<const FS*>(xg) + po + hg[k], rh[k]);
        ld_raw(I0q + hu[k], rhi[k]);
        if (MODE == 2) ld_raw(Eg + po + hg[k], rhe[k]);
      }
    }
  };
  // convert the last fetch: F pair (fa, fb), I0 pair (ia, ib); store F's plane
  double fa = 0, fb = 0, ia = 0, ib = 0;
  auto stash = [&](int q) {
    const bool okq = q >= 0 && q < nz, mA = okq && vA, mB = okq && vB;
    if (KIND == 1) {
      ia = mA ? raw_a(ri) : 0.0;
      ib = mB ? raw_b(ri) : 0.0;
    }
    fa = mA ? raw_a(rf) : 0.0;
    fb = mB ? raw_b(rf) : 0.0;
    if (KIND == 1 && MODE == 2) {  // refinement update x64 + s e, written by the cell's owner
      fa += mA ? es * raw_a(re) : 0.0;
      fb += mB ? es * raw_b(re) : 0.0;
      if (vA && q >= q0 && q < q1) st2(x64_out + G.off + q * pl + own, vec, vB, fa, fb);
    }
    if (KIND == 1 && MODE >= 1) {
      fa -= ia;
      fb = vB ? fb - ib : 0.0;
    }
    double* P = &X[((q % 3) + 3) % 3][0][0];
    P[ly * HX + lx] = fa;
    P[ly * HX + lx + 1] = fb;
#pragma unroll
    for (int k = 0; k < NHR; ++k)
      if (tid + NT * k < NHALO) {
        double v = raw_d(rh[k]);
        if (KIND == 1 && MODE == 2) v += es * raw_d(rhe[k]);
        if (KIND == 1 && MODE >= 1) v -= raw_d(rhi[k]);
        P[hoff[k]] = (okq && hv[k]) ? v : 0.0;
      }
  };
  // I1 pair at plane q (raw), prefetched one plane ahead
  Raw2<Tin> r1n;
  auto fetch1 = [&](int q) {  // raw, clamped; used only for k in [q0, q1) with vA / vB
    if (I1g) ld_raw2(I1g + min(max(q, 0), nz - 1) * G.ipz + (vA ? ownu : 0), ivec, vB, r1n);
  };

  // registers: F and I0 at k - 1 (m), k (c), k + 1 (p)
  double fma_ = 0, fmb = 0, fca, fcb, fpa, fpb, ima = 0, imb = 0, ica = 0, icb = 0, ipa = 0, ipb = 0;
  fetch(q0 - 1);
  stash(q0 - 1);  // plane q0 - 1 goes to the ring slot of q0 + 2, rewritten before it is read
  fma_ = fa; fmb = fb; ima = ia; imb = ib;
  fetch(q0);
  stash(q0);
  fca = fa; fcb = fb; ica = ia; icb = ib;
  fetch(q0 + 1);
  fetch1(q0);
  double nrm = 0.0;
  for (int k = q0; k < q1; ++k) {
    stash(k + 1);
    fpa = fa; fpb = fb; ipa = ia; ipb = ib;
    const Raw2<Tin> r1 = r1n;
    fetch(k + 2);
    fetch1(k + 1);
    __syncthreads();
    const double v1a = I1g ? raw_a(r1) : 0.0, v1b = I1g ? raw_b(r1) : 0.0;
    const double* P = &X[k % 3][0][0];
    const bool zm = k > 0, zp = k < nz - 1;
    double ra = 0.0, rb = 0.0;
    // in-plane and z second differences of F; I0's z term for the stack
    auto lap = [&](double c, double l, bool hl, double rr, bool hr, double u_, double d_, double zm_, double zp_) {
      double s2 = 0.0;
      if (hl) s2 += wx * (c - l);
      if (hr) s2 += wx * (c - rr);
      if (up) s2 += wy * (c - u_);
      if (dn) s2 += wy * (c - d_);
      if (zm) s2 += wz * (c - zm_);
      if (zp) s2 += wz * (c - zp_);
      return s2;
    };
    if (vA) {
      const double c = fca;
      const double lf = lap(c, o0 ? P[ly * HX + lx - 1] : 0.0, o0, fcb, vB, up ? P[(ly - 1) * HX + lx] : 0.0,
                            dn ? P[(ly + 1) * HX + lx] : 0.0, fma_, fpa);
      double lzI = 0.0;  // w_z L_z I0 (stack only)
      if (cross) {
        const double i0 = KIND == 0 ? fca : ica, im = KIND == 0 ? fma_ : ima, ip = KIND == 0 ? fpa : ipa;
        if (zm) lzI += wz * (i0 - im);
        if (zp) lzI += wz * (i0 - ip);
      }
      if (KIND == 0) {
        const double lin = lf - (cross ? lzI : 0.0);  // canonical part of L I0
        const double bcan = alpha * v1a + lin;
        nrm += bcan * bcan;
        ra = alpha * (v1a - c) - lzI;
      } else {
        ra = alpha * (v1a - ica - c) - lf - lzI;
        nrm += ra * ra;
      }
    }
    if (vB) {
      const double c = fcb;
      const double lf = lap(c, fca, true, o1 ? P[ly * HX + lx + 2] : 0.0, o1, up ? P[(ly - 1) * HX + lx + 1] : 0.0,
                            dn ? P[(ly + 1) * HX + lx + 1] : 0.0, fmb, fpb);
      double lzI = 0.0;
      if (cross) {
        const double i0 = KIND == 0 ? fcb : icb, im = KIND == 0 ? fmb : imb, ip = KIND == 0 ? fpb : ipb;
        if (zm) lzI += wz * (i0 - im);
        if (zp) lzI += wz * (i0 - ip);
      }
      if (KIND == 0) {
        const double lin = lf - (cross ? lzI : 0.0);
        const double bcan = alpha * v1b + lin;
        nrm += bcan * bcan;
        rb = alpha * (v1b - c) - lzI;
      } else {
        rb = alpha * (v1b - icb - c) - lf - lzI;
        nrm += rb * rb;
      }
    }
    if (vA) {
      const int64_t v = G.off + k * pl + own;
      if (KIND == 0) {
        if (out0) st2(out0 + v, vec, vB, (typename Ty<S>::C)ra, (typename Ty<S>::C)rb);
        if (out1) st2(out1 + v, vec, vB, (typename Ty<S>::C)0, (typename Ty<S>::C)0);
      } else if (out0) {
        const double sc = inv_scale[t.g];
        st2(out0 + v, vec, vB, (typename Ty<S>::C)(ra * sc), (typename Ty<S>::C)(rb * sc));
      }
    }
    fma_ = fca; fmb = fcb; fca = fpa; fcb = fpb;
    ima = ica; imb = icb; ica = ipa; icb = ipb;
  }
  if (partials) {
    const double sm = block_sum(nrm, red);
    if (threadIdx.x == 0) partials[t.bid] = sm;
  }
}

template <typename Tin, typename S, int MODE>
__global__ void __launch_bounds__(256)
k_sum_shift(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
            const Tin* __restrict__ I0, const S* __restrict__ E, const double* __restrict__ x64,
            double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  double s = 0.0;
  if (i < G.nx && j < G.ny) {
    const int64_t pl = (int64_t)G.px * G.ny;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = G.off + k * pl + (int64_t)j * G.px + i;
      if (MODE == 0) {
        s += ld64(E + v);
      } else {
        const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
        s += x64[v] - in_at(I0, u);
      }
    }
  }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) partials[t.bid] = tot;
}

template <typename Tin, typename S, typename Tout, int MODE>
__global__ void __launch_bounds__(256)
k_finalize(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
           const Tin* __restrict__ I0, const S* __restrict__ E, const double* __restrict__ x64,
           const double* __restrict__ shift, Tout* __restrict__ out) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  const double sh = shift ? shift[t.g] : 0.0;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
    const int64_t v = G.off + k * pl + (int64_t)j * G.px + i;
    const double x = (MODE == 0) ? in_at(I0, u) + ld64(E + v) : x64[v];
    st64(out + u, x - sh);
  }
}

template <typename Tin>
__global__ void __launch_bounds__(256)
k_refine_init(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
              const Tin* __restrict__ I0, double* __restrict__ x64) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t u = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
    x64[G.off + k * pl + (int64_t)j * G.px + i] = in_at(I0, u);
  }
}


// -------------------------------------------------- general system (Sec. 4)
// (caller's arrays, pitch px = nx)
template <typename S>
__global__ void __launch_bounds__(256)
k_rhs_general(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
              const S* __restrict__ V, const S* __restrict__ Gx, const S* __restrict__ Gy,
              const S* __restrict__ Gz, S* __restrict__ bout) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  if (i >= nx || j >= ny) return;
  const int64_t pl = (int64_t)G.ipz;
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = G.ioff + k * pl + (int64_t)j * G.ipy + i;
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
      if (j > 0) d += ld64(Gy + v - G.ipy);
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

// LIB: the arrays are a level of the library's hierarchy (offset off, row
// pitch px) instead of the caller's layout.  Only planes klo <= k < khi are
// visited (a window whose outer planes are halo).
template <typename S, bool LIB>
__global__ void __launch_bounds__(256)
k_general_residual(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids,
                   int zlen, int etx, const S* __restrict__ xin, const S* __restrict__ bin, S* __restrict__ rout,
                   double* __restrict__ partials, int klo, int khi) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  double rr = 0.0, bb = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = LIB ? (int64_t)G.px * ny : G.ipz, py = LIB ? (int64_t)G.px : G.ipy;
    const int64_t base = LIB ? G.off : G.ioff;
    const int ka = t.z0 > klo ? t.z0 : klo, kb = t.z1 < khi ? t.z1 : khi;
    for (int k = ka; k < kb; ++k) {
      const int64_t v = base + k * pl + (int64_t)j * py + i;
      const double xc = ld64(xin + v), bv = ld64(bin + v);
      double r = bv - G.alpha * xc;
      if (i > 0) r += G.wx * (ld64(xin + v - 1) - xc);
      if (i < nx - 1) r += G.wx * (ld64(xin + v + 1) - xc);
      if (j > 0) r += G.wy * (ld64(xin + v - py) - xc);
      if (j < ny - 1) r += G.wy * (ld64(xin + v + py) - xc);
      if (k > 0) r += G.wz * (ld64(xin + v - pl) - xc);
      if (k < nz - 1) r += G.wz * (ld64(xin + v + pl) - xc);
      if (rout) st64(rout + v, r);
      rr += r * r;
      bb += bv * bv;
    }
  }
  const double s1 = block_sum(rr, red);
  const double s2 = block_sum(bb, red);
  if (threadIdx.x == 0) {
    partials[2 * t.bid] = s1;
    partials[2 * t.bid + 1] = s2;
  }
}

// ------------------------------------------- gradient-modulation filter (Sec. 6)
//
// Right-hand side of the filter in correction form.  The target gradient on
// the face v -> v + e_a is V = f(v) g_a(v): g(v) the forward-difference
// gradient of I0 at v (a component is 0 where its face leaves the grid) and
// f(v) = lambda (1 - exp(-|g(v)|^2 / (2 sigma^2))).  The canonical system is
// (alpha + sum_a w_a D_a^T D_a) I = alpha I0 + sum_a w_a D_a^T V_a; for
// I = I0 + E it becomes A E = sum_a w_a D_a^T ((f - 1) g_a), written to b in
// the library's layout.  (D_a^T h)(v) = h(v - e_a) - h(v), so a voxel needs
// f and g of itself and of its three lower neighbours.  Per block: FP64
// sums of the canonical right-hand side squared and of b squared.
template <typename Tin, typename S>
__global__ void __launch_bounds__(256)
k_npr_rhs(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
          const Tin* __restrict__ I0, double lam, double inv2s2, S* __restrict__ bout,
          double* __restrict__ partials) {
  // arithmetic in the storage's compute type (FP32 for FP32 storage, FP64
  // for FP64); the z-march keeps the factor and gradient of the voxel below
  using C = typename Ty<S>::C;
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  double sb = 0.0, se = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = (int64_t)G.px * ny;
    const C w[3] = {(C)G.wx, (C)G.wy, (C)G.wz};
    const C lamc = (C)lam, i2 = (C)inv2s2, alpha = (C)G.alpha;
    auto I = [&](int di, int dj, int k) -> C {
      return (C)in_at(I0, G.ioff + (int64_t)k * G.ipz + (int64_t)(j + dj) * G.ipy + (i + di));
    };
    // forward gradient and factor of voxel (i + di, j + dj, k), value c there
    auto fwd = [&](int di, int dj, int k, C c, C g[3]) -> C {
      g[0] = (i + di + 1 < nx) ? I(di + 1, dj, k) - c : (C)0;
      g[1] = (j + dj + 1 < ny) ? I(di, dj + 1, k) - c : (C)0;
      g[2] = (k + 1 < nz) ? I(di, dj, k + 1) - c : (C)0;
      return lamc * ((C)1 - exp(-(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * i2));
    };
    C fz = 0, gz = 0;  // factor and z-gradient of the voxel below (valid for k > t.z0)
    if (t.z0 > 0) {
      C g[3];
      fz = fwd(0, 0, t.z0 - 1, I(0, 0, t.z0 - 1), g);
      gz = g[2];
    }
    for (int k = t.z0; k < t.z1; ++k) {
      const C c = I(0, 0, k);
      C gv[3];
      const C fv = fwd(0, 0, k, c, gv);
      C bc = alpha * c, be = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (w[a] == (C)0) continue;
        bc -= w[a] * fv * gv[a];  // the face this voxel owns
        be -= w[a] * (fv - (C)1) * gv[a];
      }
      // faces owned by the lower neighbours along x, y (recomputed) and z (kept)
      if (w[0] != (C)0 && i > 0) {
        C g[3];
        const C f = fwd(-1, 0, k, I(-1, 0, k), g);
        bc += w[0] * f * g[0];
        be += w[0] * (f - (C)1) * g[0];
      }
      if (w[1] != (C)0 && j > 0) {
        C g[3];
        const C f = fwd(0, -1, k, I(0, -1, k), g);
        bc += w[1] * f * g[1];
        be += w[1] * (f - (C)1) * g[1];
      }
      if (w[2] != (C)0 && k > 0) {
        bc += w[2] * fz * gz;
        be += w[2] * (fz - (C)1) * gz;
      }
      fz = fv;
      gz = gv[2];
      st64(bout + G.off + k * pl + (int64_t)j * G.px + i, (double)be);
      sb += (double)bc * (double)bc;
      se += (double)be * (double)be;
    }
  }
  const double s1 = block_sum(sb, red);
  const double s2 = block_sum(se, red);
  if (threadIdx.x == 0) {
    partials[2 * t.bid] = s1;
    partials[2 * t.bid + 1] = s2;
  }
}

// ------------------------------------------------ Hybrid discretisation
//
// Sec. 4.2 "Hybrid": the finest level keeps the 7-point operator; levels are
// linked by the B-spline nesting (1/2, 1, 1/2) per halved axis (coarse
// sample c on fine sample 2c; an odd last fine sample with no coarse sample
// to its right takes the last one alone) and every coarser operator is the
// Galerkin product, held as per-axis tridiagonal tables: a level's operator
// is alpha Mx My Mz + w_x Kx My Mz + w_y Mx Ky Mz + w_z Mx My Kz.  A table
// block of axis a (n_a samples) is six rows of n_a doubles: M below, on and
// above the diagonal, then K likewise.  These levels are one grid each and
// are addressed with the level's own offset and pitch.

struct HybAxes {
  const double* t[3];  // table blocks of x, y, z
  double alpha, w[3];
};

// weight P[f][c] of coarse sample c in fine sample f along one axis (n fine,
// nc coarse samples, halved or kept); 0 when c is not a parent of f
__device__ __forceinline__ double bsp_weight(int f, int c, int n, int nc, bool halved) {
  if (!halved) return f == c ? 1.0 : 0.0;
  if (f == 2 * c) return 1.0;
  if (f == 2 * c - 1) return 0.5;
  if (f == 2 * c + 1 && f < n) return (c + 1 < nc) ? 0.5 : 1.0;
  return 0.0;
}

// sum over the 27 neighbours of (row of A at (i, j, k)) . x, and the diagonal.
// Branch-free: a neighbour outside the grid is read at a clamped index and
// weighted by its table entry, which is 0 (the first sample has no lower and
// the last no upper coupling on every level), so all 27 loads issue at once.
template <typename S>
__device__ __forceinline__ void hyb_row(const HybAxes& A, const GridDesc& G, const S* __restrict__ x, int i, int j,
                                        int k, double& ax, double& diag) {
  const int n[3] = {G.nx, G.ny, G.nz}, c[3] = {i, j, k};
  double m[3][3], kk[3][3];  // [axis][offset + 1]
  int q[3][3];               // clamped neighbour index [axis][offset + 1]
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* T = A.t[a];
    const int na = n[a], p = c[a];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      m[a][d] = T[d * na + p];
      kk[a][d] = T[(3 + d) * na + p];
      q[a][d] = min(max(p + d - 1, 0), na - 1);
    }
  }
  const int64_t pl = (int64_t)G.px * G.ny;
  const S* base = x + G.off;
  double s = 0.0;
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const double myz = m[1][dy] * m[2][dz], kyz = kk[1][dy] * m[2][dz], mkz = m[1][dy] * kk[2][dz];
      const S* row = base + q[2][dz] * pl + (int64_t)q[1][dy] * G.px;
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const double coef = (A.alpha * m[0][dx] + A.w[0] * kk[0][dx]) * myz + m[0][dx] * (A.w[1] * kyz + A.w[2] * mkz);
        s += coef * ld64(row + q[0][dx]);
      }
    }
  ax = s;
  diag = (A.alpha * m[0][1] + A.w[0] * kk[0][1]) * m[1][1] * m[2][1] +
         m[0][1] * (A.w[1] * kk[1][1] * m[2][1] + A.w[2] * m[1][1] * kk[2][1]);
}

// Table-level kernels run on a 3-D launch: a block is 64 x 4 samples of one
// (x, y) tile, a thread HZ consecutive z-samples (no index division).
constexpr int HBX = 64, HBY = 4, HZ = 4;

// one colour of an 8-colour Gauss-Seidel sweep, in place: sample (i, j, k)
// has colour (i & 1) + 2 (j & 1) + 4 (k & 1); samples of a colour are not
// coupled by the 27-point stencil.  The launch spans the colour's
// sub-lattice (i = 2 ii + ci, ...).
template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_gs8(GridDesc G, HybAxes A, int colour, S* __restrict__ x, const S* __restrict__ b) {
  const int ci = colour & 1, cj = (colour >> 1) & 1, ck = colour >> 2;
  const int i = 2 * (int)(blockIdx.x * HBX + threadIdx.x) + ci, j = 2 * (int)(blockIdx.y * HBY + threadIdx.y) + cj;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  for (int kk = blockIdx.z * HZ; kk < (int)(blockIdx.z + 1) * HZ; ++kk) {
    const int k = 2 * kk + ck;
    if (k >= G.nz) break;
    double ax, d;
    hyb_row(A, G, x, i, j, k, ax, d);
    const int64_t v = G.off + k * pl + (int64_t)j * G.px + i;
    const double xc = ld64(x + v);
    st64(x + v, d != 0.0 ? xc + (ld64(b + v) - ax) / d : 0.0);
  }
}

// r = b - A x on a table level (all samples); with partials, the FP64 sum
// of r^2 per block (block = x + gx (y + gy z)), in a fixed order
template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_residual(GridDesc G, HybAxes A, const S* __restrict__ x, const S* __restrict__ b, S* __restrict__ r,
               double* __restrict__ partials) {
  __shared__ double red[HBY];
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  double rr = 0.0;
  if (i < G.nx && j < G.ny) {
    const int64_t pl = (int64_t)G.px * G.ny;
    for (int k = blockIdx.z * HZ; k < min((int)(blockIdx.z + 1) * HZ, G.nz); ++k) {
      double ax, d;
      hyb_row(A, G, x, i, j, k, ax, d);
      const int64_t v = G.off + k * pl + (int64_t)j * G.px + i;
      const double q = ld64(b + v) - ax;
      st64(r + v, q);
      rr += q * q;
    }
  }
  if (!partials) return;  // uniform over the launch
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o, 64);
  if (threadIdx.x == 0) red[threadIdx.y] = rr;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double t = 0.0;
    for (int w = 0; w < HBY; ++w) t += red[w];
    partials[blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)] = t;
  }
}

// the caller's input (caller layout, dtype Tin) copied into a level array
template <typename Tin, typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_load_input(GridDesc G, const Tin* __restrict__ in, S* __restrict__ out) {
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  for (int k = blockIdx.z * HZ; k < min((int)(blockIdx.z + 1) * HZ, G.nz); ++k)
    st64(out + G.off + k * pl + (int64_t)j * G.px + i, in_at(in, G.ioff + (int64_t)k * G.ipz + (int64_t)j * G.ipy + i));
}

// r = b - A x on the finest (7-point) level, with the FP64 sum of r^2 per
// block (partials[block], block = x + gx (y + gy z)), summed in a fixed
// order.  A thread takes HZ7 z-samples; a full chunk is unrolled so that its
// loads issue together.
constexpr int HZ7 = 8;

template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_residual7(GridDesc G, const S* __restrict__ x, const S* __restrict__ b, S* __restrict__ r,
                double* __restrict__ partials) {
  using C = typename Ty<S>::C;
  __shared__ double red[HBY];
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  double rr = 0.0;
  if (i < G.nx && j < G.ny) {
    const int64_t pl = (int64_t)G.px * G.ny, py = G.px;
    const C alpha = (C)G.alpha;
    const C wl = i > 0 ? (C)G.wx : (C)0, wr = i + 1 < G.nx ? (C)G.wx : (C)0;
    const C wd = j > 0 ? (C)G.wy : (C)0, wu = j + 1 < G.ny ? (C)G.wy : (C)0;
    const int64_t ol = i > 0 ? -1 : 0, orr = i + 1 < G.nx ? 1 : 0, od = j > 0 ? -py : 0, ou = j + 1 < G.ny ? py : 0;
    auto one = [&](int k) {
      const int64_t v = G.off + k * pl + (int64_t)j * py + i;
      const C wb = k > 0 ? (C)G.wz : (C)0, wf = k + 1 < G.nz ? (C)G.wz : (C)0;
      const int64_t ob = k > 0 ? -pl : 0, of = k + 1 < G.nz ? pl : 0;
      const C xc = Ty<S>::ld(x + v);
      C q = Ty<S>::ld(b + v) - alpha * xc;
      q += wl * (Ty<S>::ld(x + v + ol) - xc);
      q += wr * (Ty<S>::ld(x + v + orr) - xc);
      q += wd * (Ty<S>::ld(x + v + od) - xc);
      q += wu * (Ty<S>::ld(x + v + ou) - xc);
      q += wb * (Ty<S>::ld(x + v + ob) - xc);
      q += wf * (Ty<S>::ld(x + v + of) - xc);
      Ty<S>::st(r + v, q);
      rr += (double)q * (double)q;
    };
    const int k0 = blockIdx.z * HZ7;
    if (k0 + HZ7 <= G.nz) {
#pragma unroll
      for (int t = 0; t < HZ7; ++t) one(k0 + t);
    } else {
      for (int k = k0; k < G.nz; ++k) one(k);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o, 64);
  if (threadIdx.x == 0) red[threadIdx.y] = rr;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    double t = 0.0;
    for (int w = 0; w < HBY; ++w) t += red[w];
    partials[blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z)] = t;
  }
}

// coarse b = P^T r (gathered by each coarse sample), coarse x = 0
template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_restrict(GridDesc G, const S* __restrict__ r, S* __restrict__ bc, S* __restrict__ xc) {
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  if (i >= G.cnx || j >= G.cny) return;
  const int64_t pl = (int64_t)G.px * G.ny, cpl = (int64_t)G.cpx * G.cny;
  const bool hx = G.fx == 2, hy = G.fy == 2, hz = G.fz == 2;
  const int x0 = hx ? 2 * i : i, y0 = hy ? 2 * j : j;
  for (int k = blockIdx.z * HZ; k < min((int)(blockIdx.z + 1) * HZ, G.cnz); ++k) {
    const int z0 = hz ? 2 * k : k;
    double s = 0.0;
    for (int dz = (hz ? -1 : 0); dz <= (hz ? 1 : 0); ++dz) {
      const int f = z0 + dz;
      if (f < 0 || f >= G.nz) continue;
      const double wz = bsp_weight(f, k, G.nz, G.cnz, hz);
      for (int dy = (hy ? -1 : 0); dy <= (hy ? 1 : 0); ++dy) {
        const int g = y0 + dy;
        if (g < 0 || g >= G.ny) continue;
        const double wyz = wz * bsp_weight(g, j, G.ny, G.cny, hy);
        for (int dx = (hx ? -1 : 0); dx <= (hx ? 1 : 0); ++dx) {
          const int h = x0 + dx;
          if (h < 0 || h >= G.nx) continue;
          s += wyz * bsp_weight(h, i, G.nx, G.cnx, hx) * ld64(r + G.off + f * pl + (int64_t)g * G.px + h);
        }
      }
    }
    const int64_t v = G.coff + k * cpl + (int64_t)j * G.cpx + i;
    st64(bc + v, s);
    st64(xc + v, 0.0);
  }
}

// x += P e (each fine sample gathers its coarse parents)
template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_prolong(GridDesc G, const S* __restrict__ e, S* __restrict__ x) {
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny, cpl = (int64_t)G.cpx * G.cny;
  const bool hv[3] = {G.fx == 2, G.fy == 2, G.fz == 2};
  const int nc[3] = {G.cnx, G.cny, G.cnz};
  // parents along an axis: (index, weight) x 2, weight 0 when absent
  auto parents = [&](int a, int f, int* pa, double* pw) {
    if (!hv[a] || (f & 1) == 0) { pa[0] = pa[1] = hv[a] ? f / 2 : f; pw[0] = 1.0; pw[1] = 0.0; return; }
    const int lo = (f - 1) / 2, hi = (f + 1) / 2;
    if (hi < nc[a]) { pa[0] = lo; pa[1] = hi; pw[0] = pw[1] = 0.5; }
    else { pa[0] = pa[1] = lo; pw[0] = 1.0; pw[1] = 0.0; }
  };
  int px_[2], py_[2], pz_[2];
  double wx_[2], wy_[2], wz_[2];
  parents(0, i, px_, wx_);
  parents(1, j, py_, wy_);
  for (int k = blockIdx.z * HZ; k < min((int)(blockIdx.z + 1) * HZ, G.nz); ++k) {
    parents(2, k, pz_, wz_);
    double s = 0.0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cx = 0; cx < 2; ++cx) {
          const double wgt = wx_[cx] * wy_[cy] * wz_[cz];
          if (wgt != 0.0) s += wgt * ld64(e + G.coff + pz_[cz] * cpl + (int64_t)py_[cy] * G.cpx + px_[cx]);
        }
    const int64_t v = G.off + k * pl + (int64_t)j * G.px + i;
    st64(x + v, ld64(x + v) + s);
  }
}

// ------------------------------------------------- Krylov vector kernels
// (caller's layout, one grid).  q = A p with the per-block FP64 sum of p.q.
template <typename S>
__global__ void __launch_bounds__(256)
k_apply_dot(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
            const S* __restrict__ pin, S* __restrict__ qout, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  double pq = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = G.ipz, py = G.ipy;
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = G.ioff + k * pl + (int64_t)j * py + i;
      const double pc = ld64(pin + v);
      double q = G.alpha * pc;
      if (i > 0) q += G.wx * (pc - ld64(pin + v - 1));
      if (i < nx - 1) q += G.wx * (pc - ld64(pin + v + 1));
      if (j > 0) q += G.wy * (pc - ld64(pin + v - py));
      if (j < ny - 1) q += G.wy * (pc - ld64(pin + v + py));
      if (k > 0) q += G.wz * (pc - ld64(pin + v - pl));
      if (k < nz - 1) q += G.wz * (pc - ld64(pin + v + pl));
      st64(qout + v, q);
      pq += pc * q;
    }
  }
  const double s = block_sum(pq, red);
  if (threadIdx.x == 0) partials[t.bid] = s;
}

// per-block FP64 sum of a.b
template <typename S>
__global__ void __launch_bounds__(256)
k_dot(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
      const S* __restrict__ a, const S* __restrict__ b, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  double s = 0.0;
  if (i < G.nx && j < G.ny)
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
      s += ld64(a + v) * ld64(b + v);
    }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) partials[t.bid] = tot;
}

// x += alpha p, r -= alpha q, per-block FP64 sum of r^2 (alpha = coef[0])
template <typename S>
__global__ void __launch_bounds__(256)
k_cg_update(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
            const double* __restrict__ coef, S* __restrict__ x, S* __restrict__ r, const S* __restrict__ p,
            const S* __restrict__ q, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  const double a = coef[0];
  double s = 0.0;
  if (i < G.nx && j < G.ny)
    for (int k = t.z0; k < t.z1; ++k) {
      const int64_t v = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
      st64(x + v, ld64(x + v) + a * ld64(p + v));
      const double rn = ld64(r + v) - a * ld64(q + v);
      st64(r + v, rn);
      s += rn * rn;
    }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) partials[t.bid] = tot;
}

// out = a X + b Y (coef[0], coef[1]); Y may alias out
template <typename S>
__global__ void __launch_bounds__(256)
k_axpby(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
        const double* __restrict__ coef, const S* X, const S* Y, S* out) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  const int i = t.x0 + (threadIdx.x % etx), j = t.y0 + (threadIdx.x / etx);
  if (i >= G.nx || j >= G.ny) return;
  const double a = coef[0], b = coef[1];
  for (int k = t.z0; k < t.z1; ++k) {
    const int64_t v = G.ioff + k * G.ipz + (int64_t)j * G.ipy + i;
    st64(out + v, a * ld64(X + v) + b * ld64(Y + v));
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

#define GD_ARGS(geom) dim3((unsigned)(geom).nblocks), dim3(256), 0, st, (geom).grids, (geom).block0, (geom).ngrids, (geom).zlen, (geom).etx

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

template <typename T, bool FP, bool VEC>
static void sweep_launch3(const Geom& g, const void* xin, void* xout, const void* b, const void* ec, int pmode,
                          hipStream_t st) {
  if (g.row) {
    hipLaunchKernelGGL((k_rb_sweep<T, SWR_TX, 1, FP, VEC>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 2), 0, st,
                       g.grids, g.block0, g.ngrids, g.zlen, (const T*)xin, (T*)xout, (const T*)b, (const T*)ec,
                       pmode, g.order);
  } else {
#define SWEEP_TILE(TX, TY)                                                                                     \
  hipLaunchKernelGGL((k_rb_sweep<T, TX, TY, FP, VEC>), dim3((unsigned)g.nblocks), dim3(TX * TY / 2), 0, st,    \
                     g.grids, g.block0, g.ngrids, g.zlen, (const T*)xin, (T*)xout, (const T*)b, (const T*)ec, pmode, \
                     g.order)
    if (FP || g.tile == 0) {
      SWEEP_TILE(64, 8);
    } else if constexpr (!FP) {  // the fused prolongation exists for the 64 x 8 tile only
      switch (g.tile) {
        case 1: SWEEP_TILE(128, 8); break;
        case 2: SWEEP_TILE(64, 16); break;
        default: SWEEP_TILE(128, 16); break;
      }
    }
#undef SWEEP_TILE
  }
}

template <typename T>
static void sweep_launch(const Geom& g, const void* xin, void* xout, const void* b, const void* ec, int pmode,
                         hipStream_t st) {
  // the library's arrays are pair-aligned (g.vec); a caller's odd-width arrays are not
  if (ec) sweep_launch3<T, true, true>(g, xin, xout, b, ec, pmode, st);
  else if (g.vec) sweep_launch3<T, false, true>(g, xin, xout, b, ec, pmode, st);
  else sweep_launch3<T, false, false>(g, xin, xout, b, ec, pmode, st);
}

hipError_t launch_rb_sweep(gd_dtype s, const Geom& g, const void* xin, void* xout, const void* b,
                           const void* ec, int pmode, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) sweep_launch<T>(g, xin, xout, b, ec, pmode, st)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

template <typename T>
static void restrict_z_launch(const Geom& g, const void* x, const void* b, void* bc, void* xc, double* partials,
                              hipStream_t st) {
  if (g.row)
    hipLaunchKernelGGL((k_restrict_z<T, SWR_TX, 1>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 2), 0, st, g.grids,
                       g.block0, g.ngrids, g.zlen, (const T*)x, (const T*)b, (T*)bc, (T*)xc, partials);
  else
    hipLaunchKernelGGL((k_restrict_z<T, SW_TX, SW_TY>), dim3((unsigned)g.nblocks), dim3(SW_TX * SW_TY / 2), 0, st,
                       g.grids, g.block0, g.ngrids, g.zlen, (const T*)x, (const T*)b, (T*)bc, (T*)xc, partials);
}

hipError_t launch_restrict_z(gd_dtype s, const Geom& g, const void* x, const void* b, void* bc, void* xc,
                             double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) restrict_z_launch<T>(g, x, b, bc, xc, partials, st)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

template <typename T, bool KEEPX>
static void prolong_pair_launch(const Geom& g, const void* ec, void* x, int mode, hipStream_t st) {
  if (g.row)
    hipLaunchKernelGGL((k_prolong_pair<T, SWR_TX, 1, KEEPX>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 2), 0, st,
                       g.grids, g.block0, g.ngrids, g.zlen, (const T*)ec, (T*)x, mode);
  else
    hipLaunchKernelGGL((k_prolong_pair<T, SW_TX, SW_TY, KEEPX>), dim3((unsigned)g.nblocks), dim3(SW_TX * SW_TY / 2),
                       0, st, g.grids, g.block0, g.ngrids, g.zlen, (const T*)ec, (T*)x, mode);
}

hipError_t launch_prolong_pair(gd_dtype s, const Geom& g, const void* ec, void* x, int mode, bool keep_x,
                               hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) keep_x ? prolong_pair_launch<T, true>(g, ec, x, mode, st) : prolong_pair_launch<T, false>(g, ec, x, mode, st)
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

template <typename TI, typename T, int KIND, int MODE>
static void corr_stencil_launch(const Geom& g, const void* I0, const void* I1, const void* E, const double* x64,
                                void* o0, void* o1, const double* inv_scale, double* partials, double* x64o,
                                const double* escale, hipStream_t st) {
  if (g.row)
    hipLaunchKernelGGL((k_corr_stencil<TI, T, SWR_TX, 1, KIND, MODE>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 2), 0,
                       st, g.grids, g.block0, g.ngrids, g.zlen, (const TI*)I0, (const TI*)I1, (const T*)E, x64, (T*)o0,
                       (T*)o1, inv_scale, partials, x64o, escale);
  else
    hipLaunchKernelGGL((k_corr_stencil<TI, T, SW_TX, SW_TY, KIND, MODE>), dim3((unsigned)g.nblocks),
                       dim3(SW_TX * SW_TY / 2), 0, st, g.grids, g.block0, g.ngrids, g.zlen, (const TI*)I0,
                       (const TI*)I1, (const T*)E, x64, (T*)o0, (T*)o1, inv_scale, partials, x64o, escale);
}

hipError_t launch_rhs_corr(gd_dtype tin, gd_dtype s, const Geom& g, const void* I0, const void* I1, void* b,
                           void* x, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T) \
  corr_stencil_launch<TI, T, 0, 0>(g, I0, I1, nullptr, nullptr, b, x, nullptr, partials, nullptr, nullptr, st)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  return last();
}

hipError_t launch_canon_residual(gd_dtype tin, gd_dtype s, int mode, const Geom& g, const void* I0,
                                 const void* I1, const void* E, const double* x64, void* r_out,
                                 const double* inv_scale, double* partials, hipStream_t st, double* x64_out,
                                 const double* e_scale) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T)                                                                                              \
  if (mode == 0)                                                                                               \
    corr_stencil_launch<TI, T, 1, 0>(g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, nullptr, nullptr, st); \
  else if (mode == 1)                                                                                          \
    corr_stencil_launch<TI, T, 1, 1>(g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, nullptr, nullptr, st); \
  else                                                                                                         \
    corr_stencil_launch<TI, T, 1, 2>(g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, x64_out, e_scale, st)
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


hipError_t launch_rhs_general(gd_dtype s, const Geom& g, const void* V, const void* Gx, const void* Gy,
                              const void* Gz, void* b, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_rhs_general<T>, GD_ARGS(g), (const T*)V, (const T*)Gx, (const T*)Gy, (const T*)Gz, (T*)b)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_general_residual(gd_dtype s, const Geom& g, const void* x, const void* b, void* r_out,
                                   double* partials, hipStream_t st, bool lib_layout, int klo, int khi) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T)                                                                                              \
  if (lib_layout)                                                                                         \
    hipLaunchKernelGGL((k_general_residual<T, true>), GD_ARGS(g), (const T*)x, (const T*)b, (T*)r_out,  \
                       partials, klo, khi);                                                               \
  else                                                                                                    \
    hipLaunchKernelGGL((k_general_residual<T, false>), GD_ARGS(g), (const T*)x, (const T*)b, (T*)r_out, \
                       partials, klo, khi)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

static dim3 hyb_grid(int64_t nx, int64_t ny, int64_t nz) {
  return dim3((unsigned)((nx + HBX - 1) / HBX), (unsigned)((ny + HBY - 1) / HBY), (unsigned)((nz + HZ - 1) / HZ));
}

hipError_t launch_hyb_gs8(gd_dtype s, const GridDesc& G, const HybTables& T, int colour, void* x, const void* b,
                          hipStream_t st) {
  const int ci = colour & 1, cj = (colour >> 1) & 1, ck = colour >> 2;
  const int64_t mx = (G.nx - ci + 1) / 2, my = (G.ny - cj + 1) / 2, mz = (G.nz - ck + 1) / 2;
  if (mx * my * mz == 0) return hipSuccess;
  HybAxes A{{T.t[0], T.t[1], T.t[2]}, T.alpha, {T.w[0], T.w[1], T.w[2]}};
#define L(TT) hipLaunchKernelGGL(k_hyb_gs8<TT>, hyb_grid(mx, my, mz), dim3(HBX, HBY), 0, st, G, A, colour, (TT*)x, \
                                 (const TT*)b)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

int64_t hyb_residual_blocks(const GridDesc& G) {
  const dim3 g = hyb_grid(G.nx, G.ny, G.nz);
  return (int64_t)g.x * g.y * g.z;
}

hipError_t launch_hyb_residual(gd_dtype s, const GridDesc& G, const HybTables& T, const void* x, const void* b,
                               void* r, hipStream_t st, double* partials) {
  HybAxes A{{T.t[0], T.t[1], T.t[2]}, T.alpha, {T.w[0], T.w[1], T.w[2]}};
#define L(TT) hipLaunchKernelGGL(k_hyb_residual<TT>, hyb_grid(G.nx, G.ny, G.nz), dim3(HBX, HBY), 0, st, G, A, \
                                 (const TT*)x, (const TT*)b, (TT*)r, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

template <typename TI>
static void load_input_launch(gd_dtype s, const GridDesc& G, const void* in, void* out, hipStream_t st) {
#define L(TT) hipLaunchKernelGGL((k_load_input<TI, TT>), hyb_grid(G.nx, G.ny, G.nz), dim3(HBX, HBY), 0, st, G, \
                                 (const TI*)in, (TT*)out)
  switch (s) {
    case GD_F64: L(double); break;
    case GD_F32: L(float); break;
    case GD_F16: L(__half); break;
    case GD_BF16: L(__hip_bfloat16); break;
    default: break;
  }
#undef L
}

hipError_t launch_load_input(gd_dtype tin, gd_dtype s, const GridDesc& G, const void* in, void* out, hipStream_t st) {
#define L(TI) load_input_launch<TI>(s, G, in, out, st)
  GD_DISPATCH_S(tin, L)
#undef L
  return last();
}

static dim3 hyb7_grid(const GridDesc& G) {
  return dim3((unsigned)((G.nx + HBX - 1) / HBX), (unsigned)((G.ny + HBY - 1) / HBY),
              (unsigned)((G.nz + HZ7 - 1) / HZ7));
}

int64_t hyb_residual7_blocks(const GridDesc& G) {
  const dim3 g = hyb7_grid(G);
  return (int64_t)g.x * g.y * g.z;
}

hipError_t launch_hyb_residual7(gd_dtype s, const GridDesc& G, const void* x, const void* b, void* r,
                                double* partials, hipStream_t st) {
#define L(TT) hipLaunchKernelGGL(k_hyb_residual7<TT>, hyb7_grid(G), dim3(HBX, HBY), 0, st, G, \
                                 (const TT*)x, (const TT*)b, (TT*)r, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_hyb_restrict(gd_dtype s, const GridDesc& G, const void* r, void* bc, void* xc, hipStream_t st) {
#define L(TT) hipLaunchKernelGGL(k_hyb_restrict<TT>, hyb_grid(G.cnx, G.cny, G.cnz), dim3(HBX, HBY), 0, st, G, \
                                 (const TT*)r, (TT*)bc, (TT*)xc)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_hyb_prolong(gd_dtype s, const GridDesc& G, const void* e, void* x, hipStream_t st) {
#define L(TT) hipLaunchKernelGGL(k_hyb_prolong<TT>, hyb_grid(G.nx, G.ny, G.nz), dim3(HBX, HBY), 0, st, G, \
                                 (const TT*)e, (TT*)x)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

template <typename TI>
static void npr_rhs_launch(gd_dtype s, const Geom& g, const void* I0, double lam, double inv2s2, void* b,
                           double* partials, hipStream_t st) {
#define L(T) hipLaunchKernelGGL((k_npr_rhs<TI, T>), GD_ARGS(g), (const TI*)I0, lam, inv2s2, (T*)b, partials)
  switch (s) {
    case GD_F64: L(double); break;
    case GD_F32: L(float); break;
    case GD_F16: L(__half); break;
    case GD_BF16: L(__hip_bfloat16); break;
    default: break;
  }
#undef L
}

hipError_t launch_npr_rhs(gd_dtype tin, gd_dtype s, const Geom& g, const void* I0, double lam, double sigma,
                          void* b, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
#define L(TI) npr_rhs_launch<TI>(s, g, I0, lam, inv2s2, b, partials, st)
  GD_DISPATCH_S(tin, L)
#undef L
  return last();
}

hipError_t launch_apply_dot(gd_dtype s, const Geom& g, const void* p, void* q, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_apply_dot<T>, GD_ARGS(g), (const T*)p, (T*)q, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_dot(gd_dtype s, const Geom& g, const void* a, const void* b, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_dot<T>, GD_ARGS(g), (const T*)a, (const T*)b, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_cg_update(gd_dtype s, const Geom& g, const double* coef, void* x, void* r, const void* p,
                            const void* q, double* partials, hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_cg_update<T>, GD_ARGS(g), coef, (T*)x, (T*)r, (const T*)p, (const T*)q, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return last();
}

hipError_t launch_axpby(gd_dtype s, const Geom& g, const double* coef, const void* X, const void* Y, void* out,
                        hipStream_t st) {
  if (g.nblocks == 0) return hipSuccess;
#define L(T) hipLaunchKernelGGL(k_axpby<T>, GD_ARGS(g), coef, (const T*)X, (const T*)Y, (T*)out)
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
