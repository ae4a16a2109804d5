// gfx950 red-black Gauss-Seidel relaxation (Sec. 4.1, multi-coloured GS) of
// the multigrid solver for the screened anisotropic Poisson systems of
// Kazhdan et al., "Gradient-Domain Processing for Large EM Image Stacks".
// Layout and difference-form conventions as in kernels.hip.
#include "gd_kcommon.h"

namespace gd {

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
  if (G.skip) return;  // a converged grid of a batch
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

// ------------------------------------------------ red-black sweep, quad form
//
// The same sweep with four consecutive x cells per thread (thread t owns
// gx .. gx + 3, gx = x0 + 4 (t mod TX/4), of row gy = y0 + t / (TX/4)), for
// the library's own arrays (x pitch and grid offsets multiples of four, so a
// quad is one aligned 8-byte (16-bit types) or 16-byte (FP32) access) and
// compute type float.  In every plane two cells of a quad are red and two
// black: positions c and c + 2 with c = (gy + p) & 1 are the red cells of
// plane p, and the black cells of planes p - 1 and p + 1 (so the updates of
// a step, red of plane p and black of plane p - 1, are both at positions c
// and c + 2).  The plane pipeline, the LDS planes, the recomputed 1-cell red
// ring and the neighbour order of every update are those of k_rb_sweep, so
// both forms give the same values bit for bit; the quad form issues half the
// loads, address computations and conversions per cell.  The LDS plane is
// TX + 8 wide with the tile at x offset 4, so that a quad is one aligned
// 16-byte LDS access; the 2-cell halo is loaded in aligned quads (full quads
// of the two rows above and below the tile, one quad on each side of its
// rows).
template <int TX, int TY>
struct SweepShape4 {
  static constexpr bool ROW = (TY == 1);
  static constexpr int NT = TX * TY / 4;                 // threads: one x-quad each
  static constexpr int YO = ROW ? 0 : 2;                 // tile row 0 inside the LDS plane
  static constexpr int XO = 4;                           // tile column 0 inside the LDS plane
  static constexpr int HX = TX + 8, HY = ROW ? 1 : TY + 4;
  static constexpr int QR = TX / 4 + 2;                  // quads of a full halo row
  static constexpr int NHQ = ROW ? 2 : 4 * QR + 2 * TY;  // halo quads per plane
  static constexpr int NHQR = (NHQ + NT - 1) / NT;       // halo quads per thread
  static constexpr int NRING = ROW ? 1 : (TX + 2) + TY;  // red ring-1 cells per plane
};

// LDS coordinates (row, first column) of halo quad h
template <int TX, int TY>
__device__ __forceinline__ void halo_quad(int h, int& hy, int& hx) {
  using SS = SweepShape4<TX, TY>;
  constexpr int QR = SS::QR;
  if constexpr (SS::ROW) {
    hy = 0;
    hx = h == 0 ? 0 : TX + 4;
  } else {
    if (h < 2 * QR) { hy = h / QR; hx = 4 * (h - hy * QR); return; }
    h -= 2 * QR;
    if (h < 2 * QR) { const int r = h / QR; hy = TY + 2 + r; hx = 4 * (h - r * QR); return; }
    h -= 2 * QR;
    hy = 2 + (h >> 1);
    hx = (h & 1) ? TX + 4 : 0;
  }
}

// four consecutive raw values (one aligned access)
template <typename S> struct Raw4 {
  using W = std::conditional_t<sizeof(S) == 4, float4, uint2>;
  W w;
};
template <typename S> __device__ __forceinline__ void ld_raw4(const S* p, Raw4<S>& r) {
  r.w = *reinterpret_cast<const typename Raw4<S>::W*>(p);
}
template <typename S> __device__ __forceinline__ float raw4_at(const Raw4<S>& r, int i) {
  if constexpr (sizeof(S) == 4) {
    return i == 0 ? r.w.x : i == 1 ? r.w.y : i == 2 ? r.w.z : r.w.w;
  } else {
    const uint32_t v = (i < 2) ? r.w.x : r.w.y;
    return from_bits16f<S>((i & 1) ? (v >> 16) : (v & 0xffffu));
  }
}
template <typename S> __device__ __forceinline__ uint32_t bits16(float v) {
  S h;
  Ty<S>::st(&h, v);
  uint16_t u;
  __builtin_memcpy(&u, &h, 2);
  return u;
}
template <typename S> __device__ __forceinline__ void st4(S* p, float a, float b, float c, float d) {
  // the stored value is the rounding of the float the sweep computed and
  // keeps using: no instruction may fuse the last multiply-add with the
  // conversion (a mixed-precision FMA would round once, straight to 16 bits)
  asm volatile("" : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
  if constexpr (sizeof(S) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
  } else {
    *reinterpret_cast<uint2*>(p) =
        make_uint2(bits16<S>(a) | (bits16<S>(b) << 16), bits16<S>(c) | (bits16<S>(d) << 16));
  }
}

// Split launch of a one-grid 3-D level: the tiles whose cells, ring and halo
// all lie inside the grid (interior) and the others (the edge ring of tiles).
// Interior tiles are those with tx >= 1, ty >= 1, (tx + 1) TX + 4 <= nx and
// (ty + 1) TY + 2 <= ny.
struct SplitTiles {
  int ntx, nty, txh, tyh, nix, niy;
  __device__ __forceinline__ SplitTiles(int nx, int ny, int TX, int TY) {
    ntx = (nx + TX - 1) / TX;
    nty = (ny + TY - 1) / TY;
    txh = (nx - 4) / TX;
    tyh = (ny - 2) / TY;
    nix = max(0, txh - 1);
    niy = max(0, tyh - 1);
  }
};
// MAP 1: block -> interior tile; MAP 2: block -> edge tile (rows above and
// below the interior band, then the tiles left and right of it)
template <int TX, int TY, int MAP>
__device__ __forceinline__ Tile decode_split(const GridDesc* __restrict__ grids, int zlen) {
  const GridDesc& G = grids[0];
  const SplitTiles s(G.nx, G.ny, TX, TY);
  const int64_t per = MAP == 1 ? (int64_t)s.nix * s.niy : (int64_t)s.ntx * s.nty - (int64_t)s.nix * s.niy;
  const int64_t b = blockIdx.x;
  const int zc = (int)(b / per);
  int r = (int)(b - (int64_t)zc * per), tx, ty;
  if (MAP == 1) {
    ty = 1 + r / s.nix;
    tx = 1 + r % s.nix;
  } else if (r < s.ntx) {  // tile row 0
    ty = 0;
    tx = r;
  } else if ((r -= s.ntx) < s.niy * (1 + s.ntx - s.txh)) {  // left and right of the interior band
    const int m = 1 + s.ntx - s.txh;
    ty = 1 + r / m;
    const int k = r % m;
    tx = k == 0 ? 0 : s.txh + k - 1;
  } else {  // tile rows below the interior band
    r -= s.niy * (1 + s.ntx - s.txh);
    ty = 1 + s.niy + r / s.ntx;
    tx = r % s.ntx;
  }
  Tile t;
  t.g = 0;
  t.bid = b;
  t.x0 = tx * TX;
  t.y0 = ty * TY;
  t.z0 = zc * zlen;
  t.z1 = min(t.z0 + zlen, G.nz);
  return t;
}

// ZX: the input iterate is zero (the first sweep of a V-cycle started from
// zero): x is not read, the sweep starts from zeros.
// MAP 0: the level's tile table; MAP 1: interior tiles of a one-grid level
// (every weight the same, no masks: the per-cell weights, inverse diagonals
// and validity flags fold into uniform values, which frees registers for
// more waves per CU); MAP 2: its edge tiles (the general body).
template <typename S, int TX, int TY, bool ZX, int MAP>
__global__ void __launch_bounds__(TX * TY / 4)
k_rb_sweep4(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
            const S* __restrict__ xin, S* __restrict__ xout, const S* __restrict__ bin, int order) {
  constexpr bool INT = MAP == 1;
  static_assert(sizeof(S) <= 4, "the quad form computes in float");
  using C = float;
  using SS = SweepShape4<TX, TY>;
  constexpr int NT = SS::NT, YO = SS::YO, XO = SS::XO, HX = SS::HX, HY = SS::HY, NHQR = SS::NHQR;
  constexpr int PLANE = HX * HY;
  constexpr bool ROW = SS::ROW;
  constexpr int QPR = TX / 4;                 // quads per tile row
  constexpr int RPW = QPR >= 64 ? 1 : 64 / QPR;  // tile rows per wave
  static_assert(ROW || TY % (2 * RPW) == 0, "waves of rows of one parity");
  using Ring = WaveSplit<SS::NRING, NT>;
  static_assert(Ring::PER <= 64, "ring share per wave");
  // four planes, then one slot per thread that takes the masked writes of
  // threads without a ring cell
  __shared__ __align__(16) C X[4 * PLANE + NT];

  const Tile t = MAP == 0 ? decode_tile(grids, block0, ngrids, zlen, TX, TY, false, order)
                           : decode_split<TX, TY, MAP>(grids, zlen);
  const GridDesc& G = grids[t.g];
  if (G.skip) return;  // a converged grid of a batch
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const C alpha = (C)G.alpha, wx = (C)G.wx, wy = (C)G.wy, wz = (C)G.wz;
  const int64_t pl = (int64_t)px * ny;
  const S* xg = xin + G.off;
  const S* bg = bin + G.off;
  S* xo = xout + G.off;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;

  // ---- own quad (gx .. gx + 3) of row gy.  The rows of a wave have one
  // parity (wave w takes rows 2 RPW (w / 2) + (w & 1) + 2 j), so the cells a
  // step updates (positions c, c + 2, c = (gy + p) & 1) are the same for the
  // whole wave and the step branches on c uniformly.
  const int wv = tid >> 6, ln = tid & 63;
  const int tyl = ROW ? 0 : 2 * RPW * (wv >> 1) + (wv & 1) + 2 * (ln / QPR);
  const int qxl = ROW ? tid : ln % QPR;
  const int wpar = __builtin_amdgcn_readfirstlane((y0 + tyl) & 1);  // row parity, uniform per wave
  const int gx = x0 + 4 * qxl, gy = y0 + tyl;
  const bool rowok = INT || gy < ny;
  const bool v0 = INT || (rowok && gx < nx), v1 = INT || (rowok && gx + 1 < nx), v2 = INT || (rowok && gx + 2 < nx),
             v3 = INT || (rowok && gx + 3 < nx);
  const int lo = (YO + tyl) * HX + XO + 4 * qxl;  // LDS index of gx inside a plane (16-byte aligned)
  const int own = gy * px + gx;                  // element offset inside a plane (< 2^28)
  const C wU = (INT || gy > 0) ? wy : (C)0, wD = (INT || gy + 1 < ny) ? wy : (C)0;
  // per position class k (the updated cells at F = k and S = k + 2): x-weights,
  // inverse diagonals inside the z-range and on its first or last plane, and
  // whether the diagonal is non-zero (keep = 0: the cell is set to 0)
  C wLF[2], wRF[2], wLS[2], wRS[2], invIF[2], invEF[2], invIS[2], invES[2], kIF[2], kEF[2], kIS[2], kES[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int xF = gx + k, xS = gx + k + 2;
    // weights as the pair form gives them: a neighbour in the grid has w_x
    wLF[k] = (INT || xF > 0) ? wx : (C)0;
    wRF[k] = (INT || xF + 1 < nx) ? wx : (C)0;
    wLS[k] = wx;
    wRS[k] = (INT || xS + 1 < nx) ? wx : (C)0;
    const C wz1 = nz > 1 ? wz : (C)0;
    const C dF = alpha + wLF[k] + wRF[k] + wU + wD, dS = alpha + wLS[k] + wRS[k] + wU + wD;
    const C diF = (dF + wz1) + wz1, deF = dF + wz1, diS = (dS + wz1) + wz1, deS = dS + wz1;
    invIF[k] = diF > (C)0 ? (C)1 / diF : (C)0;
    invEF[k] = deF > (C)0 ? (C)1 / deF : (C)0;
    invIS[k] = diS > (C)0 ? (C)1 / diS : (C)0;
    invES[k] = deS > (C)0 ? (C)1 / deS : (C)0;
    kIF[k] = diF > (C)0 ? (C)1 : (C)0;
    kEF[k] = deF > (C)0 ? (C)1 : (C)0;
    kIS[k] = diS > (C)0 ? (C)1 : (C)0;
    kES[k] = deS > (C)0 ? (C)1 : (C)0;
  }

  // ---- halo quads of this thread (loaded every plane)
  int hoff[NHQR], hg[NHQR], hxs[NHQR];
  bool hv[NHQR], hs[NHQR];
#pragma unroll
  for (int k = 0; k < NHQR; ++k) {
    const int h = tid + NT * k;
    int hy = 0, hx = 0;
    if (h < SS::NHQ) halo_quad<TX, TY>(h, hy, hx);
    const int cx = x0 - XO + hx, cy = y0 - YO + hy;
    hs[k] = h < SS::NHQ;
    hv[k] = hs[k] && (INT || (cx >= 0 && cx < nx && cy >= 0 && cy < ny));
    hoff[k] = hy * HX + hx;
    hg[k] = hv[k] ? cy * px + cx : 0;
    hxs[k] = cx;
  }

  // ---- ring red cell of this thread, for each plane parity (k_rb_sweep's
  // ring, in this LDS layout)
  const int rm = Ring::item(tid);
  int ro[2], rg[2];
  bool rv[2];
  C rwl[2], rwr[2], rwu[2], rwd[2], rinvI[2], rinvE[2], rkI[2], rkE[2];
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    int hy = 0, hx = 0;
    if (rm >= 0) ring_red_cell<TX, TY>(rm, x0, y0, par, hy, hx);
    hx += XO - 2;  // the pair form's LDS column -> this layout
    const int cx = x0 - XO + hx, cy = y0 - YO + hy;
    rv[par] = rm >= 0 && (INT || (cx >= 0 && cx < nx && cy >= 0 && cy < ny));
    ro[par] = rm >= 0 ? hy * HX + hx : lo;
    rg[par] = rv[par] ? cy * px + cx : 0;
    rwl[par] = (INT || cx > 0) ? wx : (C)0;
    rwr[par] = (INT || cx < nx - 1) ? wx : (C)0;
    rwu[par] = (INT || cy > 0) ? wy : (C)0;
    rwd[par] = (INT || cy < ny - 1) ? wy : (C)0;
    const C dxy = alpha + rwl[par] + rwr[par] + rwu[par] + rwd[par];
    const C wz1 = nz > 1 ? wz : (C)0;
    const C di = (dxy + wz1) + wz1, de = dxy + wz1;
    rinvI[par] = di > (C)0 ? (C)1 / di : (C)0;
    rinvE[par] = de > (C)0 ? (C)1 / de : (C)0;
    rkI[par] = di > (C)0 ? (C)1 : (C)0;
    rkE[par] = de > (C)0 ? (C)1 : (C)0;
  }

  // Gauss-Seidel value in correction form (the neighbour order of relax());
  // keep = 0 where the diagonal is zero sets the cell to 0 (relax() does that
  // by a test; the two agree in value)
  auto gs = [&](C x, C b, C wl, C nl, C wr, C nr, C wu_, C nu, C wd_, C nd, C wzm, C nzm, C wzp, C nzp, C inv,
                C keep) -> C {
    C r = fmac(-alpha, x, b);
    r = fmac(wl, nl - x, r);
    r = fmac(wr, nr - x, r);
    if (!ROW) {
      r = fmac(wu_, nu - x, r);
      r = fmac(wd_, nd - x, r);
    }
    r = fmac(wzm, nzm - x, r);
    r = fmac(wzp, nzp - x, r);
    return fmac(r, inv, x * keep);
  };

  struct XSet {
    Raw4<S> p;          // own quad
    Raw4<S> h[NHQR];    // halo quads
  };
  // loads from clamped, always valid addresses: a plane outside [0, nz) only
  // ever enters with a zero z-weight, cells outside the grid are masked to 0
  auto plane_ptr = [&](const S* base, int q) { return base + (int64_t)min(max(q, 0), nz - 1) * pl; };
  auto fetch_x = [&](int q, XSet& o) {
    if constexpr (ZX) {
      __builtin_memset(&o, 0, sizeof o);
      (void)q;
    } else {
      const S* P = plane_ptr(xg, q);
      ld_raw4(P + (v0 ? own : 0), o.p);
#pragma unroll
      for (int k = 0; k < NHQR; ++k) ld_raw4(P + hg[k], o.h[k]);
    }
  };
  auto xq = [&](const Raw4<S>& r, int i, bool v) -> C { return v ? raw4_at(r, i) : (C)0; };
  auto stash = [&](int q, const XSet& o) {
    C* P = X + (q & 3) * PLANE;
    *reinterpret_cast<float4*>(P + lo) = make_float4(xq(o.p, 0, v0), xq(o.p, 1, v1), xq(o.p, 2, v2), xq(o.p, 3, v3));
#pragma unroll
    for (int k = 0; k < NHQR; ++k)
      if (hs[k]) {
        float4 v;
        const bool ok = hv[k];
        v.x = (ok && hxs[k] + 0 < nx) ? raw4_at(o.h[k], 0) : (C)0;
        v.y = (ok && hxs[k] + 1 < nx) ? raw4_at(o.h[k], 1) : (C)0;
        v.z = (ok && hxs[k] + 2 < nx) ? raw4_at(o.h[k], 2) : (C)0;
        v.w = (ok && hxs[k] + 3 < nx) ? raw4_at(o.h[k], 3) : (C)0;
        *reinterpret_cast<float4*>(P + hoff[k]) = v;
      }
  };
  auto fetch_b = [&](int q, Raw4<S>& r) { ld_raw4(plane_ptr(bg, q) + (v0 ? own : 0), r); };
  // quad of a plane whose red cells are at c, c + 2 -> red (a, b), black (a, b)
  auto split = [&](auto CC, const Raw4<S>& r, C& Ra, C& Rb, C& Ka, C& Kb) {
    constexpr int c = decltype(CC)::value;
    const C a0 = xq(r, 0, v0), a1 = xq(r, 1, v1), a2 = xq(r, 2, v2), a3 = xq(r, 3, v3);
    Ra = c ? a1 : a0;
    Rb = c ? a3 : a2;
    Ka = c ? a0 : a1;
    Kb = c ? a2 : a3;
  };
  using K0 = std::integral_constant<int, 0>;
  using K1 = std::integral_constant<int, 1>;
  auto split_q = [&](int q, const Raw4<S>& r, C& Ra, C& Rb, C& Ka, C& Kb) {
    if (((wpar + q) & 1) != 0) split(K1{}, r, Ra, Rb, Ka, Kb);
    else split(K0{}, r, Ra, Rb, Ka, Kb);
  };
  auto ring_b = [&](int q) -> Raw<S> {
    Raw<S> r;
    ld_raw(plane_ptr(bg, q) + rg[q & 1], r);
    return r;
  };

  // column registers: red (a, b) / black (a, b) of planes p-2 .. p+1; b of planes p-1, p
  C RAm2 = 0, RBm2 = 0, KAm2 = 0, KBm2 = 0;
  C RAm1, RBm1, KAm1, KBm1, RA0, RB0, KA0, KB0, RAp1, RBp1, KAp1, KBp1;
  C bRAm1, bRBm1, bKAm1, bKBm1, bRA0, bRB0, bKA0, bKB0;
  XSet S0, S1;
  Raw4<S> B0, B1;
  Raw<S> RB0r, RB1r;
  const int pfirst = max(q0 - 1, 0);
  const int plast = (q1 < nz) ? q1 : nz;  // p == nz: black of the last plane only
  {
    XSet t0;
    Raw4<S> tb;
    fetch_x(pfirst - 1, t0); stash(pfirst - 1, t0); split_q(pfirst - 1, t0.p, RAm1, RBm1, KAm1, KBm1);
    fetch_x(pfirst, t0);     stash(pfirst, t0);     split_q(pfirst, t0.p, RA0, RB0, KA0, KB0);
    fetch_x(pfirst + 1, t0); stash(pfirst + 1, t0); split_q(pfirst + 1, t0.p, RAp1, RBp1, KAp1, KBp1);
    fetch_b(pfirst - 1, tb); split_q(pfirst - 1, tb, bRAm1, bRBm1, bKAm1, bKBm1);
    fetch_b(pfirst, tb);     split_q(pfirst, tb, bRA0, bRB0, bKA0, bKB0);
  }
  RB0r = ring_b(pfirst);
  RB1r = ring_b(pfirst + 1);
  fetch_x(pfirst + 2, S0);
  fetch_x(pfirst + 3, S1);
  fetch_b(pfirst + 1, B1);
  fetch_b(pfirst + 2, B0);

  // one plane step for plane parity PAR and updated positions c, c + 2 (CC)
  auto body = [&](auto PC, auto CC, int p, XSet& XS, Raw4<S>& BS, Raw<S>& RBS) {
    constexpr int par = decltype(PC)::value;
    constexpr int c = decltype(CC)::value;
    constexpr bool EDGE = true;
    __syncthreads();
    constexpr int dF = c, dS = c + 2, dO = c ? 4 : -1;  // LDS offsets from lo: F, S, outside neighbour
    if (p < nz) {
      // ---- red cells of plane p (F, S) and the ring cell
      C* P = X + (p & 3) * PLANE;
      const C* Pm = X + ((p - 1) & 3) * PLANE;
      const C* Pp = X + ((p + 1) & 3) * PLANE;
      const C wzm = (!EDGE || p > 0) ? wz : (C)0, wzp = (!EDGE || p < nz - 1) ? wz : (C)0;
      const bool edge = EDGE && (p == 0 || p == nz - 1);
      const C out = P[lo + dO];
      const C upF = ROW ? (C)0 : P[lo + dF - HX], dnF = ROW ? (C)0 : P[lo + dF + HX];
      const C upS = ROW ? (C)0 : P[lo + dS - HX], dnS = ROW ? (C)0 : P[lo + dS + HX];
      const int o = ro[par];
      const C rx = P[o], rl = P[o - 1], rr = P[o + 1];
      const C ru = ROW ? (C)0 : P[o - HX], rd = ROW ? (C)0 : P[o + HX];
      const C rzm = Pm[o], rzp = Pp[o];
      const C nF = gs(RA0, bRA0, wLF[c], c ? KA0 : out, wRF[c], c ? KB0 : KA0, wU, upF, wD, dnF, wzm, KAm1, wzp,
                      KAp1, edge ? invEF[c] : invIF[c], edge ? kEF[c] : kIF[c]);
      const C nS = gs(RB0, bRB0, wLS[c], c ? KB0 : KA0, wRS[c], c ? out : KB0, wU, upS, wD, dnS, wzm, KBm1, wzp,
                      KBp1, edge ? invES[c] : invIS[c], edge ? kES[c] : kIS[c]);
      RA0 = (c ? v1 : v0) ? nF : (C)0;
      RB0 = (c ? v3 : v2) ? nS : (C)0;
      P[lo + dF] = RA0;
      P[lo + dS] = RB0;
      const C rb = rv[par] ? raw_c(RBS) : (C)0;
      const C rn = gs(rx, rb, rwl[par], rl, rwr[par], rr, rwu[par], ru, rwd[par], rd, wzm, rzm, wzp, rzp,
                      edge ? rinvE[par] : rinvI[par], edge ? rkE[par] : rkI[par]);
      *(rv[par] ? P + o : X + 4 * PLANE + tid) = rn;
    }
    // no barrier here: the black cells of plane p - 1 read only plane
    // p - 1's buffer, whose red cells were written in the previous step
    const int q = p - 1;
    if (q >= q0 && q < q1) {
      // ---- black cells of plane q = p - 1 (at F, S: the red positions of plane p)
      const C* P = X + (q & 3) * PLANE;
      const C wzm = (!EDGE || q > 0) ? wz : (C)0, wzp = (!EDGE || q < nz - 1) ? wz : (C)0;
      const bool edge = EDGE && (q == 0 || q == nz - 1);
      const C out = P[lo + dO];
      const C upF = ROW ? (C)0 : P[lo + dF - HX], dnF = ROW ? (C)0 : P[lo + dF + HX];
      const C upS = ROW ? (C)0 : P[lo + dS - HX], dnS = ROW ? (C)0 : P[lo + dS + HX];
      const C nF = gs(KAm1, bKAm1, wLF[c], c ? RAm1 : out, wRF[c], c ? RBm1 : RAm1, wU, upF, wD, dnF, wzm, RAm2,
                      wzp, RA0, edge ? invEF[c] : invIF[c], edge ? kEF[c] : kIF[c]);
      const C nS = gs(KBm1, bKBm1, wLS[c], c ? RBm1 : RAm1, wRS[c], c ? out : RBm1, wU, upS, wD, dnS, wzm, RBm2,
                      wzp, RB0, edge ? invES[c] : invIS[c], edge ? kES[c] : kIS[c]);
      KAm1 = (c ? v1 : v0) ? nF : (C)0;
      KBm1 = (c ? v3 : v2) ? nS : (C)0;
      // memory order of plane q: red at c ^ 1 and (c ^ 1) + 2, black at c and c + 2
      if (v0) {
        if (c) st4(xo + (int64_t)q * pl + own, RAm1, KAm1, RBm1, KBm1);
        else st4(xo + (int64_t)q * pl + own, KAm1, RAm1, KBm1, RBm1);
      }
    }
    stash(p + 2, XS);
    RAm2 = RAm1; RBm2 = RBm1; KAm2 = KAm1; KBm2 = KBm1;
    RAm1 = RA0; RBm1 = RB0; KAm1 = KA0; KBm1 = KB0;
    RA0 = RAp1; RB0 = RBp1; KA0 = KAp1; KB0 = KBp1;
    // plane p + 2 has plane p's parity: its red cells are at c, c + 2
    split(CC, XS.p, RAp1, RBp1, KAp1, KBp1);
    bRAm1 = bRA0; bRBm1 = bRB0; bKAm1 = bKA0; bKBm1 = bKB0;
    split(std::integral_constant<int, 1 - c>{}, BS, bRA0, bRB0, bKA0, bKB0);  // plane p + 1
    fetch_x(p + 4, XS);
    fetch_b(p + 3, BS);
    ld_raw(plane_ptr(bg, p + 2) + rg[par], RBS);  // ring b of plane p + 2 (same parity)
  };
  // The updated positions of a step, c = (gy + p) & 1, are uniform per wave
  // and alternate with p, so the unrolled pair of steps of the loop has a
  // fixed (c, 1 - c): one loop per (parity of the first plane, its c).
  auto loop = [&](auto P0, auto C0) {
    using P1 = std::integral_constant<int, 1 - decltype(P0)::value>;
    using C1 = std::integral_constant<int, 1 - decltype(C0)::value>;
    int p = pfirst;
    for (; p + 1 <= plast; p += 2) {
      body(P0, C0, p, S0, B1, RB0r);
      body(P1{}, C1{}, p + 1, S1, B0, RB1r);
    }
    if (p <= plast) body(P0, C0, p, S0, B1, RB0r);
  };
  using E0 = std::integral_constant<int, 0>;
  using E1 = std::integral_constant<int, 1>;
  const int c0 = (wpar + pfirst) & 1;  // wave-uniform
  if ((pfirst & 1) == 0) {
    if (c0) loop(E0{}, K1{});
    else loop(E0{}, K0{});
  } else {
    if (c0) loop(E1{}, K1{});
    else loop(E1{}, K0{});
  }
}

// ============================================================ launchers

template <typename T, bool FP, bool VEC>
static hipError_t sweep_launch3(const Geom& g, const void* xin, void* xout, const void* b, const void* ec, int pmode,
                          hipStream_t st) {
  if (g.row) {
    hipLaunchKernelGGL((k_rb_sweep<T, SWR_TX, 1, FP, VEC>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 2), 0, st,
                       g.grids, g.block0, g.ngrids, g.zlen, (const T*)xin, (T*)xout, (const T*)b, (const T*)ec,
                       pmode, g.order);
  } else if (g.tile >= kPairTiles) {
    return hipErrorInvalidValue;  // the wide tiles exist in the quad form only
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
  return hipSuccess;
}

// The quad form for the library's arrays (float compute types), unless
// GD_SWEEP_QUAD=0 asks for the pair form (same values either way).
static bool quad_on() {
  static const bool v = [] {
    const char* e = std::getenv("GD_SWEEP_QUAD");
    return !(e && std::atoi(e) == 0);
  }();
  return v;
}

template <typename T, bool ZX, int TX, int TY>
static void sweep_launch4t(const Geom& g, const void* xin, void* xout, const void* b, hipStream_t st) {
#define SWEEP4(MAP, NB, ZL)                                                                                      \
  hipLaunchKernelGGL((k_rb_sweep4<T, TX, TY, ZX, MAP>), dim3((unsigned)(NB)), dim3(TX * TY / 4), 0, st, g.grids, \
                     g.block0, g.ngrids, ZL, (const T*)xin, (T*)xout, (const T*)b, g.order)
  if (g.n_int > 0) {  // one-grid level: interior tiles, then the edge tiles
    SWEEP4(1, g.n_int, g.zlen);
    if (g.n_edge > 0) SWEEP4(2, g.n_edge, g.zlen_edge);
  } else {
    SWEEP4(0, g.nblocks, g.zlen);
  }
#undef SWEEP4
}

template <typename T, bool ZX>
static void sweep_launch4(const Geom& g, const void* xin, void* xout, const void* b, hipStream_t st) {
  if (g.row) {
    hipLaunchKernelGGL((k_rb_sweep4<T, SWR_TX, 1, ZX, 0>), dim3((unsigned)g.nblocks), dim3(SWR_TX / 4), 0, st, g.grids,
                       g.block0, g.ngrids, g.zlen, (const T*)xin, (T*)xout, (const T*)b, g.order);
    return;
  }
  switch (g.tile) {
    case 0: sweep_launch4t<T, ZX, 64, 8>(g, xin, xout, b, st); break;
    case 1: sweep_launch4t<T, ZX, 128, 8>(g, xin, xout, b, st); break;
    case 2: sweep_launch4t<T, ZX, 64, 16>(g, xin, xout, b, st); break;
    case 3: sweep_launch4t<T, ZX, 128, 16>(g, xin, xout, b, st); break;
    case 4: sweep_launch4t<T, ZX, 256, 8>(g, xin, xout, b, st); break;
    default: sweep_launch4t<T, ZX, 256, 12>(g, xin, xout, b, st); break;
  }
}

static bool quad_form(size_t es, const Geom& g, const void* ec) {
  // the row form (slices) of FP32 measured no faster in quads: pairs there
  return es <= 4 && !ec && g.quad && quad_on() && (es == 2 || !g.row);
}

bool sweep_starts_from_zero_ok(gd_dtype s, const Geom& g) {
  return s != GD_F64 && quad_form(s == GD_F32 ? 4 : 2, g, nullptr);
}

bool sweep_wide_tiles_ok(gd_dtype s, bool quad) { return s != GD_F64 && quad && quad_on(); }

template <typename T>
static hipError_t sweep_launch(const Geom& g, const void* xin, void* xout, const void* b, const void* ec, int pmode,
                               bool xzero, hipStream_t st) {
  if constexpr (sizeof(T) <= 4) {
    if (quad_form(sizeof(T), g, ec)) {
      if (xzero) sweep_launch4<T, true>(g, xin, xout, b, st);
      else sweep_launch4<T, false>(g, xin, xout, b, st);
      return hipSuccess;
    }
  }
  // the library's arrays are pair-aligned (g.vec); a caller's odd-width arrays are not
  if (ec) return sweep_launch3<T, true, true>(g, xin, xout, b, ec, pmode, st);
  if (g.vec) return sweep_launch3<T, false, true>(g, xin, xout, b, ec, pmode, st);
  return sweep_launch3<T, false, false>(g, xin, xout, b, ec, pmode, st);
}

hipError_t launch_rb_sweep(gd_dtype s, const Geom& g, const void* xin, void* xout, const void* b,
                           const void* ec, int pmode, hipStream_t st, bool xzero) {
  if (g.nblocks == 0) return hipSuccess;
  if (xzero && !sweep_starts_from_zero_ok(s, g)) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
#define L(T) e = sweep_launch<T>(g, xin, xout, b, ec, pmode, xzero, st)
  GD_DISPATCH_S(s, L)
#undef L
  if (e != hipSuccess) return e;
  return last();
}

}  // namespace gd
