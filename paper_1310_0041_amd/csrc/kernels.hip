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
#include "gd_kcommon.h"

namespace gd {

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
  if (G.skip) return;  // a converged grid of a batch
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
  if (G.skip) return;  // a converged grid of a batch
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
  if (G.skip) return;  // a converged grid of a batch
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

// sum over the 27 neighbours of (row of A at (i, j, k)) . x, and the diagonal,
// with fetch(qx, qy, qz) giving the current value of sample (qx, qy, qz) and
// tab(a, r, p) row r of axis a's table at sample p.
// Branch-free: a neighbour outside the grid is read at a clamped index and
// weighted by its table entry, which is 0 (the first sample has no lower and
// the last no upper coupling on every level), so all 27 reads issue at once.
// Every table-level relaxation goes through this one body, so they agree
// bit for bit whatever memory the values come from.
template <typename TB, typename F>
__device__ __forceinline__ void hyb_row_f(const HybAxes& A, const GridDesc& G, int i, int j, int k, TB&& tab,
                                          F&& fetch, double& ax, double& diag) {
  // Every multiply-add is written out: left to the compiler, the choice of
  // which product joins an add differs between call sites, and the 27-point
  // coefficients are short sums of larger products (the finite-element
  // stencils cancel), so it moved them by ~1e-11 relative.
#pragma clang fp contract(off)
  const int n[3] = {G.nx, G.ny, G.nz}, c[3] = {i, j, k};
  double m[3][3], kk[3][3];  // [axis][offset + 1]
  int q[3][3];               // clamped neighbour index [axis][offset + 1]
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int na = n[a], p = c[a];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      m[a][d] = tab(a, d, p);
      kk[a][d] = tab(a, 3 + d, p);
      q[a][d] = min(max(p + d - 1, 0), na - 1);
    }
  }
  // x-axis factors alpha M_x + w_x K_x
  double px_[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) px_[d] = __builtin_fma(A.w[0], kk[0][d], A.alpha * m[0][d]);
  // one partial sum per neighbour plane (three independent chains of nine
  // multiply-adds instead of one of 27), added in a fixed order
  double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
      const double myz = m[1][dy] * m[2][dz];
      const double yz = __builtin_fma(A.w[2], m[1][dy] * kk[2][dz], A.w[1] * (kk[1][dy] * m[2][dz]));
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const double coef = __builtin_fma(m[0][dx], yz, px_[dx] * myz);
        s[dz] = __builtin_fma(coef, fetch(q[0][dx], q[1][dy], q[2][dz]), s[dz]);
      }
    }
  ax = (s[0] + s[1]) + s[2];
  diag = __builtin_fma(m[0][1], __builtin_fma(A.w[2], m[1][1] * kk[2][1], A.w[1] * (kk[1][1] * m[2][1])),
                       px_[1] * (m[1][1] * m[2][1]));
}

// the same with the values in a level array x
template <typename S>
__device__ __forceinline__ void hyb_row(const HybAxes& A, const GridDesc& G, const S* __restrict__ x, int i, int j,
                                        int k, double& ax, double& diag) {
  const int64_t pl = (int64_t)G.px * G.ny;
  const S* base = x + G.off;
  const int n[3] = {G.nx, G.ny, G.nz};
  hyb_row_f(A, G, i, j, k, [&](int a, int r, int p) { return A.t[a][r * n[a] + p]; },
            [&](int qx, int qy, int qz) { return ld64(base + qz * pl + (int64_t)qy * G.px + qx); }, ax, diag);
}

// the Gauss-Seidel update of one sample from its row (a zero diagonal, a
// sample with no coupling at all, is set to 0)
__device__ __forceinline__ double hyb_update(double xc, double bv, double ax, double d) {
  return d != 0.0 ? xc + (bv - ax) / d : 0.0;
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
    st64(x + v, hyb_update(ld64(x + v), ld64(b + v), ax, d));
  }
}

// The same sweep in two launches, one per z-parity ck of the planes.  The
// 8-colour order (colours 0..3 on every even plane before colours 4..7 on
// the odd ones) means: an even plane reads its odd neighbour planes as they
// were before the sweep, an odd plane reads its even neighbours as they are
// after it, and within a plane the four colours (x, y parity (0,0), (1,0),
// (0,1), (1,1)) follow each other.  A block owns an HGX x HGY tile of a run
// of planes of its parity; the plane's window (tile plus a ring of HGR) and
// the two neighbour planes sit in LDS, and the four colours run in turn on
// the tile widened by 3, 2, 1 and 0 samples (a colour reads the colours
// before it up to one sample away), so the tile's new values need no other
// block.  Reads come from xin (this parity's planes, before the sweep) and
// xnb (the neighbour planes: xin for ck = 0, xout for ck = 1); the tile's
// new values go to xout.  Every update is hyb_row_f / hyb_update on the
// values the colour launches would read, so the result is theirs bit for bit.
constexpr int HGX = 64, HGY = 16, HGR = 4, HGZ = 4;  // tile, ring, planes of a parity per block
constexpr int HGWX = HGX + 2 * HGR, HGWY = HGY + 2 * HGR;
constexpr int HGT = 256;

// LDS cell of a window: the storage type, 16-bit ones as raw bits (their
// types have constructors, which __shared__ arrays may not have); values go
// in and out through st64 / ld64, so they round exactly as stores to a level
template <typename S> struct HybLds { using T = S; };
template <> struct HybLds<__half> { using T = uint16_t; };
template <> struct HybLds<__hip_bfloat16> { using T = uint16_t; };
template <typename S>
__device__ __forceinline__ double hl_ld(typename HybLds<S>::T w) {
  const S v = __builtin_bit_cast(S, w);
  return ld64(&v);
}
template <typename S>
__device__ __forceinline__ typename HybLds<S>::T hl_st(double v) {
  S t;
  st64(&t, v);
  return __builtin_bit_cast(typename HybLds<S>::T, t);
}

template <typename S>
__global__ void __launch_bounds__(HGT)
k_hyb_gs8z(GridDesc G, HybAxes A, int ck, const S* xin, const S* xnb, S* xout, const S* __restrict__ b) {
  using LT = typename HybLds<S>::T;
  __shared__ __align__(16) LT W[3][HGWY][HGWX];  // plane slots: the tile's plane and its two neighbours
  __shared__ double TXs[6][HGWX], TYs[6][HGWY];  // the x and y tables over the window
  const int nx = G.nx, ny = G.ny, nz = G.nz;
  const int ntx = (nx + HGX - 1) / HGX;
  const int x0 = (int)(blockIdx.x % ntx) * HGX, y0 = (int)(blockIdx.x / ntx) * HGY;
  const int wx0 = x0 - HGR, wy0 = y0 - HGR;  // grid coordinates of the window's corner
  const int64_t pl = (int64_t)G.px * ny;
  const int mz = (nz - ck + 1) / 2;
  const int kk0 = blockIdx.y * HGZ, kk1 = min(kk0 + HGZ, mz);
  const int tid = threadIdx.x;
  for (int m = tid; m < 6 * HGWX; m += HGT) {
    const int r = m / HGWX, w = m - r * HGWX, g = wx0 + w;
    if (g >= 0 && g < nx) TXs[r][w] = A.t[0][r * nx + g];
  }
  for (int m = tid; m < 6 * HGWY; m += HGT) {
    const int r = m / HGWY, w = m - r * HGWY, g = wy0 + w;
    if (g >= 0 && g < ny) TYs[r][w] = A.t[1][r * ny + g];
  }
  // the window of plane k of src into slot sl (samples outside the grid are never read)
  auto load = [&](int sl, const S* src, int k) {
    const LT* p = reinterpret_cast<const LT*>(src + G.off + k * pl);
    for (int m = tid; m < HGWX * HGWY; m += HGT) {
      const int wy = m / HGWX, wx = m - wy * HGWX;
      const int gx = wx0 + wx, gy = wy0 + wy;
      if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) W[sl][wy][wx] = p[(int64_t)gy * G.px + gx];
    }
  };
  int lo = 1, hi = 2;
  constexpr int cen = 0;
  for (int kk = kk0; kk < kk1; ++kk) {
    const int k = 2 * kk + ck;
    if (kk > kk0) {
      __syncthreads();  // the previous plane's reads of every slot are done
      const int t = lo;  // plane k - 1 is the previous plane's k + 1
      lo = hi;
      hi = t;
    } else if (k > 0) {
      load(lo, xnb, k - 1);
    }
    load(cen, xin, k);
    if (k + 1 < nz) load(hi, xnb, k + 1);
    __syncthreads();
    const int ls = k > 0 ? lo : cen, hs = k + 1 < nz ? hi : cen;  // clamped planes read the tile's own
    auto fetch = [&](int qx, int qy, int qz) {
      const int sl = qz == k ? cen : (qz < k ? ls : hs);
      return hl_ld<S>(W[sl][qy - wy0][qx - wx0]);
    };
    auto tab = [&](int a, int r, int p) {
      return a == 0 ? TXs[r][p - wx0] : (a == 1 ? TYs[r][p - wy0] : A.t[2][r * nz + p]);
    };
    const S* bk = b + G.off + k * pl;
#pragma unroll 1
    for (int ph = 0; ph < 4; ++ph) {
      const int pi = ph & 1, pj = ph >> 1, r = 3 - ph;  // colour (pi, pj) on the tile widened by r
      const int xa = max(x0 - r, 0), xb = min(x0 + HGX + r, nx), ya = max(y0 - r, 0), yb = min(y0 + HGY + r, ny);
      const int ia = xa + ((xa & 1) ^ pi), ja = ya + ((ya & 1) ^ pj);
      const int nu = xb > ia ? (xb - ia + 1) / 2 : 0, nv = yb > ja ? (yb - ja + 1) / 2 : 0;
      for (int m = tid; m < nu * nv; m += HGT) {
        const int v = m / nu, u = m - v * nu;
        const int i = ia + 2 * u, j = ja + 2 * v;
        double ax, d;
        hyb_row_f(A, G, i, j, k, tab, fetch, ax, d);
        LT& c = W[cen][j - wy0][i - wx0];
        c = hl_st<S>(hyb_update(hl_ld<S>(c), ld64(bk + (int64_t)j * G.px + i), ax, d));
      }
      __syncthreads();
    }
    LT* o = reinterpret_cast<LT*>(xout + G.off + k * pl);
    for (int m = tid; m < HGX * HGY; m += HGT) {
      const int ty = m / HGX, tx = m - ty * HGX;
      const int gx = x0 + tx, gy = y0 + ty;
      if (gx < nx && gy < ny) o[(int64_t)gy * G.px + gx] = W[cen][gy - wy0][gx - wx0];
    }
  }
}

// r = b - A x on a table level (all samples); with partials, the FP64 sum
// of r^2 per block (block = x + gx (y + gy z), a block spanning hz planes),
// in a fixed order
template <typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_hyb_residual(GridDesc G, HybAxes A, const S* __restrict__ x, const S* __restrict__ b, S* __restrict__ r,
               double* __restrict__ partials, int hz) {
  __shared__ double red[HBY];
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  double rr = 0.0;
  if (i < G.nx && j < G.ny) {
    const int64_t pl = (int64_t)G.px * G.ny;
    for (int k = blockIdx.z * hz; k < min((int)(blockIdx.z + 1) * hz, G.nz); ++k) {
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

// out = c0 in0 + c1 in1 (FP64 arithmetic) from the caller's arrays into a
// level array; in1 (may be NULL) has the layout of in0
template <typename Tin, typename T1, typename S>
__global__ void __launch_bounds__(HBX * HBY)
k_load_comb(GridDesc G, const Tin* __restrict__ in0, const T1* __restrict__ in1, double c0, double c1,
            S* __restrict__ out) {
  const int i = blockIdx.x * HBX + threadIdx.x, j = blockIdx.y * HBY + threadIdx.y;
  if (i >= G.nx || j >= G.ny) return;
  const int64_t pl = (int64_t)G.px * G.ny;
  for (int k = blockIdx.z * HZ; k < min((int)(blockIdx.z + 1) * HZ, G.nz); ++k) {
    const int64_t u = G.ioff + (int64_t)k * G.ipz + (int64_t)j * G.ipy + i;
    double v = c0 * in_at(in0, u);
    if (in1) v += c1 * in_at(in1, u);
    st64(out + G.off + k * pl + (int64_t)j * G.px + i, v);
  }
}

// Right-hand side of the anisotropic diffusion (Eq. (1)) in correction form
// for the planes [k0, k1) of a window of the caller's input, dense
// [planes][ny][nx] with window plane 0 at global plane z0 of an nzg-plane
// stack: b = -b_z L_z I0 (written dense, plane k0 first), the cross-slice
// term summed z-1 then z+1 as the in-core pass does; per block the FP64 sum
// of the canonical right-hand side squared, ((b_x L_x + b_y L_y) I0)^2.  L_a
// is the Neumann second difference over the whole stack.
template <typename Tin, typename S>
__global__ void __launch_bounds__(256)
k_stream_rhs(const Tin* __restrict__ I0, S* __restrict__ b, int nx, int ny, int nzg, int z0, int k0, int k1,
             double bx, double by, double bz, double* __restrict__ partials) {
  __shared__ double red[4];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63), j = blockIdx.y * 4 + (threadIdx.x >> 6);
  double s = 0.0;
  if (i < nx && j < ny) {
    const int64_t pl = (int64_t)nx * ny;
    for (int k = k0; k < k1; ++k) {
      const int64_t v = (int64_t)k * pl + (int64_t)j * nx + i;
      const double c = ld64(I0 + v);
      double lin = 0.0;
      if (i > 0) lin += bx * (c - ld64(I0 + v - 1));
      if (i + 1 < nx) lin += bx * (c - ld64(I0 + v + 1));
      if (j > 0) lin += by * (c - ld64(I0 + v - nx));
      if (j + 1 < ny) lin += by * (c - ld64(I0 + v + nx));
      s += lin * lin;
      const int gz = z0 + k;
      double lz = 0.0;
      if (gz > 0) lz += bz * (c - ld64(I0 + v - pl));
      if (gz + 1 < nzg) lz += bz * (c - ld64(I0 + v + pl));
      Ty<S>::st(b + (int64_t)(k - k0) * pl + (int64_t)j * nx + i, (typename Ty<S>::C)(0.0 - lz));
    }
  }
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.y * gridDim.x + blockIdx.x] = tot;
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
// ============================================================ launchers

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

hipError_t launch_hyb_gs8z(gd_dtype s, const GridDesc& G, const HybTables& T, const void* xin, void* xout,
                           const void* b, hipStream_t st) {
  if ((int64_t)G.nx * G.ny * G.nz == 0) return hipSuccess;
  HybAxes A{{T.t[0], T.t[1], T.t[2]}, T.alpha, {T.w[0], T.w[1], T.w[2]}};
  const int64_t tiles = (int64_t)((G.nx + HGX - 1) / HGX) * ((G.ny + HGY - 1) / HGY);
  for (int ck = 0; ck < 2; ++ck) {
    const int64_t mz = (G.nz - ck + 1) / 2;
    if (mz == 0) continue;
    const dim3 grid((unsigned)tiles, (unsigned)((mz + HGZ - 1) / HGZ));
    // even planes read their neighbours before the sweep (xin), odd ones after it (xout)
    const void* nb = ck == 0 ? xin : xout;
#define L(TT) hipLaunchKernelGGL(k_hyb_gs8z<TT>, grid, dim3(HGT), 0, st, G, A, ck, (const TT*)xin, (const TT*)nb, \
                                 (TT*)xout, (const TT*)b)
    GD_DISPATCH_S(s, L)
#undef L
  }
  return last();
}

int64_t hyb_residual_blocks(const GridDesc& G, bool per_plane) {
  const dim3 g = hyb_grid(G.nx, G.ny, G.nz);
  return per_plane ? (int64_t)g.x * g.y * G.nz : (int64_t)g.x * g.y * g.z;
}

hipError_t launch_hyb_residual(gd_dtype s, const GridDesc& G, const HybTables& T, const void* x, const void* b,
                               void* r, hipStream_t st, double* partials, bool per_plane) {
  HybAxes A{{T.t[0], T.t[1], T.t[2]}, T.alpha, {T.w[0], T.w[1], T.w[2]}};
  const int hz = per_plane ? 1 : HZ;
  const dim3 grid((unsigned)((G.nx + HBX - 1) / HBX), (unsigned)((G.ny + HBY - 1) / HBY), (unsigned)((G.nz + hz - 1) / hz));
#define L(TT) hipLaunchKernelGGL(k_hyb_residual<TT>, grid, dim3(HBX, HBY), 0, st, G, A, (const TT*)x, (const TT*)b, \
                                 (TT*)r, partials, hz)
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

template <typename TI, typename T1>
static hipError_t load_comb_launch(gd_dtype s, const GridDesc& G, const void* in0, const void* in1, double c0,
                                   double c1, void* out, hipStream_t st) {
#define L(TT) hipLaunchKernelGGL((k_load_comb<TI, T1, TT>), hyb_grid(G.nx, G.ny, G.nz), dim3(HBX, HBY), 0, st, G, \
                                 (const TI*)in0, (const T1*)in1, c0, c1, (TT*)out)
  GD_DISPATCH_S(s, L)
#undef L
  return hipSuccess;
}

hipError_t launch_load_comb(gd_dtype tin, gd_dtype t1, gd_dtype s, const GridDesc& G, const void* in0,
                            const void* in1, double c0, double c1, void* out, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (!in1 || t1 == tin) {
#define L(TI) e = load_comb_launch<TI, TI>(s, G, in0, in1, c0, c1, out, st)
    GD_DISPATCH_S(tin, L)
#undef L
  } else if (t1 == GD_F64) {
#define L(TI) e = load_comb_launch<TI, double>(s, G, in0, in1, c0, c1, out, st)
    GD_DISPATCH_S(tin, L)
#undef L
  } else if (t1 == GD_F32) {
#define L(TI) e = load_comb_launch<TI, float>(s, G, in0, in1, c0, c1, out, st)
    GD_DISPATCH_S(tin, L)
#undef L
  } else {
    return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return last();
}

template <typename TI>
static hipError_t stream_rhs_launch(gd_dtype s, const void* I0, void* b, int nx, int ny, int nzg, int z0, int k0,
                                    int k1, double bx, double by, double bz, double* partials, hipStream_t st) {
  const dim3 grid((unsigned)((nx + 63) / 64), (unsigned)((ny + 3) / 4));
#define L(TT) hipLaunchKernelGGL((k_stream_rhs<TI, TT>), grid, dim3(256), 0, st, (const TI*)I0, (TT*)b, nx, ny, nzg, \
                                 z0, k0, k1, bx, by, bz, partials)
  GD_DISPATCH_S(s, L)
#undef L
  return hipSuccess;
}

int64_t stream_rhs_blocks(int64_t nx, int64_t ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }

hipError_t launch_stream_rhs(gd_dtype tin, gd_dtype s, const void* I0, void* b, int nx, int ny, int nzg, int z0,
                             int k0, int k1, double bx, double by, double bz, double* partials, hipStream_t st) {
  hipError_t e = hipSuccess;
#define L(TI) e = stream_rhs_launch<TI>(s, I0, b, nx, ny, nzg, z0, k0, k1, bx, by, bz, partials, st)
  GD_DISPATCH_S(tin, L)
#undef L
  if (e != hipSuccess) return e;
  return last();
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
