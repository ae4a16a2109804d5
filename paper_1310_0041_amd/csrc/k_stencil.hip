// gfx950 finest-level passes of the anisotropic-diffusion (Eq. (1)) and
// per-slice screened-Poisson (Eq. (2)) solves of Kazhdan et al.,
// "Gradient-Domain Processing for Large EM Image Stacks": correction-form
// right-hand side, FP64 canonical residual and refinement update, gauge
// sums and output.  Layout conventions as in kernels.hip.
#include "gd_kcommon.h"

namespace gd {

// ------------------------------------------- finest level of AD / SP (Eq. 1, 2)
//
// Canonical system of both phases: A = alpha + w_x L_x + w_y L_y + w_z L_z,
// b = alpha I1 + (w_x L_x + w_y L_y) I0 (AD: alpha = 0; SP: w_z = 0).  In
// the grid description the caller's y axis is the grid's y axis for a stack
// and its z axis for a slice (ny = 1); the in-slice weights are then w_x and
// w_z.  GridDesc::zin flags the slice form.
// The plain solver iterates on the correction E = x - I0, whose right-hand
// side is b - A I0 = alpha (I1 - I0) - (cross-slice part of A) I0.


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
// x64 - I0 in MODE 1, x64 + s e - I0 in MODE 2, I0 + s e - I0 in MODE 3 (the
// first refinement update, from x64 = I0 without reading it), where the refinement's
// update x64 + s e is also written to x64_out, s = e_scale[grid]) the I0
// terms of b and A x cancel except across slices:
//   r = alpha (I1 - I0 - F) - (w_x L_x + w_y L_y + w_z L_z) F - [stack] w_z L_z I0
//   ||r||^2 per block; r * inv_scale stored when rout is set.
// L_a v is the Neumann second difference sum over existing neighbours of
// (v_c - v_n).  Row tiles (TY == 1) serve grids with ny == 1.
// I1 may have a wider type T1 than I0 (the FP64 result of a refined first
// phase feeding the second).
template <typename Tin, typename T1, typename S, int TX, int TY, int KIND, int MODE>
__global__ void __launch_bounds__(TX * TY / 2)
k_corr_stencil(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
               const Tin* __restrict__ I0, const T1* __restrict__ I1, const S* __restrict__ E,
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
  constexpr bool UPD = MODE >= 2;  // the refinement update x64' = (x64 or I0) + s e
  __shared__ double X[3][HY][HX];
  __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];
  __shared__ double red2[NT / 64 > 0 ? NT / 64 : 1];

  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false);
  const GridDesc& G = grids[t.g];
  if (G.skip) return;  // a converged grid of a batch
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const bool slice = G.zin != 0;
  const double alpha = G.alpha, wx = G.wx, wy = ROW ? 0.0 : G.wy, wz = G.wz;
  const bool cross = !slice && wz != 0.0;  // the stack's cross-slice term of I0
  const int64_t pl = (int64_t)px * ny;
  const Tin* I0g = I0 + G.ioff;
  const T1* I1g = (I1 && alpha != 0.0) ? I1 + G.ioff : nullptr;
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
  // x and in-plane y weights of the pair's cells (0 where the neighbour is
  // outside the grid)
  const double wlA = o0 ? wx : 0.0, wrA = vB ? wx : 0.0, wlB = wx, wrB = o1 ? wx : 0.0;
  const double wu = up ? wy : 0.0, wd = dn ? wy : 0.0;

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
  using FS = std::conditional_t<KIND == 0, Tin, std::conditional_t<MODE == 0 || MODE == 3, S, double>>;
  // Loads of a plane sit in one of two slots: a plane is fetched two planes
  // ahead of its use, and the loop is unrolled by two so that no slot is
  // copied (a copy would make the wave wait for the newest loads).
  struct Pre {
    Raw2<FS> rf;
    Raw2<Tin> ri;
    Raw2<S> re;  // MODE 2, 3: the correction e
    Raw<FS> rh[NHR];
    Raw<Tin> rhi[NHR];
    Raw<S> rhe[NHR];
    Raw2<T1> r1;  // the I1 pair (alpha != 0)
  };
  const double es = UPD ? e_scale[t.g] : 0.0;
  // loads from clamped addresses without branches around them (masked in stash)
  auto fetch = [&](int q, Pre& o) {
    const int qc = min(max(q, 0), nz - 1);
    const Tin* I0q = I0g + qc * G.ipz;
    const int64_t po = qc * pl;
    const int64_t oo = vA ? own : 0, ou = vA ? ownu : 0;
    if (KIND == 0) {
      ld_raw2(reinterpret_cast<const FS*>(I0q) + ou, ivec, vB, o.rf);
    } else {
      ld_raw2(I0q + ou, ivec, vB, o.ri);
      if (MODE == 0) {
        ld_raw2(reinterpret_cast<const FS*>(Eg) + po + oo, true, true, o.rf);
      } else if (MODE == 3) {
        ld_raw2(Eg + po + oo, true, true, o.re);
      } else {
        ld_raw2(reinterpret_cast<const FS*>(xg) + po + oo, true, true, o.rf);
        if (MODE == 2) ld_raw2(Eg + po + oo, true, true, o.re);
      }
    }
#pragma unroll
    for (int k = 0; k < NHR; ++k) {
      if (KIND == 0) ld_raw(reinterpret_cast<const FS*>(I0q) + hu[k], o.rh[k]);
      else if (MODE == 0) ld_raw(reinterpret_cast<const FS*>(Eg) + po + hg[k], o.rh[k]);
      else if (MODE == 3) {
        ld_raw(I0q + hu[k], o.rhi[k]);
        ld_raw(Eg + po + hg[k], o.rhe[k]);
      } else {
        ld_raw(reinterpret_cast<const FS*>(xg) + po + hg[k], o.rh[k]);
        ld_raw(I0q + hu[k], o.rhi[k]);
        if (MODE == 2) ld_raw(Eg + po + hg[k], o.rhe[k]);
      }
    }
    // I1 (raw, clamped; used only for planes in [q0, q1) with vA / vB)
    if (I1g) ld_raw2(I1g + qc * G.ipz + ou, ivec, vB, o.r1);
  };
  // convert a slot: F pair (fa, fb), I0 pair (ia, ib), I1 pair (ja, jb);
  // store F's plane in LDS
  double fa = 0, fb = 0, ia = 0, ib = 0, ja = 0, jb = 0;
  auto stash = [&](int q, const Pre& o) {
    const bool okq = q >= 0 && q < nz, mA = okq && vA, mB = okq && vB;
    if (KIND == 1) {
      ia = mA ? raw_a(o.ri) : 0.0;
      ib = mB ? raw_b(o.ri) : 0.0;
    }
    ja = I1g ? raw_a(o.r1) : 0.0;
    jb = I1g ? raw_b(o.r1) : 0.0;
    if (MODE == 3) {  // x64 = I0 before the first update
      fa = ia;
      fb = ib;
    } else {
      fa = mA ? raw_a(o.rf) : 0.0;
      fb = mB ? raw_b(o.rf) : 0.0;
    }
    if (KIND == 1 && UPD) {  // refinement update x64 + s e, written by the cell's owner
      // one fused multiply-add, as for the halo copies of the same cell
      // (other tiles must see the value this tile stores)
      fa = mA ? __builtin_fma(es, raw_a(o.re), fa) : fa;
      fb = mB ? __builtin_fma(es, raw_b(o.re), fb) : fb;
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
        double v = MODE == 3 ? raw_d(o.rhi[k]) : raw_d(o.rh[k]);
        if (KIND == 1 && UPD) v = __builtin_fma(es, raw_d(o.rhe[k]), v);
        if (KIND == 1 && MODE >= 1) v -= raw_d(o.rhi[k]);
        P[hoff[k]] = (okq && hv[k]) ? v : 0.0;
      }
  };

  // registers: F and I0 at k - 1 (m), k (c), k + 1 (p); I1 at k (c) and k + 1 (p)
  double fma_ = 0, fmb = 0, fca, fcb, fpa, fpb, ima = 0, imb = 0, ica = 0, icb = 0, ipa = 0, ipb = 0;
  double jca = 0, jcb = 0, jpa = 0, jpb = 0;
  Pre A, B;
  fetch(q0 - 1, A);
  stash(q0 - 1, A);  // plane q0 - 1 goes to the ring slot of q0 + 2, rewritten before it is read
  fma_ = fa; fmb = fb; ima = ia; imb = ib;
  fetch(q0, A);
  stash(q0, A);
  fca = fa; fcb = fb; ica = ia; icb = ib; jca = ja; jcb = jb;
  fetch(q0 + 1, A);
  fetch(q0 + 2, B);
  double nrm = 0.0, nrm2 = 0.0;  // KIND 0: sum b^2 (canonical) and sum b_corr^2
  // plane k: slot o holds plane k + 1, refilled with plane k + 3
  auto iter = [&](int k, Pre& o) {
    stash(k + 1, o);
    fpa = fa; fpb = fb; ipa = ia; ipb = ib; jpa = ja; jpb = jb;
    fetch(k + 3, o);
    __syncthreads();
    const double v1a = jca, v1b = jcb;
    const double* P = &X[k % 3][0][0];
    // every term is computed: a neighbour outside the grid has weight 0 and
    // a finite (zero) value in LDS, so no branch or mask is needed until the
    // norm and the stores
    const double wzm = k > 0 ? wz : 0.0, wzp = k < nz - 1 ? wz : 0.0;
    // in-plane and z second differences of F (left, right, up, down, z-1,
    // z+1); I0's z term for the stack
    auto lap = [&](double c, double wl, double l, double wr, double rr, double u_, double d_, double zm_,
                   double zp_) {
      double s2 = 0.0;
      s2 += wl * (c - l);
      s2 += wr * (c - rr);
      if (!ROW) {
        s2 += wu * (c - u_);
        s2 += wd * (c - d_);
      }
      s2 += wzm * (c - zm_);
      s2 += wzp * (c - zp_);
      return s2;
    };
    const int lo_ = ly * HX + lx;
    const double uA = ROW ? 0.0 : P[lo_ - HX], uB = ROW ? 0.0 : P[lo_ - HX + 1];
    const double dA = ROW ? 0.0 : P[lo_ + HX], dB = ROW ? 0.0 : P[lo_ + HX + 1];
    const double lA = P[lo_ - 1], rB = P[lo_ + 2];
    double ra, rb;
    {
      const double c = fca;
      const double lf = lap(c, wlA, lA, wrA, fcb, uA, dA, fma_, fpa);
      double lzI = 0.0;  // w_z L_z I0 (stack only)
      if (cross) {
        const double i0 = KIND == 0 ? fca : ica, im = KIND == 0 ? fma_ : ima, ip = KIND == 0 ? fpa : ipa;
        lzI += wzm * (i0 - im);
        lzI += wzp * (i0 - ip);
      }
      if (KIND == 0) {
        const double lin = lf - (cross ? lzI : 0.0);  // canonical part of L I0
        const double bcan = alpha * v1a + lin;
        nrm += vA ? bcan * bcan : 0.0;
        ra = alpha * (v1a - c) - lzI;
        nrm2 += vA ? ra * ra : 0.0;
      } else {
        ra = alpha * (v1a - ica - c) - lf - lzI;
        nrm += vA ? ra * ra : 0.0;
      }
    }
    {
      const double c = fcb;
      const double lf = lap(c, wlB, fca, wrB, rB, uB, dB, fmb, fpb);
      double lzI = 0.0;
      if (cross) {
        const double i0 = KIND == 0 ? fcb : icb, im = KIND == 0 ? fmb : imb, ip = KIND == 0 ? fpb : ipb;
        lzI += wzm * (i0 - im);
        lzI += wzp * (i0 - ip);
      }
      if (KIND == 0) {
        const double lin = lf - (cross ? lzI : 0.0);
        const double bcan = alpha * v1b + lin;
        nrm += vB ? bcan * bcan : 0.0;
        rb = alpha * (v1b - c) - lzI;
        nrm2 += vB ? rb * rb : 0.0;
      } else {
        rb = alpha * (v1b - icb - c) - lf - lzI;
        nrm += vB ? rb * rb : 0.0;
      }
    }
    if (vA) {
      const int64_t v = G.off + k * pl + own;
      if (KIND == 0) {
        const double sc = inv_scale ? inv_scale[t.g] : 1.0;  // a power of two (exact)
        if (out0) st2(out0 + v, vec, vB, (typename Ty<S>::C)(ra * sc), (typename Ty<S>::C)(rb * sc));
        if (out1) st2(out1 + v, vec, vB, (typename Ty<S>::C)0, (typename Ty<S>::C)0);
      } else if (out0) {
        const double sc = inv_scale[t.g];
        st2(out0 + v, vec, vB, (typename Ty<S>::C)(ra * sc), (typename Ty<S>::C)(rb * sc));
      }
    }
    fma_ = fca; fmb = fcb; fca = fpa; fcb = fpb;
    ima = ica; imb = icb; ica = ipa; icb = ipb;
    jca = jpa; jcb = jpb;
  };
  int k = q0;
  for (; k + 1 < q1; k += 2) {
    iter(k, A);
    iter(k + 1, B);
  }
  if (k < q1) iter(k, A);
  if (partials) {
    const double sm = block_sum(nrm, red);
    if (KIND == 0) {
      const double sm2 = block_sum(nrm2, red2);
      if (threadIdx.x == 0) {
        partials[2 * t.bid] = sm;
        partials[2 * t.bid + 1] = sm2;
      }
    } else if (threadIdx.x == 0) {
      partials[t.bid] = sm;
    }
  }
}

// ------------------------------------- quad form of the same passes
//
// The passes above on 3-D grids with four consecutive x cells per thread,
// for caller arrays whose offset and pitches are multiples of four (one
// aligned access per quad) and the library's level arrays.  Every cell is
// computed by the expressions of the pair form in the same order, so both
// forms store the same values; the per-block norm partials are the same
// terms summed in another order.  The LDS plane is TX + 8 wide with the tile
// at x offset 4 (aligned quads): the halo is the full quad rows above and
// below the tile and one quad on each side of its rows.

template <typename T> struct Q4 {  // four consecutive raw values
  using W = std::conditional_t<sizeof(T) == 8, double2, std::conditional_t<sizeof(T) == 4, float4, uint2>>;
  W w[sizeof(T) == 8 ? 2 : 1];
};
template <typename T> __device__ __forceinline__ void ld_q4(const T* p, Q4<T>& r) {
  if constexpr (sizeof(T) == 8) {
    r.w[0] = reinterpret_cast<const double2*>(p)[0];
    r.w[1] = reinterpret_cast<const double2*>(p)[1];
  } else {
    r.w[0] = *reinterpret_cast<const typename Q4<T>::W*>(p);
  }
}
template <typename T> __device__ __forceinline__ double q4_d(const Q4<T>& r, int i) {
  if constexpr (sizeof(T) == 8) {
    const double2 v = r.w[i >> 1];
    return (i & 1) ? v.y : v.x;
  } else if constexpr (sizeof(T) == 4) {
    const float4 v = r.w[0];
    return (double)(i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w);
  } else {
    const uint32_t v = (i < 2) ? r.w[0].x : r.w[0].y;
    return from_bits16<T>((i & 1) ? (v >> 16) : (v & 0xffffu));
  }
}
// four values of the compute type Ty<S>::C into an aligned quad of S
template <typename S, typename C>
__device__ __forceinline__ void st_q4(S* p, C a, C b, C c, C d) {
  if constexpr (sizeof(S) == 8) {
    reinterpret_cast<double2*>(p)[0] = make_double2((double)a, (double)b);
    reinterpret_cast<double2*>(p)[1] = make_double2((double)c, (double)d);
  } else if constexpr (sizeof(S) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4((float)a, (float)b, (float)c, (float)d);
  } else {
    S h[4];
    Ty<S>::st(&h[0], a);
    Ty<S>::st(&h[1], b);
    Ty<S>::st(&h[2], c);
    Ty<S>::st(&h[3], d);
    uint16_t u[4];
    __builtin_memcpy(u, h, 8);
    *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)u[0] | ((uint32_t)u[1] << 16),
                                              (uint32_t)u[2] | ((uint32_t)u[3] << 16));
  }
}

template <typename Tin, typename S, int TX, int TY, int KIND, int MODE>
__global__ void __launch_bounds__(TX * TY / 4)
k_corr_stencil4(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen,
                const Tin* __restrict__ I0, const Tin* __restrict__ I1, const S* __restrict__ E,
                const double* __restrict__ x64, S* __restrict__ out0, S* __restrict__ out1,
                const double* __restrict__ inv_scale, double* __restrict__ partials,
                double* __restrict__ x64_out, const double* __restrict__ e_scale) {
  constexpr int NT = TX * TY / 4, QPR = TX / 4;
  constexpr int XO = 4, HX = TX + 8, HY = TY + 2;
  constexpr int QR = TX / 4 + 2;        // quads of a full halo row
  constexpr int NHQ = 2 * QR + 2 * TY;  // halo quads per plane
  constexpr int NHQR = (NHQ + NT - 1) / NT;
  static_assert(MODE < 2 || KIND == 1, "the refinement update belongs to the residual pass");
  static_assert(NT % 64 == 0, "whole waves");
  constexpr bool UPD = MODE >= 2;
  using C = typename Ty<S>::C;
  __shared__ __align__(16) double X[3][HY * HX];
  __shared__ double red[NT / 64];
  __shared__ double red2[NT / 64];

  const Tile t = decode_tile(grids, block0, ngrids, zlen, TX, TY, false);
  const GridDesc& G = grids[t.g];
  if (G.skip) return;  // a converged grid of a batch
  const int nx = G.nx, ny = G.ny, nz = G.nz, px = G.px;
  const double alpha = G.alpha, wx = G.wx, wy = G.wy, wz = G.wz;
  const bool cross = G.zin == 0 && wz != 0.0;  // the stack's cross-slice term of I0
  const int64_t pl = (int64_t)px * ny;
  const Tin* I0g = I0 + G.ioff;
  const Tin* I1g = (I1 && alpha != 0.0) ? I1 + G.ioff : nullptr;
  const S* Eg = E + G.off;
  const double* xg = x64 + G.off;
  const int tid = threadIdx.x;
  const int x0 = t.x0, y0 = t.y0, q0 = t.z0, q1 = t.z1;
  const int tyl = tid / QPR, qxl = tid - tyl * QPR;
  const int gx = x0 + 4 * qxl, gy = y0 + tyl;
  const bool rowok = gy < ny;
  bool v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = rowok && gx + j < nx;
  const int lo = (1 + tyl) * HX + XO + 4 * qxl;
  const int64_t own = (int64_t)gy * px + gx, ownu = (int64_t)gy * G.ipy + gx;
  // x and in-plane y weights of the quad's cells (0 where the neighbour is
  // outside the grid), as the pair form gives them
  double wl[4], wr[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    wl[j] = gx + j > 0 ? wx : 0.0;
    wr[j] = gx + j + 1 < nx ? wx : 0.0;
  }
  const double wu = gy > 0 ? wy : 0.0, wd = gy + 1 < ny ? wy : 0.0;

  int hoff[NHQR], hx0[NHQR];
  int64_t hg[NHQR], hu[NHQR];
  bool hs[NHQR], hq[NHQR];
#pragma unroll
  for (int k = 0; k < NHQR; ++k) {
    const int h = tid + NT * k;
    int hy = 0, hx = 0;
    if (h < QR) {
      hx = 4 * h;
    } else if (h < 2 * QR) {
      hy = HY - 1;
      hx = 4 * (h - QR);
    } else {
      const int m = h - 2 * QR;
      hy = 1 + (m >> 1);
      hx = (m & 1) ? TX + XO : 0;
    }
    const int cx = x0 - XO + hx, cy = y0 - 1 + hy;  // cx is a multiple of 4
    hs[k] = h < NHQ;
    hq[k] = hs[k] && cx >= 0 && cx < nx && cy >= 0 && cy < ny;
    hoff[k] = hy * HX + hx;
    hg[k] = hq[k] ? (int64_t)cy * px + cx : 0;
    hu[k] = hq[k] ? (int64_t)cy * G.ipy + cx : 0;
    hx0[k] = cx;
  }
  using FS = std::conditional_t<KIND == 0, Tin, std::conditional_t<MODE == 0 || MODE == 3, S, double>>;
  struct Pre {
    Q4<FS> rf;
    Q4<Tin> ri;
    Q4<S> re;  // MODE 2, 3: the correction e
    Q4<FS> rh[NHQR];
    Q4<Tin> rhi[NHQR];
    Q4<S> rhe[NHQR];
    Q4<Tin> r1;  // I1 (alpha != 0)
  };
  const double es = UPD ? e_scale[t.g] : 0.0;
  // loads from clamped addresses without branches around them (masked in stash)
  auto fetch = [&](int q, Pre& o) {
    const int qc = min(max(q, 0), nz - 1);
    const Tin* I0q = I0g + qc * G.ipz;
    const int64_t po = qc * pl;
    const int64_t oo = v[0] ? own : 0, ou = v[0] ? ownu : 0;
    if (KIND == 0) {
      ld_q4(reinterpret_cast<const FS*>(I0q) + ou, o.rf);
    } else {
      ld_q4(I0q + ou, o.ri);
      if (MODE == 0) {
        ld_q4(reinterpret_cast<const FS*>(Eg) + po + oo, o.rf);
      } else if (MODE == 3) {
        ld_q4(Eg + po + oo, o.re);
      } else {
        ld_q4(reinterpret_cast<const FS*>(xg) + po + oo, o.rf);
        if (MODE == 2) ld_q4(Eg + po + oo, o.re);
      }
    }
#pragma unroll
    for (int k = 0; k < NHQR; ++k) {
      if (KIND == 0) ld_q4(reinterpret_cast<const FS*>(I0q) + hu[k], o.rh[k]);
      else if (MODE == 0) ld_q4(reinterpret_cast<const FS*>(Eg) + po + hg[k], o.rh[k]);
      else if (MODE == 3) {
        ld_q4(I0q + hu[k], o.rhi[k]);
        ld_q4(Eg + po + hg[k], o.rhe[k]);
      } else {
        ld_q4(reinterpret_cast<const FS*>(xg) + po + hg[k], o.rh[k]);
        ld_q4(I0q + hu[k], o.rhi[k]);
        if (MODE == 2) ld_q4(Eg + po + hg[k], o.rhe[k]);
      }
    }
    if (I1g) ld_q4(I1g + qc * G.ipz + ou, o.r1);
  };
  // convert a slot: F (f), I0 (i), I1 (jv) of the quad; store F's plane in LDS
  double f[4], i4[4], jv[4];
  auto stash = [&](int q, const Pre& o) {
    const bool okq = q >= 0 && q < nz;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool m = okq && v[j];
      i4[j] = (KIND == 1 && m) ? q4_d(o.ri, j) : 0.0;
      jv[j] = I1g ? q4_d(o.r1, j) : 0.0;
      if (MODE == 3) f[j] = i4[j];  // x64 = I0 before the first update
      else f[j] = m ? q4_d(o.rf, j) : 0.0;
      if (KIND == 1 && UPD) f[j] = m ? __builtin_fma(es, q4_d(o.re, j), f[j]) : f[j];  // as for the halo copies
    }
    if (KIND == 1 && UPD && v[0] && q >= q0 && q < q1) {
      double* xo = x64_out + G.off + q * pl + own;
      reinterpret_cast<double2*>(xo)[0] = make_double2(f[0], f[1]);
      reinterpret_cast<double2*>(xo)[1] = make_double2(f[2], f[3]);
    }
    if (KIND == 1 && MODE >= 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) f[j] -= i4[j];
    }
    double* P = X[((q % 3) + 3) % 3];
    reinterpret_cast<double2*>(P + lo)[0] = make_double2(f[0], f[1]);
    reinterpret_cast<double2*>(P + lo)[1] = make_double2(f[2], f[3]);
#pragma unroll
    for (int k = 0; k < NHQR; ++k)
      if (hs[k]) {
        double hv4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          double vv = MODE == 3 ? q4_d(o.rhi[k], j) : q4_d(o.rh[k], j);
          if (KIND == 1 && UPD) vv = __builtin_fma(es, q4_d(o.rhe[k], j), vv);
          if (KIND == 1 && MODE >= 1) vv -= q4_d(o.rhi[k], j);
          hv4[j] = (okq && hq[k] && hx0[k] + j < nx) ? vv : 0.0;
        }
        reinterpret_cast<double2*>(P + hoff[k])[0] = make_double2(hv4[0], hv4[1]);
        reinterpret_cast<double2*>(P + hoff[k])[1] = make_double2(hv4[2], hv4[3]);
      }
  };

  // registers: F and I0 at k - 1 (m), k (c), k + 1 (p); I1 at k (c) and k + 1 (p)
  double fm[4], fc[4], fp[4], im[4], ic[4], ip[4], jc[4], jp[4];
  Pre A, B;
  fetch(q0 - 1, A);
  stash(q0 - 1, A);  // plane q0 - 1 goes to the ring slot of q0 + 2, rewritten before it is read
#pragma unroll
  for (int j = 0; j < 4; ++j) { fm[j] = f[j]; im[j] = i4[j]; }
  fetch(q0, A);
  stash(q0, A);
#pragma unroll
  for (int j = 0; j < 4; ++j) { fc[j] = f[j]; ic[j] = i4[j]; jc[j] = jv[j]; }
  fetch(q0 + 1, A);
  fetch(q0 + 2, B);
  double nrm = 0.0, nrm2 = 0.0;  // KIND 0: sum b^2 (canonical) and sum b_corr^2
  // plane k: slot o holds plane k + 1, refilled with plane k + 3
  auto iter = [&](int k, Pre& o) {
    stash(k + 1, o);
#pragma unroll
    for (int j = 0; j < 4; ++j) { fp[j] = f[j]; ip[j] = i4[j]; jp[j] = jv[j]; }
    fetch(k + 3, o);
    __syncthreads();
    const double* P = X[k % 3];
    const double wzm = k > 0 ? wz : 0.0, wzp = k < nz - 1 ? wz : 0.0;
    auto lap = [&](double c, double wl_, double l, double wr_, double rr, double u_, double d_, double zm_,
                   double zp_) {
      double s2 = 0.0;
      s2 += wl_ * (c - l);
      s2 += wr_ * (c - rr);
      s2 += wu * (c - u_);
      s2 += wd * (c - d_);
      s2 += wzm * (c - zm_);
      s2 += wzp * (c - zp_);
      return s2;
    };
    const double2 u01 = reinterpret_cast<const double2*>(P + lo - HX)[0];
    const double2 u23 = reinterpret_cast<const double2*>(P + lo - HX)[1];
    const double2 d01 = reinterpret_cast<const double2*>(P + lo + HX)[0];
    const double2 d23 = reinterpret_cast<const double2*>(P + lo + HX)[1];
    const double uu[4] = {u01.x, u01.y, u23.x, u23.y}, dd[4] = {d01.x, d01.y, d23.x, d23.y};
    const double lft = P[lo - 1], rgt = P[lo + 4];
    double r4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double c = fc[j];
      const double l = j == 0 ? lft : fc[j - 1], rr = j == 3 ? rgt : fc[j + 1];
      const double lf = lap(c, wl[j], l, wr[j], rr, uu[j], dd[j], fm[j], fp[j]);
      double lzI = 0.0;  // w_z L_z I0 (stack only)
      if (cross) {
        const double i0 = KIND == 0 ? fc[j] : ic[j], im_ = KIND == 0 ? fm[j] : im[j], ip_ = KIND == 0 ? fp[j] : ip[j];
        lzI += wzm * (i0 - im_);
        lzI += wzp * (i0 - ip_);
      }
      if (KIND == 0) {
        const double lin = lf - (cross ? lzI : 0.0);  // canonical part of L I0
        const double bcan = alpha * jc[j] + lin;
        nrm += v[j] ? bcan * bcan : 0.0;
        r4[j] = alpha * (jc[j] - c) - lzI;
        nrm2 += v[j] ? r4[j] * r4[j] : 0.0;
      } else {
        r4[j] = alpha * (jc[j] - ic[j] - c) - lf - lzI;
        nrm += v[j] ? r4[j] * r4[j] : 0.0;
      }
    }
    if (v[0]) {
      const int64_t vo = G.off + k * pl + own;
      if (KIND == 0) {
        const double sc = inv_scale ? inv_scale[t.g] : 1.0;  // a power of two (exact)
        if (out0) st_q4<S, C>(out0 + vo, (C)(r4[0] * sc), (C)(r4[1] * sc), (C)(r4[2] * sc), (C)(r4[3] * sc));
        if (out1) st_q4<S, C>(out1 + vo, (C)0, (C)0, (C)0, (C)0);
      } else if (out0) {
        const double sc = inv_scale[t.g];
        st_q4<S, C>(out0 + vo, (C)(r4[0] * sc), (C)(r4[1] * sc), (C)(r4[2] * sc), (C)(r4[3] * sc));
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      fm[j] = fc[j]; fc[j] = fp[j];
      im[j] = ic[j]; ic[j] = ip[j];
      jc[j] = jp[j];
    }
  };
  int k = q0;
  for (; k + 1 < q1; k += 2) {
    iter(k, A);
    iter(k + 1, B);
  }
  if (k < q1) iter(k, A);
  if (partials) {
    const double sm = block_sum(nrm, red);
    if (KIND == 0) {
      const double sm2 = block_sum(nrm2, red2);
      if (threadIdx.x == 0) {
        partials[2 * t.bid] = sm;
        partials[2 * t.bid + 1] = sm2;
      }
    } else if (threadIdx.x == 0) {
      partials[t.bid] = sm;
    }
  }
}

template <typename Tin, typename S, int MODE>
__global__ void __launch_bounds__(256)
k_sum_shift(const GridDesc* __restrict__ grids, const int64_t* __restrict__ block0, int ngrids, int zlen, int etx,
            const Tin* __restrict__ I0, const S* __restrict__ E, const S* __restrict__ E2,
            const double* __restrict__ x64, double* __restrict__ partials) {
  __shared__ double red[4];
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  if (G.alt) E = E2;  // the grid's correction is in the level's other buffer
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
           const Tin* __restrict__ I0, const S* __restrict__ E, const S* __restrict__ E2,
           const double* __restrict__ x64, const double* __restrict__ shift, Tout* __restrict__ out) {
  const Tile t = decode_tile(grids, block0, ngrids, zlen, etx, 256 / etx, false);
  const GridDesc& G = grids[t.g];
  if (G.alt) E = E2;  // the grid's correction is in the level's other buffer
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


// ============================================================ launchers

template <typename TI, typename T1, typename T, int KIND, int MODE>
static hipError_t corr_stencil_launch2(const Geom& g, const void* I0, const void* I1, const void* E,
                                       const double* x64, void* o0, void* o1, const double* inv_scale,
                                       double* partials, double* x64o, const double* escale, hipStream_t st) {
  if (g.stencil4) {  // quad form: 3-D grids, I1 of I0's type, the quad table of the level
    if constexpr (std::is_same_v<TI, T1>) {
      if (g.row) return hipErrorInvalidValue;
#define CS4(TX, TY)                                                                                             \
  hipLaunchKernelGGL((k_corr_stencil4<TI, T, TX, TY, KIND, MODE>), dim3((unsigned)g.nblocks), dim3(TX * TY / 4), 0, \
                     st, g.grids, g.block0, g.ngrids, g.zlen, (const TI*)I0, (const TI*)I1, (const T*)E, x64,     \
                     (T*)o0, (T*)o1, inv_scale, partials, x64o, escale)
      if (g.tile == 0) CS4(128, 8);
      else CS4(64, 16);
#undef CS4
      return hipSuccess;
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (g.row) {
    hipLaunchKernelGGL((k_corr_stencil<TI, T1, T, SWR_TX, 1, KIND, MODE>), dim3((unsigned)g.nblocks),
                       dim3(SWR_TX / 2), 0, st, g.grids, g.block0, g.ngrids, g.zlen, (const TI*)I0, (const T1*)I1,
                       (const T*)E, x64, (T*)o0, (T*)o1, inv_scale, partials, x64o, escale);
  } else if constexpr (std::is_same_v<TI, T1>) {
    hipLaunchKernelGGL((k_corr_stencil<TI, TI, T, SW_TX, SW_TY, KIND, MODE>), dim3((unsigned)g.nblocks),
                       dim3(SW_TX * SW_TY / 2), 0, st, g.grids, g.block0, g.ngrids, g.zlen, (const TI*)I0,
                       (const TI*)I1, (const T*)E, x64, (T*)o0, (T*)o1, inv_scale, partials, x64o, escale);
  } else {
    return hipErrorInvalidValue;  // a wider I1 comes with slice (one-line) grids only
  }
  return hipSuccess;
}

// I1's type: that of I0, or FP32 / FP64
template <typename TI, typename T, int KIND, int MODE>
static hipError_t corr_stencil_launch(gd_dtype t1, gd_dtype tin, const Geom& g, const void* I0, const void* I1,
                                      const void* E, const double* x64, void* o0, void* o1,
                                      const double* inv_scale, double* partials, double* x64o,
                                      const double* escale, hipStream_t st) {
  if (t1 == tin || !I1)
    return corr_stencil_launch2<TI, TI, T, KIND, MODE>(g, I0, I1, E, x64, o0, o1, inv_scale, partials, x64o, escale,
                                                       st);
  if (t1 == GD_F64)
    return corr_stencil_launch2<TI, double, T, KIND, MODE>(g, I0, I1, E, x64, o0, o1, inv_scale, partials, x64o,
                                                           escale, st);
  if (t1 == GD_F32)
    return corr_stencil_launch2<TI, float, T, KIND, MODE>(g, I0, I1, E, x64, o0, o1, inv_scale, partials, x64o,
                                                          escale, st);
  return hipErrorInvalidValue;
}

hipError_t launch_rhs_corr(gd_dtype tin, gd_dtype t1, gd_dtype s, const Geom& g, const void* I0, const void* I1,
                           void* b, void* x, double* partials, hipStream_t st, const double* inv_scale) {
  if (g.nblocks == 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define L2(TI, T) \
  e = corr_stencil_launch<TI, T, 0, 0>(t1, tin, g, I0, I1, nullptr, nullptr, b, x, inv_scale, partials, nullptr, nullptr, st)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  if (e != hipSuccess) return e;
  return last();
}

hipError_t launch_canon_residual(gd_dtype tin, gd_dtype t1, gd_dtype s, int mode, const Geom& g, const void* I0,
                                 const void* I1, const void* E, const double* x64, void* r_out,
                                 const double* inv_scale, double* partials, hipStream_t st, double* x64_out,
                                 const double* e_scale) {
  if (g.nblocks == 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define L2(TI, T)                                                                                               \
  if (mode == 0)                                                                                                \
    e = corr_stencil_launch<TI, T, 1, 0>(t1, tin, g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, nullptr, \
                                         nullptr, st);                                                          \
  else if (mode == 1)                                                                                           \
    e = corr_stencil_launch<TI, T, 1, 1>(t1, tin, g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, nullptr, \
                                         nullptr, st);                                                          \
  else if (mode == 2)                                                                                           \
    e = corr_stencil_launch<TI, T, 1, 2>(t1, tin, g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, x64_out, \
                                         e_scale, st);                                                          \
  else                                                                                                          \
    e = corr_stencil_launch<TI, T, 1, 3>(t1, tin, g, I0, I1, E, x64, r_out, nullptr, inv_scale, partials, x64_out, \
                                         e_scale, st)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  if (e != hipSuccess) return e;
  return last();
}

hipError_t launch_sum_shift(gd_dtype tin, gd_dtype s, int mode, const Geom& g, const void* I0, const void* E,
                            const double* x64, double* partials, hipStream_t st, const void* E2) {
  if (g.nblocks == 0) return hipSuccess;
#define L2(TI, T)                                                                                             \
  if (mode == 0)                                                                                              \
    hipLaunchKernelGGL((k_sum_shift<TI, T, 0>), GD_ARGS(g), (const TI*)I0, (const T*)E, (const T*)E2, x64,     \
                       partials);                                                                             \
  else                                                                                                        \
    hipLaunchKernelGGL((k_sum_shift<TI, T, 1>), GD_ARGS(g), (const TI*)I0, (const T*)E, (const T*)E2, x64, partials)
#define L1(TI) GD_DISPATCH_S2(s, TI, L2)
  GD_DISPATCH_S(tin, L1)
#undef L1
#undef L2
  return last();
}

template <typename TI, typename T>
static hipError_t finalize_out(gd_dtype tout, int mode, const Geom& g, const void* I0, const void* E, const void* E2,
                               const double* x64, const double* shift, void* out, hipStream_t st) {
#define L(TO)                                                                                                \
  if (mode == 0)                                                                                             \
    hipLaunchKernelGGL((k_finalize<TI, T, TO, 0>), GD_ARGS(g), (const TI*)I0, (const T*)E, (const T*)E2, x64, \
                       shift, (TO*)out);                                                                     \
  else                                                                                                       \
    hipLaunchKernelGGL((k_finalize<TI, T, TO, 1>), GD_ARGS(g), (const TI*)I0, (const T*)E, (const T*)E2, x64, \
                       shift, (TO*)out)
  GD_DISPATCH_S(tout, L)
#undef L
  return hipSuccess;
}

hipError_t launch_finalize(gd_dtype tin, gd_dtype s, gd_dtype tout, int mode, const Geom& g, const void* I0,
                           const void* E, const double* x64, const double* shift, void* out, hipStream_t st,
                           const void* E2) {
  if (g.nblocks == 0) return hipSuccess;
  hipError_t e = hipSuccess;
#define L2(TI, T) e = finalize_out<TI, T>(tout, mode, g, I0, E, E2, x64, shift, out, st)
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

}  // namespace gd
