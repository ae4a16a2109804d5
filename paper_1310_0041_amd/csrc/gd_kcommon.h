// Device helpers and launch macros shared by the gfx950 kernel files.
#pragma once

#include <cstdlib>
#include <type_traits>
#include "gd_launch.h"

namespace gd {

// ---------------------------------------------------------------- helpers

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

// Fused multiply-add in the compute type (explicit, so that the rounding
// order is fixed wherever an expression is written with it).
template <typename C>
__device__ __forceinline__ C fmac(C a, C b, C c) {
  if constexpr (sizeof(C) == 8) return __builtin_fma(a, b, c);
  else return __builtin_fmaf(a, b, c);
}

// Exact FP64 value of element v of a caller's array.
template <typename Tin>
__device__ __forceinline__ double in_at(const Tin* p, int64_t v) { return ld64(p + v); }

// ---------------------------------------------------------- launch macros

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

static inline hipError_t last() { return hipGetLastError(); }

}  // namespace gd
