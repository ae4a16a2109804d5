// Host-side launchers of the gfx950 kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gd.h"
#include "gd_device.h"

namespace gd {

// Tile shapes of the kernel families.
constexpr int SW_TX = 64, SW_TY = 8;   // relaxation tile of 3-D grids, 256 threads (one x-pair each)
constexpr int SWR_TX = 256;            // relaxation tile of one-line grids (2-D slices), 128 threads
constexpr int EW_TX = 64, EW_TY = 4;   // per-voxel kernels on 3-D grids: 256 threads
constexpr int EWR_TX = 256;            // per-voxel kernels on one-line grids
// Relaxation tile variants of 3-D grids: 0: 64 x 8, 1: 128 x 8, 2: 64 x 16,
// 3: 128 x 16, and for the quad form only 4: 256 x 8, 5: 256 x 12.  Wider
// and taller tiles re-read a smaller share of halo cells per voxel (at
// 1024 threads, 256 x 16, the registers of a thread no longer fit).
constexpr int kSweepTiles = 6, kPairTiles = 4;
constexpr int SWEEP_TILE_TX[kSweepTiles] = {64, 128, 64, 128, 256, 256};
constexpr int SWEEP_TILE_TY[kSweepTiles] = {8, 8, 16, 16, 8, 12};

// A launch over the grids of one level: blocks [block0[g], block0[g+1])
// belong to grid g; each block covers one (x, y) tile and `zlen` planes.
struct Geom {
  const GridDesc* grids = nullptr;  // device array
  const int64_t* block0 = nullptr;  // device array, ngrids + 1 entries
  int ngrids = 0;
  int64_t nblocks = 0;
  int zlen = 1;
  int etx = EW_TX;   // per-voxel kernels: tile etx x (256 / etx)
  bool row = false;  // relaxation: one-line (slice) tiles
  bool vec = true;   // every grid's pitch and offset are even (x pairs aligned)
  int tile = 0;      // relaxation tile variant of 3-D grids (SWEEP_TILE_TX / TY)
  int order = 0;     // relaxation block order: 0 plain, 1 contiguous runs per XCD
  bool quad = false; // the library's own arrays (x pitch and offsets multiples of 4, aligned):
                     // the relaxation may use its quad form
  int64_t n_int = 0, n_edge = 0;  // quad relaxation of a one-grid 3-D level: blocks of its interior and
                                  // edge tiles (n_int 0: one launch over the tile table)
  int zlen_edge = 1;              // z-chunk of the edge tiles' launch
  bool stencil4 = false;  // the finest-level stencil passes in their quad form (tiles
                          // CS4_TX[tile] x CS4_TY[tile]; 3-D grids, quad-aligned inputs)
};
// Tiles of the quad-form finest-level stencil passes of 3-D grids.
constexpr int CS4_TX[2] = {128, 64};
constexpr int CS4_TY[2] = {8, 16};

// xzero: x_in is all zero (not read; the quad form only, see
// sweep_starts_from_zero_ok)
hipError_t launch_rb_sweep(gd_dtype s, const Geom& g, const void* xin, void* xout, const void* b,
                           const void* e_coarse, int prolong_mode, hipStream_t st, bool xzero = false);
bool sweep_starts_from_zero_ok(gd_dtype s, const Geom& g);
// the relaxation of the library's 3-D arrays in storage s takes the quad
// form (quad: the caller's sweep_quad option), so the wide tiles 4 and 5 exist
bool sweep_wide_tiles_ok(gd_dtype s, bool quad);
// Residual + restriction (tiles as the relaxation, zlen even); per-block
// sum r^2 into partials when non-NULL, coarse x zeroed when non-NULL.
hipError_t launch_restrict_z(gd_dtype s, const Geom& g, const void* x, const void* b, void* b_coarse,
                             void* x_coarse, double* partials, hipStream_t st);
// x += P e for the library's arrays, relaxation tiles (one x-pair per thread).
// keep_x: every grid of the level keeps x (f_x == 1).
hipError_t launch_prolong_pair(gd_dtype s, const Geom& g, const void* e_coarse, void* x, int mode, bool keep_x,
                               hipStream_t st);
hipError_t launch_prolong_add(gd_dtype s, const Geom& g, const void* e_coarse, void* x, int mode,
                              hipStream_t st);
// Finest level of the AD/SP systems in correction form: b = alpha (I1 - I0)
// - w_z L_z I0 (written when b != NULL, times inv_scale[g] when that is
// given, a power of two; x zeroed when x != NULL) and per
// block two FP64 sums (partials[2 block], [2 block + 1]): the squares of the
// canonical right-hand side alpha I1 + (w_x L_x + w_y L_y) I0 and of b.
// I1 (read only when alpha != 0) has type t1: tin, or F32 / F64 on slice
// (one-line) grids.
hipError_t launch_rhs_corr(gd_dtype tin, gd_dtype t1, gd_dtype s, const Geom& g, const void* I0, const void* I1,
                           void* b, void* x, double* partials, hipStream_t st, const double* inv_scale = nullptr);
// FP64 canonical residual r = b - A x of the AD/SP system for x = I0 + E
// (mode 0, E packed in `s`), x = x64 (mode 1) or x = x64 + e_scale[g] E
// (mode 2, the refinement update, also written to x64_out, which must not
// alias x64), or x = I0 + e_scale[g] E (mode 3: the first update, x64 not
// read).  Per block: sum r^2.  When r_out != NULL also writes
// r * inv_scale[g] packed in `s`.
hipError_t launch_canon_residual(gd_dtype tin, gd_dtype t1, gd_dtype s, int mode, const Geom& g, const void* I0,
                                 const void* I1, const void* E, const double* x64, void* r_out,
                                 const double* inv_scale, double* partials, hipStream_t st,
                                 double* x64_out = nullptr, const double* e_scale = nullptr);
// Per block: sum (x - I0) for x = I0 + E (mode 0) or x64 (mode 1).  A grid
// flagged `alt` reads E from E2 (the level's other buffer).
hipError_t launch_sum_shift(gd_dtype tin, gd_dtype s, int mode, const Geom& g, const void* I0,
                            const void* E, const double* x64, double* partials, hipStream_t st,
                            const void* E2 = nullptr);
// out = x - shift[g] in the caller's layout, x = I0 + E (mode 0) or x64 (mode 1);
// E2 as for launch_sum_shift.
hipError_t launch_finalize(gd_dtype tin, gd_dtype s, gd_dtype tout, int mode, const Geom& g,
                           const void* I0, const void* E, const double* x64, const double* shift,
                           void* out, hipStream_t st, const void* E2 = nullptr);
hipError_t launch_refine_init(gd_dtype tin, const Geom& g, const void* I0, double* x64, hipStream_t st);
// Generic system: b = alpha V + sum_a w_a D_a^T G_a.
hipError_t launch_rhs_general(gd_dtype s, const Geom& g, const void* V, const void* Gx,
                              const void* Gy, const void* Gz, void* b, hipStream_t st);
// Generic system: per block (sum (b - A x)^2, sum b^2) in FP64; r_out
// (may be NULL) receives b - A x.  lib_layout: x, b, r are a hierarchy level
// (offset off, pitch px) instead of the caller's arrays.  Planes outside
// [klo, khi) are skipped (neither summed nor written).
hipError_t launch_general_residual(gd_dtype s, const Geom& g, const void* x, const void* b, void* r_out,
                                   double* partials, hipStream_t st, bool lib_layout = false, int klo = 0,
                                   int khi = 0x7fffffff);
// Hybrid discretisation (Sec. 4.2): a table level's operator is
// alpha Mx My Mz + w_x Kx My Mz + w_y Mx Ky Mz + w_z Mx My Kz, t[a] the device
// table block of axis a (six rows of n_a doubles: M below/on/above the
// diagonal, then K).  G: the level's descriptor (one grid; offset and pitch
// of the level arrays, child sizes and factors for the transfers).
struct HybTables {
  const double* t[3];
  double alpha, w[3];
};
// one colour (0..7) of an 8-colour Gauss-Seidel sweep of a table level, in place
hipError_t launch_hyb_gs8(gd_dtype s, const GridDesc& G, const HybTables& T, int colour, void* x, const void* b,
                          hipStream_t st);
// one whole 8-colour sweep of a table level from xin into xout (two launches,
// one per z-parity of the planes; same values as the eight colour launches);
// xin and xout must not overlap
hipError_t launch_hyb_gs8z(gd_dtype s, const GridDesc& G, const HybTables& T, const void* xin, void* xout,
                           const void* b, hipStream_t st);
// r = b - A x on a table level; with partials, per-block FP64 sums of r^2
// in partials[0 .. hyb_residual_blocks(G, per_plane)); per_plane: every block
// spans one plane, plane z's blocks at [z B, (z + 1) B), B = blocks / nz
int64_t hyb_residual_blocks(const GridDesc& G, bool per_plane = false);
hipError_t launch_hyb_residual(gd_dtype s, const GridDesc& G, const HybTables& T, const void* x, const void* b,
                               void* r, hipStream_t st, double* partials = nullptr, bool per_plane = false);
// the caller's input I0 (dtype tin, layout ioff / ipy / ipz of G) into a level array of dtype s
hipError_t launch_load_input(gd_dtype tin, gd_dtype s, const GridDesc& G, const void* in, void* out, hipStream_t st);
// out = c0 in0 + c1 in1 (FP64 arithmetic): the caller's inputs (layout ioff /
// ipy / ipz of G; in1 of type t1 = tin, F32 or F64, or NULL) into a level array
hipError_t launch_load_comb(gd_dtype tin, gd_dtype t1, gd_dtype s, const GridDesc& G, const void* in0,
                            const void* in1, double c0, double c1, void* out, hipStream_t st);
// Streamed anisotropic diffusion: b = -b_z L_z I0 of the planes [k0, k1) of a
// dense window of the caller's input (window plane 0 = global plane z0 of an
// nzg-plane stack), written dense; per-block FP64 sums of the canonical
// right-hand side squared in partials[0 .. stream_rhs_blocks(nx, ny))
int64_t stream_rhs_blocks(int64_t nx, int64_t ny);
hipError_t launch_stream_rhs(gd_dtype tin, gd_dtype s, const void* I0, void* b, int nx, int ny, int nzg, int z0,
                             int k0, int k1, double bx, double by, double bz, double* partials, hipStream_t st);
// r = b - A x on the finest (7-point) level of a Hybrid hierarchy, with
// per-block FP64 sums of r^2 in partials[0 .. hyb_residual7_blocks(G))
int64_t hyb_residual7_blocks(const GridDesc& G);
hipError_t launch_hyb_residual7(gd_dtype s, const GridDesc& G, const void* x, const void* b, void* r,
                                double* partials, hipStream_t st);
// child b = P^T r and child x = 0 (B-spline nesting along the halved axes of G)
hipError_t launch_hyb_restrict(gd_dtype s, const GridDesc& G, const void* r, void* bc, void* xc, hipStream_t st);
// x += P e, e the child correction
hipError_t launch_hyb_prolong(gd_dtype s, const GridDesc& G, const void* e, void* x, hipStream_t st);
// Gradient-modulation filter (Sec. 6): the correction-form right-hand side
// from I0 (caller's layout, dtype tin) into b (finest level, dtype s); per
// block FP64 (sum of the canonical rhs squared, sum of b squared).
hipError_t launch_npr_rhs(gd_dtype tin, gd_dtype s, const Geom& g, const void* I0, double lam, double sigma,
                          void* b, double* partials, hipStream_t st);
// Krylov vectors (caller's layout): q = A p with per-block p.q; per-block a.b;
// x += c0 p, r -= c0 q with per-block r.r; out = c0 X + c1 Y.
hipError_t launch_apply_dot(gd_dtype s, const Geom& g, const void* p, void* q, double* partials, hipStream_t st);
hipError_t launch_dot(gd_dtype s, const Geom& g, const void* a, const void* b, double* partials, hipStream_t st);
hipError_t launch_cg_update(gd_dtype s, const Geom& g, const double* coef, void* x, void* r, const void* p,
                            const void* q, double* partials, hipStream_t st);
hipError_t launch_axpby(gd_dtype s, const Geom& g, const double* coef, const void* X, const void* Y, void* out,
                        hipStream_t st);
// out[g * ncomp + c] = sum of partials[b * ncomp + c] over the blocks of grid g.
hipError_t launch_reduce(const double* partials, const int64_t* block0, int ngrids, int ncomp,
                         double* out, hipStream_t st);

}  // namespace gd
