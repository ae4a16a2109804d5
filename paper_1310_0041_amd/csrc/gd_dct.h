// Internal interface of the spectral (DCT) solver kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gd.h"

namespace gd {
// One DCT-II (forward) or inverse pass along `axis` (0 x, 1 y, 2 z) of a
// contiguous [nz][ny][nx] volume, every length a power of two <= 4096,
// reading src (tin) and writing dst (tout); src == dst is allowed.  W, Q:
// twiddle tables of that axis's length (dct_tables).  scale >= 0 (z-axis
// forward pass only): the coefficients are scaled on the way out (mode 0:
// 1 / (alpha + sum w_a lam_a), 0 for a zero eigenvalue; mode 1: the
// anisotropic-diffusion gain), lx / ly / lz the eigenvalue tables.
struct DctPass {
  int nx, ny, nz, axis;
  bool inverse;
  const void* src;
  gd_dtype tin;
  void* dst;
  gd_dtype tout;
  const double2 *W, *Q;
  int scale;
  const double *lx, *ly, *lz;
  double alpha, wx, wy, wz;
};
hipError_t dct_pass(const DctPass& p, hipStream_t st);
// W[t] = exp(-2 pi i t / n) (t < n / 2), Q[k] = exp(-i pi k / (2n)),
// lam[k] = 2 - 2 cos(pi k / n) (k < n)
hipError_t dct_tables(int n, double2* W, double2* Q, double* lam, hipStream_t st);
// the scaling as its own pass over an FP64 array
hipError_t dct_scale(double* c, int nx, int ny, int nz, int mode, const double* lx, const double* ly,
                     const double* lz, double alpha, double wx, double wy, double wz, hipStream_t st);
// out[z][x][y] = in[z][y][x] of an [nz][ny][nx] FP64 array (out must not alias in)
hipError_t dct_transpose_xy(const double* in, double* out, int nx, int ny, int nz, hipStream_t st);
// dtype t -> FP64 (to64: in = caller array, out = FP64) or FP64 -> dtype t
// (in = FP64 array, outp = caller array)
hipError_t dct_convert(const void* in, gd_dtype t, double* out, int64_t n, bool to64, void* outp, hipStream_t st);
}  // namespace gd
