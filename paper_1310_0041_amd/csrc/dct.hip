// gfx950 kernels of the spectral (DCT) solver for the constant-coefficient
// systems of Sec. 4 with natural (Neumann) boundaries.
//
// The cosines cos(pi k (j + 1/2) / n), k = 0 .. n-1, are the eigenvectors of
// the 3-point Neumann second difference (eigenvalue 2 - 2 cos(pi k / n)),
// so a DCT-II along every axis diagonalises alpha + sum_a w_a L_a: the
// discrete counterpart of the frequency-space analysis of Sec. 3.2.  A solve
// is three forward transforms, one division per coefficient and three
// inverse transforms, in FP64.
//
// A DCT-II of length n (a power of two) is one complex FFT of the input
// reordered as (x0, x2, x4, ..., x5, x3, x1) followed by a twiddle:
// X_k = Re(exp(-i pi k / (2n)) V_k) = sum_j x_j cos(pi k (2j + 1) / (2n))
// (Makhoul's method); its inverse forms V_k = exp(i pi k / (2n)) (X_k - i X_{n-k}),
// inverts the FFT and undoes the reordering.  A block holds the lines of one
// group in LDS (at most 4096 complex values), does the radix-2 FFT there and
// writes the result back in place.

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gd_dct.h"

namespace gd {

constexpr int DCT_LDS = 4096;  // complex FP64 values per block
constexpr int DCT_NT = 256;

__device__ __forceinline__ int bitrev(int v, int bits) {
  return bits == 0 ? 0 : (int)(__brev((unsigned)v) >> (32 - bits));
}

// position of input sample j in the reordered sequence
__device__ __forceinline__ int mk_pos(int j, int n) { return (j & 1) ? n - 1 - (j >> 1) : (j >> 1); }

// lines along one axis of a contiguous [nz][ny][nx] array: element j of
// line L is at (L mod nf) * sf + (L / nf) * ss + j * stride
struct DctLines {
  int n, logn;
  int64_t stride;
  int64_t nf, sf, ss;
  int64_t nlines;
  int lpb;           // lines per block
  bool adjacent;     // consecutive lines are consecutive in memory (sf == 1)
  // twiddles of this length: W[t] = exp(-2 pi i t / n), t < n / 2, and
  // Q[k] = exp(-i pi k / (2n)), k < n
  const double2* W;
  const double2* Q;
  // transform-domain scaling fused into a z-axis forward pass (mode 0 / 1,
  // see k_dct_scale); eigenvalue tables of x, y and z
  int scale;
  const double *lx, *ly, *lz;
  double alpha, wx, wy, wz;
};

// the scaling of coefficient (i, j, k): mode 0 the inverse eigenvalue (0 for
// a zero eigenvalue), mode 1 the anisotropic-diffusion gain
__device__ __forceinline__ double dct_factor(int mode, double lx, double ly, double lz, bool dc, double alpha,
                                             double wx, double wy, double wz) {
  if (mode == 0) {
    const double lam = alpha + wx * lx + wy * ly + wz * lz;
    return lam != 0.0 ? 1.0 / lam : 0.0;
  }
  const double num = wx * lx + wy * ly, den = num + wz * lz;
  return dc ? 1.0 : (den != 0.0 ? num / den : 0.0);
}

template <typename T>
__device__ __forceinline__ double ld_any(const T* p) { return (double)*p; }
template <>
__device__ __forceinline__ double ld_any<__half>(const __half* p) { return (double)__half2float(*p); }
template <>
__device__ __forceinline__ double ld_any<__hip_bfloat16>(const __hip_bfloat16* p) {
  return (double)__bfloat162float(*p);
}
template <typename T>
__device__ __forceinline__ void st_any(T* p, double v) { *p = (T)v; }
template <>
__device__ __forceinline__ void st_any<__half>(__half* p, double v) { *p = __float2half((float)v); }
template <>
__device__ __forceinline__ void st_any<__hip_bfloat16>(__hip_bfloat16* p, double v) {
  *p = __float2bfloat16((float)v);
}

// one DCT-II (INV = false) or inverse pass along the lines of d, reading src
// (type TI) and writing dst (type TO); src == dst for the FP64 work array
// LDS (dynamic, sized by the launch): the block's lines as complex values,
// then (inverse) their coefficients, read twice
template <bool INV, typename TI, typename TO>
__global__ void __launch_bounds__(DCT_NT) k_dct_lines(const TI* src, TO* dst, DctLines d) {
  extern __shared__ double2 smem[];
  const int n = d.n, lpb = d.lpb, tot = n * lpb;
  double2* V = smem;
  double* X = reinterpret_cast<double*>(smem + tot);
  const int64_t l0 = (int64_t)blockIdx.x * lpb;
  auto base = [&](int l) -> int64_t {
    const int64_t L = l0 + l;
    return (L % d.nf) * d.sf + (L / d.nf) * d.ss;
  };
  auto split = [&](int e, int& l, int& j) {
    if (d.adjacent) { l = e % lpb; j = e / lpb; }
    else { l = e / n; j = e % n; }
  };
  for (int e = threadIdx.x; e < tot; e += DCT_NT) {
    int l, j;
    split(e, l, j);
    const double v = (l0 + l < d.nlines) ? ld_any(src + base(l) + j * d.stride) : 0.0;
    if (!INV) V[l * n + bitrev(mk_pos(j, n), d.logn)] = make_double2(v, 0.0);
    else X[l * n + j] = v;
  }
  __syncthreads();
  if (INV) {
    // V_k = exp(i pi k / 2n) (X_k - i X_{n-k}) = conj(Q_k) (X_k - i X_{n-k}), X_n = 0
    for (int e = threadIdx.x; e < tot; e += DCT_NT) {
      const int l = e / n, k = e % n;
      const double xk = X[l * n + k], xm = k == 0 ? 0.0 : X[l * n + n - k];
      const double2 q = d.Q[k];
      const double ck = q.x, sk = -q.y;
      V[l * n + bitrev(k, d.logn)] = make_double2(ck * xk + sk * xm, sk * xk - ck * xm);
    }
    __syncthreads();
  }
  // radix-2 FFT: stage with half-size h uses W[p n / (2h)] (conjugated for the inverse)
  for (int st = 1; st <= d.logn; ++st) {
    const int h = 1 << (st - 1), tw = n >> st;
    for (int e = threadIdx.x; e < (n / 2) * lpb; e += DCT_NT) {
      const int l = e / (n / 2), bfly = e % (n / 2);
      const int grp = bfly / h, p = bfly % h;
      const int i0 = l * n + grp * 2 * h + p, i1 = i0 + h;
      const double2 w = d.W[p * tw];
      const double cw = w.x, sw = INV ? -w.y : w.y;
      const double2 u = V[i0], t = V[i1];
      const double2 wt = make_double2(cw * t.x - sw * t.y, cw * t.y + sw * t.x);
      V[i0] = make_double2(u.x + wt.x, u.y + wt.y);
      V[i1] = make_double2(u.x - wt.x, u.y - wt.y);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tot; e += DCT_NT) {
    int l, j;
    split(e, l, j);
    if (l0 + l >= d.nlines) continue;
    double out;
    if (!INV) {
      const double2 q = d.Q[j], v = V[l * n + j];
      out = q.x * v.x - q.y * v.y;  // Re(Q_j V_j)
      if (d.scale >= 0) {  // z-axis pass: line (i, jy), sample k = j
        const int64_t L = l0 + l;
        const int i = (int)(L % d.nf), jy = (int)(L / d.nf);
        out *= dct_factor(d.scale, d.lx[i], d.ly[jy], d.lz[j], i == 0 && jy == 0 && j == 0, d.alpha, d.wx, d.wy,
                          d.wz);
      }
    } else {
      const int m = (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
      out = V[l * n + m].x / (double)n;
    }
    st_any(dst + base(l) + j * d.stride, out);
  }
}

// transform-domain scaling as its own pass (used when nz == 1); row (j, k)
// per block row, eigenvalue tables per axis
__global__ void __launch_bounds__(DCT_NT) k_dct_scale(double* __restrict__ c, int nx, int ny, int nz, int mode,
                                                       const double* __restrict__ lx, const double* __restrict__ ly,
                                                       const double* __restrict__ lz, double alpha, double wx,
                                                       double wy, double wz) {
  const int j = blockIdx.y, k = blockIdx.z;
  for (int i = blockIdx.x * DCT_NT + threadIdx.x; i < nx; i += gridDim.x * DCT_NT) {
    const int64_t q = ((int64_t)k * ny + j) * nx + i;
    c[q] *= dct_factor(mode, lx[i], ly[j], lz[k], i == 0 && j == 0 && k == 0, alpha, wx, wy, wz);
  }
}

// twiddle tables of one length n
__global__ void k_dct_tables(int n, double2* W, double2* Q, double* lam) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    double s, c;
    if (t < n / 2) {
      sincospi(-2.0 * (double)t / (double)n, &s, &c);
      W[t] = make_double2(c, s);
    }
    sincospi(-(double)t / (2.0 * (double)n), &s, &c);
    Q[t] = make_double2(c, s);
    lam[t] = 2.0 - 2.0 * cospi((double)t / (double)n);
  }
}

// whole-array conversions (only for grids with every axis of length 1, where
// no transform pass reads the input or writes the output)
template <typename T>
__global__ void __launch_bounds__(DCT_NT) k_to64(const T* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * DCT_NT + threadIdx.x; q < n; q += (int64_t)gridDim.x * DCT_NT)
    out[q] = ld_any(in + q);
}
template <typename T>
__global__ void __launch_bounds__(DCT_NT) k_from64(const double* __restrict__ in, T* __restrict__ out, int64_t n) {
  for (int64_t q = (int64_t)blockIdx.x * DCT_NT + threadIdx.x; q < n; q += (int64_t)gridDim.x * DCT_NT)
    st_any(out + q, in[q]);
}

hipError_t dct_convert(const void* in, gd_dtype t, double* out, int64_t n, bool to64, void* outp, hipStream_t st) {
  const unsigned blocks = (unsigned)((n + DCT_NT - 1) / DCT_NT > 65536 ? 65536 : (n + DCT_NT - 1) / DCT_NT);
#define C(T)                                                                                                     \
  if (to64) hipLaunchKernelGGL(k_to64<T>, dim3(blocks), dim3(DCT_NT), 0, st, (const T*)in, out, n);            \
  else hipLaunchKernelGGL(k_from64<T>, dim3(blocks), dim3(DCT_NT), 0, st, (const double*)in, (T*)outp, n)
  switch (t) {
    case GD_F64: C(double); break;
    case GD_F32: C(float); break;
    case GD_F16: C(__half); break;
    case GD_BF16: C(__hip_bfloat16); break;
    default: return hipErrorInvalidValue;
  }
#undef C
  return hipGetLastError();
}

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

hipError_t dct_tables(int n, double2* W, double2* Q, double* lam, hipStream_t st) {
  hipLaunchKernelGGL(k_dct_tables, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, W, Q, lam);
  return hipGetLastError();
}

template <bool INV, typename TI, typename TO>
static void lines_launch(const void* src, void* dst, const DctLines& d, unsigned blocks, hipStream_t st) {
  const size_t lds = (size_t)d.n * d.lpb * (sizeof(double2) + (INV ? sizeof(double) : 0));
  hipLaunchKernelGGL((k_dct_lines<INV, TI, TO>), dim3(blocks), dim3(DCT_NT), lds, st, (const TI*)src, (TO*)dst, d);
}

template <bool INV, typename TI>
static hipError_t lines_out(gd_dtype to, const void* src, void* dst, const DctLines& d, unsigned blocks,
                            hipStream_t st) {
  switch (to) {
    case GD_F64: lines_launch<INV, TI, double>(src, dst, d, blocks, st); break;
    case GD_F32: lines_launch<INV, TI, float>(src, dst, d, blocks, st); break;
    case GD_F16: lines_launch<INV, TI, __half>(src, dst, d, blocks, st); break;
    case GD_BF16: lines_launch<INV, TI, __hip_bfloat16>(src, dst, d, blocks, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t dct_pass(const DctPass& p, hipStream_t st) {
  DctLines d{};
  const int64_t nx = p.nx, ny = p.ny, nz = p.nz, pl = nx * ny;
  if (p.axis == 0) { d.n = p.nx; d.stride = 1; d.nf = ny; d.sf = nx; d.ss = pl; d.nlines = ny * nz; }
  else if (p.axis == 1) { d.n = p.ny; d.stride = nx; d.nf = nx; d.sf = 1; d.ss = pl; d.nlines = nx * nz; }
  else { d.n = p.nz; d.stride = pl; d.nf = nx; d.sf = 1; d.ss = nx; d.nlines = nx * ny; }
  d.logn = ilog2(d.n);
  d.adjacent = d.sf == 1;
  // about 2048 values per block (several blocks per CU), except long strided
  // lines (y or z, n >= 512), which keep up to 4096 so that the adjacent lines
  // of a block still form runs of 4 or more values in memory
  d.lpb = ((!d.adjacent || d.n <= 256) ? DCT_LDS / 2 : DCT_LDS) / d.n;
  if (d.lpb < 1) d.lpb = 1;
  if (d.lpb > 64) d.lpb = 64;
  if (d.lpb > d.nlines) d.lpb = (int)d.nlines;
  d.W = p.W; d.Q = p.Q;
  d.scale = p.scale;
  d.lx = p.lx; d.ly = p.ly; d.lz = p.lz;
  d.alpha = p.alpha; d.wx = p.wx; d.wy = p.wy; d.wz = p.wz;
  const unsigned blocks = (unsigned)((d.nlines + d.lpb - 1) / d.lpb);
#define IN(TI) return p.inverse ? lines_out<true, TI>(p.tout, p.src, p.dst, d, blocks, st) \
                                : lines_out<false, TI>(p.tout, p.src, p.dst, d, blocks, st)
  switch (p.tin) {
    case GD_F64: IN(double);
    case GD_F32: IN(float);
    case GD_F16: IN(__half);
    case GD_BF16: IN(__hip_bfloat16);
    default: return hipErrorInvalidValue;
  }
#undef IN
}

hipError_t dct_scale(double* c, int nx, int ny, int nz, int mode, const double* lx, const double* ly,
                     const double* lz, double alpha, double wx, double wy, double wz, hipStream_t st) {
  const unsigned gx = (unsigned)((nx + DCT_NT - 1) / DCT_NT);
  hipLaunchKernelGGL(k_dct_scale, dim3(gx, (unsigned)ny, (unsigned)nz), dim3(DCT_NT), 0, st, c, nx, ny, nz, mode, lx,
                     ly, lz, alpha, wx, wy, wz);
  return hipGetLastError();
}

}  // namespace gd
