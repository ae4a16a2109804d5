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
// line L is at (L mod nf) * sf + (L / nf) * ss + j * stride; every length
// is a power of two, so the divisions are shifts
struct DctLines {
  int n, logn;
  int64_t stride;
  int64_t nf, sf, ss;
  int lognf;
  int64_t nlines;
  int lpb, loglpb;   // lines per block
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

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// LDS position of complex value i of a block: the low four bits are XORed
// with the XOR of the next three nibbles.  This permutes each aligned group
// of 16 (no extra LDS), and spreads over the banks both the bit-reversed
// scatter of the loads and the short strides of the first FFT steps, which
// would otherwise fall on a few banks.
__device__ __forceinline__ int swz(int i) { return i ^ (((i >> 4) ^ (i >> 8) ^ (i >> 12)) & 15); }

// one DCT-II (INV = false) or inverse pass along the lines of d, reading src
// (type TI) and writing dst (type TO); src == dst for the FP64 work array
// LDS (dynamic, sized by the launch): the block's lines as complex values,
// then the FFT twiddles of this length (loaded once per block instead of at
// every step).  The inverse first keeps its real coefficients in the complex
// buffer's space; each thread reads the pairs it needs into registers before
// the buffer is overwritten, so no second buffer costs occupancy.
// The FFT is decimation in time on bit-reversed input; two radix-2 stages
// (half sizes h and 2h) are done at once as one radix-4 step on four values
// h apart, so a length-2^m transform takes ceil(m / 2) barriers.
template <bool INV, typename TI, typename TO>
__global__ void __launch_bounds__(DCT_NT) k_dct_lines(const TI* src, TO* dst, DctLines d) {
  extern __shared__ double2 smem[];
  const int n = d.n, logn = d.logn, lpb = d.lpb, tot = n << d.loglpb;
  double2* V = smem;
  double* X = reinterpret_cast<double*>(smem);  // inverse: coefficients, until the twiddle step
  double2* Wt = smem + tot;
  for (int t = threadIdx.x; t < (n >> 1); t += DCT_NT) Wt[t] = d.W[t];
  const int64_t l0 = (int64_t)blockIdx.x << d.loglpb;
  const int64_t fmask = d.nf - 1;
  auto base = [&](int l) -> int64_t {
    const int64_t L = l0 + l;
    return (L & fmask) * d.sf + (L >> d.lognf) * d.ss;
  };
  auto split = [&](int e, int& l, int& j) {
    if (d.adjacent) { l = e & (lpb - 1); j = e >> d.loglpb; }
    else { l = e >> logn; j = e & (n - 1); }
  };
  for (int e = threadIdx.x; e < tot; e += DCT_NT) {
    int l, j;
    split(e, l, j);
    const double v = (l0 + l < d.nlines) ? ld_any(src + base(l) + j * d.stride) : 0.0;
    if (!INV) V[swz((l << logn) + bitrev(mk_pos(j, n), logn))] = make_double2(v, 0.0);
    else X[(l << logn) + j] = v;
  }
  __syncthreads();
  if (INV) {
    // V_k = exp(i pi k / 2n) (X_k - i X_{n-k}) = conj(Q_k) (X_k - i X_{n-k}), X_n = 0;
    // all reads of X before the barrier, all writes of V after it
    constexpr int R = DCT_LDS / DCT_NT;
    double2 tv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = threadIdx.x + r * DCT_NT;
      if (e < tot) {
        const int l = e >> logn, k = e & (n - 1);
        const double xk = X[(l << logn) + k], xm = k == 0 ? 0.0 : X[(l << logn) + n - k];
        const double2 q = d.Q[k];
        const double ck = q.x, sk = -q.y;
        tv[r] = make_double2(ck * xk + sk * xm, sk * xk - ck * xm);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = threadIdx.x + r * DCT_NT;
      if (e < tot) V[swz(((e >> logn) << logn) + bitrev(e & (n - 1), logn))] = tv[r];
    }
    __syncthreads();
  }
  int lh = 0;  // log2 of the half size of the next stage
  if (logn & 1) {  // odd length exponent: one radix-2 stage of half size 1 (twiddle 1)
    for (int e = threadIdx.x; e < (tot >> 1); e += DCT_NT) {
      const int a = swz(2 * e), b = swz(2 * e + 1);
      const double2 u = V[a], t = V[b];
      V[a] = cadd(u, t);
      V[b] = csub(u, t);
    }
    __syncthreads();
    lh = 1;
  }
  for (; lh + 2 <= logn; lh += 2) {
    // stages of half sizes h and 2h: twiddles W_{2h}^p = W[p n / 2h] and
    // W_{4h}^p = W[p n / 4h]; the second stage's pair (p + h, p + 3h) takes
    // W_{4h}^{p+h} = -i W_{4h}^p (+i for the inverse)
    const int h = 1 << lh, t2 = logn - lh - 2;
    for (int e = threadIdx.x; e < (tot >> 2); e += DCT_NT) {
      const int l = e >> (logn - 2), q = e & ((n >> 2) - 1);
      const int p = q & (h - 1);
      const int i0 = (l << logn) + ((q >> lh) << (lh + 2)) + p;
      double2 w1 = Wt[p << (t2 + 1)], w2 = Wt[p << t2];
      if (INV) { w1.y = -w1.y; w2.y = -w2.y; }
      const int p0 = swz(i0), p1 = swz(i0 + h), p2 = swz(i0 + 2 * h), p3 = swz(i0 + 3 * h);
      const double2 a = V[p0], b = cmul(w1, V[p1]), c = V[p2], dd = cmul(w1, V[p3]);
      const double2 a1 = cadd(a, b), b1 = csub(a, b);
      const double2 c1 = cmul(w2, cadd(c, dd)), d1 = cmul(w2, csub(c, dd));
      const double2 jd = INV ? make_double2(-d1.y, d1.x) : make_double2(d1.y, -d1.x);
      V[p0] = cadd(a1, c1);
      V[p1] = cadd(b1, jd);
      V[p2] = csub(a1, c1);
      V[p3] = csub(b1, jd);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < tot; e += DCT_NT) {
    int l, j;
    split(e, l, j);
    if (l0 + l >= d.nlines) continue;
    double out;
    if (!INV) {
      const double2 q = d.Q[j], v = V[swz((l << logn) + j)];
      out = q.x * v.x - q.y * v.y;  // Re(Q_j V_j)
      if (d.scale >= 0) {  // z-axis pass: line (i, jy), sample k = j
        const int64_t L = l0 + l;
        const int i = (int)(L & fmask), jy = (int)(L >> d.lognf);
        out *= dct_factor(d.scale, d.lx[i], d.ly[jy], d.lz[j], i == 0 && jy == 0 && j == 0, d.alpha, d.wx, d.wy,
                          d.wz);
      }
    } else {
      const int m = (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
      out = V[swz((l << logn) + m)].x / (double)n;
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

// out[z][x][y] = in[z][y][x] for an [nz][ny][nx] FP64 array, through a
// 32 x 32 LDS tile (one padding column against bank conflicts)
__global__ void __launch_bounds__(256) k_transpose_xy(const double* __restrict__ in, double* __restrict__ out, int nx,
                                                      int ny) {
  __shared__ double T[32][33];
  const int64_t z = blockIdx.z;
  const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const double* src = in + z * (int64_t)nx * ny;
  double* dst = out + z * (int64_t)nx * ny;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int y = y0 + r, x = x0 + threadIdx.x;
    if (x < nx && y < ny) T[r][threadIdx.x] = src[(int64_t)y * nx + x];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int x = x0 + r, y = y0 + threadIdx.x;
    if (x < nx && y < ny) dst[(int64_t)x * ny + y] = T[threadIdx.x][r];
  }
}

hipError_t dct_transpose_xy(const double* in, double* out, int nx, int ny, int nz, hipStream_t st) {
  const dim3 grid((unsigned)((nx + 31) / 32), (unsigned)((ny + 31) / 32), (unsigned)nz);
  hipLaunchKernelGGL(k_transpose_xy, grid, dim3(32, 8), 0, st, in, out, nx, ny);
  return hipGetLastError();
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
  const size_t lds = ((size_t)d.n * d.lpb + (size_t)(d.n / 2)) * sizeof(double2);
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
  // values per block, the fastest measured on MI355X: about 1024 in a
  // forward pass, 2048 in an inverse one.  Long lines of adjacent columns
  // (n >= 512) keep up to 4096 values, so that the lines of a block still
  // form runs of 4 or more values in memory.
  const int vals = (d.adjacent && d.n > 256) ? DCT_LDS : (p.inverse ? DCT_LDS / 2 : DCT_LDS / 4);
  d.lpb = vals / d.n;
  if (d.lpb < 1) d.lpb = 1;
  if (d.lpb > 64) d.lpb = 64;
  if (d.lpb > d.nlines) d.lpb = (int)d.nlines;
  d.loglpb = ilog2(d.lpb);
  d.lognf = ilog2((int)d.nf);
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
