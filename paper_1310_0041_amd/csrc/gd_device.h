// Device-side types shared by the gfx950 kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <type_traits>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace gd {

// One grid of one multigrid level.  A level holds one grid (a 3-D stack) or
// many (a batch of independent 2-D slices); every array of a level is the
// concatenation of its grids' [nz][ny][nx] blocks.
struct GridDesc {
  int64_t off;    // first element of this grid in the level's arrays
  int64_t coff;   // first element of its child grid in the next level's arrays
  int64_t ioff;   // first element in the caller's arrays (finest level I/O)
  int64_t ipy;    // caller's row pitch (elements)
  int64_t ipz;    // caller's plane pitch (elements)
  int32_t nx, ny, nz;
  int32_t cnx, cny, cnz;  // child grid size
  int32_t fx, fy, fz;     // coarsening factor per axis (1 or 2)
  int32_t px;             // x pitch of this level's arrays (>= nx)
  int32_t cpx;            // x pitch of the child grid's arrays
  int32_t zin;            // 1: a 2-D slice seen as nz rows of one line (z is in-slice)
  int32_t skip;           // 1: the cycle kernels leave this grid alone (a slice of a batch
                          // that has converged)
  int32_t alt;            // 1: the output pass reads this grid's finest correction from the
                          // level's second buffer (where it was when the grid converged)
  int32_t pad_;
  double alpha, wx, wy, wz;  // operator alpha*Id + sum_a w_a L_a of this level
};

// Storage-type traits: load to / store from the arithmetic type.
template <typename S> struct Ty;
template <> struct Ty<double> {
  using C = double;
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
  static __device__ __forceinline__ void st(double* p, double v) { *p = v; }
};
template <> struct Ty<float> {
  using C = float;
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
  static __device__ __forceinline__ void st(float* p, float v) { *p = v; }
};
// A 16-bit store rounds the FP32 value it is given.  A value computed in
// FP64 and cast to float first is thus rounded twice; the empty asm keeps the
// compiler from folding the two roundings into one (it does so for some
// call sites and not others, which made equal expressions store different
// values) and from fusing the last multiply-add into a mixed-precision FMA
// that rounds once to 16 bits.
template <> struct Ty<__half> {
  using C = float;
  static __device__ __forceinline__ float ld(const __half* p) { return __half2float(*p); }
  static __device__ __forceinline__ void st(__half* p, float v) {
    asm volatile("" : "+v"(v));
    *p = __float2half_rn(v);
  }
};
template <> struct Ty<__hip_bfloat16> {
  using C = float;
  static __device__ __forceinline__ float ld(const __hip_bfloat16* p) { return __bfloat162float(*p); }
  static __device__ __forceinline__ void st(__hip_bfloat16* p, float v) {
    asm volatile("" : "+v"(v));
    *p = __float2bfloat16(v);
  }
};

// Two consecutive values (p aligned to two elements when vec).
template <typename S>
__device__ __forceinline__ void ld2(const S* p, bool vec, bool second, typename Ty<S>::C& a,
                                    typename Ty<S>::C& b) {
  using C = typename Ty<S>::C;
  if (vec) {
    if constexpr (sizeof(S) == 8) {
      const double2 v = *reinterpret_cast<const double2*>(p);
      a = (C)v.x; b = (C)v.y;
    } else if constexpr (sizeof(S) == 4) {
      const float2 v = *reinterpret_cast<const float2*>(p);
      a = (C)v.x; b = (C)v.y;
    } else {
      const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
      S lo, hi;
      const uint16_t l16 = (uint16_t)(v & 0xffffu), h16 = (uint16_t)(v >> 16);
      __builtin_memcpy(&lo, &l16, 2);
      __builtin_memcpy(&hi, &h16, 2);
      a = Ty<S>::ld(&lo); b = Ty<S>::ld(&hi);
    }
  } else {
    a = Ty<S>::ld(p);
    b = second ? Ty<S>::ld(p + 1) : (C)0;
  }
}

template <typename S>
__device__ __forceinline__ void st2(S* p, bool vec, bool second, typename Ty<S>::C a, typename Ty<S>::C b) {
  if (vec) {
    if constexpr (sizeof(S) == 8) {
      *reinterpret_cast<double2*>(p) = make_double2((double)a, (double)b);
    } else if constexpr (sizeof(S) == 4) {
      *reinterpret_cast<float2*>(p) = make_float2((float)a, (float)b);
    } else {
      S lo, hi;
      Ty<S>::st(&lo, a); Ty<S>::st(&hi, b);
      uint16_t l16, h16;
      __builtin_memcpy(&l16, &lo, 2);
      __builtin_memcpy(&h16, &hi, 2);
      *reinterpret_cast<uint32_t*>(p) = (uint32_t)l16 | ((uint32_t)h16 << 16);
    }
  } else {
    Ty<S>::st(p, a);
    if (second) Ty<S>::st(p + 1, b);
  }
}

// Raw (unconverted) values: a load whose result is converted at once makes
// the wave wait for it right there; kept raw, the wait moves to the first
// use and the load stays in flight meanwhile.
template <typename S> struct Raw {
  using W = std::conditional_t<sizeof(S) == 8, double, std::conditional_t<sizeof(S) == 4, float, uint32_t>>;
  W w = 0;
};
template <typename S> struct Raw2 {  // two consecutive values
  using W = std::conditional_t<sizeof(S) == 8, double2, std::conditional_t<sizeof(S) == 4, float2, uint32_t>>;
  W w;
  __device__ __forceinline__ Raw2() { __builtin_memset(&w, 0, sizeof(W)); }
};

template <typename S> __device__ __forceinline__ void ld_raw(const S* p, Raw<S>& r) {
  if constexpr (sizeof(S) == 2) r.w = *reinterpret_cast<const uint16_t*>(p);
  else r.w = *p;
}
template <typename S> __device__ __forceinline__ void ld_raw2(const S* p, bool vec, bool second, Raw2<S>& r) {
  if constexpr (sizeof(S) == 8) {
    if (vec) r.w = *reinterpret_cast<const double2*>(p);
    else { r.w.x = p[0]; r.w.y = second ? p[1] : 0.0; }
  } else if constexpr (sizeof(S) == 4) {
    if (vec) r.w = *reinterpret_cast<const float2*>(p);
    else { r.w.x = p[0]; r.w.y = second ? p[1] : 0.f; }
  } else {
    if (vec) {
      r.w = *reinterpret_cast<const uint32_t*>(p);
    } else {
      const uint32_t lo = *reinterpret_cast<const uint16_t*>(p);
      const uint32_t hi = second ? (uint32_t)*reinterpret_cast<const uint16_t*>(p + 1) : 0u;
      r.w = lo | (hi << 16);
    }
  }
}
template <typename S> __device__ __forceinline__ float from_bits16f(uint32_t h) {
  if constexpr (std::is_same_v<S, __hip_bfloat16>) return __uint_as_float(h << 16);
  else return __half2float(__ushort_as_half((unsigned short)h));
}
// conversions to the compute type Ty<S>::C
template <typename S> __device__ __forceinline__ typename Ty<S>::C raw_c(const Raw<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16f<S>(r.w);
  else return r.w;
}
template <typename S> __device__ __forceinline__ typename Ty<S>::C raw_ca(const Raw2<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16f<S>(r.w & 0xffffu);
  else return r.w.x;
}
template <typename S> __device__ __forceinline__ typename Ty<S>::C raw_cb(const Raw2<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16f<S>(r.w >> 16);
  else return r.w.y;
}
template <typename S> __device__ __forceinline__ double from_bits16(uint32_t h) {
  if constexpr (std::is_same_v<S, __hip_bfloat16>) return (double)__uint_as_float(h << 16);
  else return (double)__half2float(__ushort_as_half((unsigned short)h));
}
template <typename S> __device__ __forceinline__ double raw_d(const Raw<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16<S>(r.w);
  else return (double)r.w;
}
template <typename S> __device__ __forceinline__ double raw_a(const Raw2<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16<S>(r.w & 0xffffu);
  else return (double)r.w.x;
}
template <typename S> __device__ __forceinline__ double raw_b(const Raw2<S>& r) {
  if constexpr (sizeof(S) == 2) return from_bits16<S>(r.w >> 16);
  else return (double)r.w.y;
}

// Exact upcast to double (every storage type embeds in binary64).
template <typename T> __device__ __forceinline__ double ld64(const T* p) { return (double)Ty<T>::ld(p); }
template <typename T> __device__ __forceinline__ void st64(T* p, double v) { Ty<T>::st(p, (typename Ty<T>::C)v); }

// Block index -> grid: largest g with block0[g] <= bid (block0 has n+1 entries).
__device__ __forceinline__ int find_grid(const int64_t* __restrict__ block0, int n, int64_t bid) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (block0[mid] <= bid) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace gd
