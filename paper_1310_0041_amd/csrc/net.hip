// gfx950 kernels of the learned preconditioner: a small 2-D U-Net of 3x3
// convolutions that maps a normalised multigrid residual to an estimate of
// the error.  Activations are bf16, channel-fastest ([b][y][x][c], a pixel
// stride >= the channel count so that skip connections can live in the
// channel range of a concatenation buffer); arithmetic accumulates in FP32 on
// the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Convolution as an implicit GEMM: out[co][p] = sum_k W[co][k] * col[k][p],
// k = tap * Cin + ci, tap = 3 * dy + dx, col[k][p] = in[p + (dy - 1, dx - 1)][ci]
// with zero padding.  MFMA operand layouts (16x16x32 bf16): A[i][k] sits in
// lane i + 16 (k / 8), element k % 8; B[k][j] in lane j + 16 (k / 8),
// element k % 8; D[i][j] in lane j + 16 (i / 4), element i % 4.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>

#include "gd_net.h"

namespace gd {
namespace net {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __hip_bfloat16 bf;

// Drain the matrix cores before the accumulators are read.  The compiler
// spaces an accumulator read from the MFMA that produced it by fewer wait
// states than the last result register of a 16x16x32 MFMA needs on gfx950
// (that register was read stale when the read came right after a loop
// exit); 24 idle cycles here, with the accumulators as operands so that no
// read is scheduled before them.
__device__ __forceinline__ void mfma_drain(v4f& a) {
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(a));
}

// Elementwise kernels walk their index space with a grid stride: a full
// stack of slices can exceed what one launch may address per thread.
#define GRID_STRIDE(i, n) for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < (n); i += (int64_t)gridDim.x * 256)

__device__ __forceinline__ float b2f(bf v) { return __bfloat162float(v); }
__device__ __forceinline__ bf f2b(float v) { return __float2bfloat16(v); }

// ------------------------------------------------------------ convolution
//
// Block: a 64-pixel segment of CONV_RB consecutive rows of one image, all
// output channels, marching down the rows.  The three input rows a row
// needs (66 pixels, all channels) sit in an LDS ring; each new row is read
// into registers while the current one is computed and enters LDS after.
// The 4 waves split the work into WP pixel groups x WM output-channel groups
// (WP * WM = 4); a wave keeps its weight fragments (A operands) for all
// k-steps in registers for the whole block and reads only activations (B
// operands) from LDS.
// in: pixel stride in_s, channel offset in_o; out likewise (bf16 or fp32);
// mask (optional, bf16 view): the result is zeroed where mask <= 0 (ReLU'
// of the layer that produced this layer's input, for the data gradient).
// With in2 set, the input is a concatenation read in place: channels
// [0, cup) are `in` at half resolution, nearest up-sampled (pixel (y, x)
// reads (y / 2, x / 2) of an H/2 x W/2 image), and [cup, CIN) are in2
// (stride in2_s, offset in2_o) at full resolution.
constexpr int CONV_RB = 16;

template <int CIN, int COUT, bool RIN>
__global__ void __launch_bounds__(256)
k_conv3x3(const bf* __restrict__ in, int in_s, int in_o, const bf* __restrict__ W, const float* __restrict__ bias,
          int relu, bf* __restrict__ out_b, float* __restrict__ out_f, int out_s, int out_o, int cstore,
          const bf* __restrict__ mask, int mask_s, int mask_o, int H, int Wd, const bf* __restrict__ in2,
          int in2_s, int in2_o, int cup, const float* __restrict__ rin, const float* __restrict__ rscale,
          const float* __restrict__ oscale) {
  // rin (CIN == 8): the input is the FP32 residual image itself, channel 0 =
  // rin * rscale[image], channels 1..7 = 0.  oscale (FP32 output): the stored
  // value is multiplied by oscale[image].
  constexpr int K = 9 * CIN;
  constexpr int KPAD = (K + 31) / 32 * 32;
  constexpr int KS = KPAD / 32;
  constexpr int MT = COUT / 16;
  constexpr int WM = (MT % 4 == 0) ? 4 : (MT % 2 == 0) ? 2 : 1;  // output-channel groups
  constexpr int WP = 4 / WM;                                      // pixel groups
  constexpr int NPT = 4 / WP;                                     // 16-pixel tiles per wave
  constexpr int MTW = MT / WM;                                    // 16-channel tiles per wave
  constexpr int CH = CIN / 8;                                     // 16-byte chunks per pixel
  constexpr int NCH = (66 * CH + 255) / 256;                      // chunks of a row per thread
  static_assert(CIN % 8 == 0 && COUT % 16 == 0, "channel padding");
  __shared__ __attribute__((aligned(16))) bf T[3][66][CIN];

  const int segs = Wd / 64;
  const int rblk = (H + CONV_RB - 1) / CONV_RB;
  const int seg = blockIdx.x % segs;
  const int y0 = ((blockIdx.x / segs) % rblk) * CONV_RB;
  const int b = blockIdx.x / (segs * rblk);
  const int x0 = seg * 64;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
  const int j = l & 15, kg = l >> 4;
  const int wp = w % WP, wm = w / WP;

  // weight fragments of this wave: rows 16 (wm MTW + mt) + j, k = 32 s + 8 kg
  v8bf A[MTW][KS];
#pragma unroll
  for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
    for (int s = 0; s < KS; ++s)
      A[mt][s] = *reinterpret_cast<const v8bf*>(W + (int64_t)(16 * (wm * MTW + mt) + j) * KPAD + 32 * s + 8 * kg);

  // row staging: chunk c of a row = pixel c / CH (x0 - 1 + pixel), channels 8 (c % CH)
  uint4 R[NCH];
  auto fetch_row = [&](int yy) {
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = tid + 256 * q;
      const int px = c / CH, c8 = c - px * CH, xx = x0 + px - 1;
      R[q] = make_uint4(0, 0, 0, 0);
      if constexpr (RIN) {  // CH == 1: one chunk per pixel
        if (c < 66 && yy >= 0 && yy < H && xx >= 0 && xx < Wd) {
          const float v = rin[(int64_t)(b * H + yy) * Wd + xx] * rscale[b];
          R[q].x = (uint32_t)__builtin_bit_cast(uint16_t, f2b(v));
        }
      } else if (c < 66 * CH && yy >= 0 && yy < H && xx >= 0 && xx < Wd) {
        const bf* src;
        if (!in2) src = in + ((int64_t)(b * H + yy) * Wd + xx) * in_s + in_o + 8 * c8;
        else if (8 * c8 < cup) src = in + ((int64_t)(b * (H / 2) + yy / 2) * (Wd / 2) + xx / 2) * in_s + in_o + 8 * c8;
        else src = in2 + ((int64_t)(b * H + yy) * Wd + xx) * in2_s + in2_o + 8 * c8 - cup;
        R[q] = *reinterpret_cast<const uint4*>(src);
      }
    }
  };
  auto store_row = [&](int yy) {
    bf* P = &T[(yy + 3) % 3][0][0];
#pragma unroll
    for (int q = 0; q < NCH; ++q) {
      const int c = tid + 256 * q;
      if (c < 66 * CH) *reinterpret_cast<uint4*>(P + 8 * c) = R[q];
    }
  };
  fetch_row(y0 - 1);
  store_row(y0 - 1);
  fetch_row(y0);
  store_row(y0);
  fetch_row(y0 + 1);

  const int yend = min(y0 + CONV_RB, H);
  for (int y = y0; y < yend; ++y) {
    store_row(y + 1);
    __syncthreads();
    if (y + 2 < yend + 1) fetch_row(y + 2);  // uniform: the next row's input, in flight during the products
    v4f acc[NPT][MTW];
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt) acc[t][mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 32 * s + 8 * kg;
      const int tap = k / CIN, ci = k - tap * CIN;
      const int dy = tap / 3, dx = tap - 3 * dy;
      const bool kin = k < K;
#pragma unroll
      for (int t = 0; t < NPT; ++t) {
        const int px = 16 * (wp * NPT + t) + j;
        v8bf bv = v8bf{0, 0, 0, 0, 0, 0, 0, 0};
        if (kin) bv = *reinterpret_cast<const v8bf*>(&T[(y - 1 + dy + 3) % 3][px + dx][ci]);
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) acc[t][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][s], bv, acc[t][mt], 0, 0, 0);
      }
    }
    // the last product issued finishes last: drain it, and keep every read
    // of the other accumulators behind the drain
    mfma_drain(acc[NPT - 1][MTW - 1]);
#pragma unroll
    for (int t = 0; t < NPT; ++t)
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt) asm volatile("" : "+a"(acc[t][mt]));
    // a lane holds 4 consecutive output channels of one pixel: written (and
    // masked) 8 bytes at a time when all four are stored
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
      const int x = x0 + 16 * (wp * NPT + t) + j;
      const int64_t pix = (int64_t)(b * H + y) * Wd + x;
#pragma unroll
      for (int mt = 0; mt < MTW; ++mt) {
        const int co0 = 16 * (wm * MTW + mt) + 4 * kg;
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          v[e] = acc[t][mt][e] + ((bias && co0 + e < cstore) ? bias[co0 + e] : 0.f);  // bias has cstore entries
          if (relu) v[e] = fmaxf(v[e], 0.f);
        }
        if (co0 + 3 < cstore && !out_f) {
          if (mask) {
            const uint2 m = *reinterpret_cast<const uint2*>(mask + pix * mask_s + mask_o + co0);
            const uint32_t mw[2] = {m.x, m.y};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const uint32_t bits = (e & 1) ? (mw[e >> 1] & 0xffff0000u) : (mw[e >> 1] << 16);
              v[e] = (__uint_as_float(bits) > 0.f) ? v[e] : 0.f;
            }
          }
          const uint32_t w0 = (uint32_t)__builtin_bit_cast(uint16_t, f2b(v[0])) |
                              ((uint32_t)__builtin_bit_cast(uint16_t, f2b(v[1])) << 16);
          const uint32_t w1 = (uint32_t)__builtin_bit_cast(uint16_t, f2b(v[2])) |
                              ((uint32_t)__builtin_bit_cast(uint16_t, f2b(v[3])) << 16);
          *reinterpret_cast<uint2*>(out_b + pix * out_s + out_o + co0) = make_uint2(w0, w1);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int co = co0 + e;
            if (co >= cstore) continue;
            float u = v[e];
            if (mask) u = (b2f(mask[pix * mask_s + mask_o + co]) > 0.f) ? u : 0.f;
            if (out_f) out_f[pix * out_s + out_o + co] = oscale ? u * oscale[b] : u;
            else out_b[pix * out_s + out_o + co] = f2b(u);
          }
        }
      }
    }
    __syncthreads();  // the ring slot of row y - 1 is rewritten next
  }
}

// ------------------------------------------------------- weight gradient
//
// dW[co][k] = sum_p dout[p][co] * col[k][p]: an MFMA GEMM with the pixels as
// the reduction axis.  Block = (image b, rows y0 .. y0 + R) x (group of 32
// output tiles of 16 x 16); per 64-pixel segment, dout is staged transposed
// ([co][px]) and the three input rows as [row][ci][px] in LDS.  Each wave
// owns 8 tiles; the block's partial sums go to partial[chunk][co][k] and a
// second kernel adds the chunks in a fixed order.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256)
k_conv3x3_wgrad(const bf* __restrict__ in, int in_s, int in_o, const bf* __restrict__ dout, int d_s, int d_o,
                float* __restrict__ partial, int H, int Wd, int R) {
  constexpr int K = 9 * CIN;
  constexpr int KPAD = (K + 31) / 32 * 32;
  constexpr int NT = KPAD / 16, MT = COUT / 16;
  constexpr int TILES = MT * NT;
  constexpr int GROUPS = (TILES + 31) / 32;
  __shared__ __attribute__((aligned(16))) bf D[COUT][64];
  __shared__ __attribute__((aligned(16))) bf I[3][CIN][72];

  const int grp = blockIdx.x % GROUPS;
  const int chunk = blockIdx.x / GROUPS;
  const int rchunks = (H + R - 1) / R;
  const int b = chunk / rchunks, y0 = (chunk % rchunks) * R;
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int j = l & 15, kg = l >> 4;
  // Every wave runs all 8 of its tile products without branches (tiles past
  // the end repeat the last one and are not stored): a branch around an MFMA
  // left the last accumulator register read before its result was complete.
  v4f acc[8];
  int tm[8], tn[8];
  bool live[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tile = grp * 32 + w * 8 + t;
    live[t] = tile < TILES;
    const int tc = live[t] ? tile : TILES - 1;
    tm[t] = tc / NT;
    tn[t] = tc % NT;
    acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  }
  // one flat loop over (row, segment): no loop nest whose exit reads the
  // accumulators in the middle of the work
  const int nseg = Wd / 64, nrow = min(y0 + R, H) - y0;
  for (int it = 0; it < nrow * nseg; ++it) {
    {
      const int y = y0 + it / nseg, x0 = (it % nseg) * 64;
      __syncthreads();
      for (int i = tid; i < 64 * COUT; i += 256) {  // dout[p][co] -> D[co][p]
        const int co = i % COUT, px = i / COUT;
        D[co][px] = dout[((int64_t)(b * H + y) * Wd + x0 + px) * d_s + d_o + co];
      }
      for (int i = tid; i < 3 * 66 * CIN; i += 256) {  // in -> I[row][ci][px]
        const int ci = i % CIN, px = (i / CIN) % 66, r = i / (CIN * 66);
        const int yy = y + r - 1, xx = x0 + px - 1;
        bf v = f2b(0.f);
        if (yy >= 0 && yy < H && xx >= 0 && xx < Wd) v = in[((int64_t)(b * H + yy) * Wd + xx) * in_s + in_o + ci];
        I[r][ci][px] = v;
      }
      __syncthreads();
#pragma unroll
      for (int ps = 0; ps < 64; ps += 32) {  // two MFMA steps of 32 pixels
        const int p = ps + 8 * kg;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const int co = 16 * tm[t] + j;
          const v8bf av = *reinterpret_cast<const v8bf*>(&D[co][p]);
          const int k = 16 * tn[t] + j;
          v8bf bv = v8bf{0, 0, 0, 0, 0, 0, 0, 0};
          if (k < K) {
            const int tap = k / CIN, ci = k - tap * CIN;
            const int dy = tap / 3, dx = tap - 3 * dy;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = __builtin_bit_cast(__bf16, I[dy][ci][p + e + dx]);
          }
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
  }
  mfma_drain(acc[7]);
#pragma unroll
  for (int t = 0; t < 7; ++t) asm volatile("" : "+a"(acc[t]));
  float* P = partial + (int64_t)chunk * COUT * KPAD;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (!live[t]) continue;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int co = 16 * tm[t] + 4 * kg + e, k = 16 * tn[t] + j;
      P[(int64_t)co * KPAD + k] = acc[t][e];
    }
  }
}

// sum over chunks in order; n = COUT * KPAD
__global__ void __launch_bounds__(256)
k_sum_chunks(const float* __restrict__ partial, int nchunks, int n, float* __restrict__ out) {
  GRID_STRIDE(i, n) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += partial[(int64_t)c * n + i];
    out[i] = s;
  }
}

// bias gradient: db[co] = sum over pixels of dout[p][co]; block partials per co
__global__ void __launch_bounds__(256)
k_bias_grad(const bf* __restrict__ dout, int d_s, int d_o, int cout, int64_t npix, float* __restrict__ partial) {
  // block b sums pixels b, b + gridDim, ... for every channel; thread = channel lane
  __shared__ float red[256];
  const int co = threadIdx.x % 64, lane_grp = threadIdx.x / 64;
  float s = 0.f;
  if (co < cout)
    for (int64_t p = (int64_t)blockIdx.x * 4 + lane_grp; p < npix; p += (int64_t)gridDim.x * 4)
      s += b2f(dout[p * d_s + d_o + co]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64) {
    const float t = red[threadIdx.x] + red[threadIdx.x + 64] + red[threadIdx.x + 128] + red[threadIdx.x + 192];
    if (co < cout) partial[(int64_t)blockIdx.x * 64 + co] = t;
  }
}

// ------------------------------------------------------------- glue

// Channels move in groups of 8 (16 bytes): every channel count, stride and
// offset of these views is a multiple of 8.
struct V8 {
  float v[8];
};
__device__ __forceinline__ V8 ld8(const bf* p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
  V8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r.v[2 * i] = __uint_as_float(w[i] << 16);
    r.v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
  return r;
}
__device__ __forceinline__ void st8(bf* p, const V8& r) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t lo = __builtin_bit_cast(uint16_t, f2b(r.v[2 * i]));
    const uint32_t hi = __builtin_bit_cast(uint16_t, f2b(r.v[2 * i + 1]));
    w[i] = lo | (hi << 16);
  }
  *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
}

// average pool 2x2: out (H/2 x W/2) from in (H x W), C channels
__global__ void k_pool(const bf* __restrict__ in, int in_s, int in_o, bf* __restrict__ out, int out_s, int out_o,
                       int C, int B, int H, int Wd) {
  const int h = H / 2, w = Wd / 2, G = C / 8;
  GRID_STRIDE(i, (int64_t)B * h * w * G) {
    const int c = (int)(i % G) * 8;
    const int64_t q = i / G;
    const int x = q % w, y = (q / w) % h, b = q / ((int64_t)w * h);
    V8 s;
#pragma unroll
    for (int e = 0; e < 8; ++e) s.v[e] = 0.f;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const V8 t = ld8(in + ((int64_t)(b * H + 2 * y + dy) * Wd + 2 * x + dx) * in_s + in_o + c);
#pragma unroll
        for (int e = 0; e < 8; ++e) s.v[e] += t.v[e];
      }
#pragma unroll
    for (int e = 0; e < 8; ++e) s.v[e] *= 0.25f;
    st8(out + ((int64_t)(b * h + y) * w + x) * out_s + out_o + c, s);
  }
}

// pool backward, accumulated: din(2y+dy, 2x+dx) += dout(y, x) / 4
__global__ void k_pool_bwd_acc(const bf* __restrict__ dout, int d_s, int d_o, bf* __restrict__ din, int i_s, int i_o,
                               int C, int B, int H, int Wd) {
  const int G = C / 8;
  GRID_STRIDE(i, (int64_t)B * H * Wd * G) {
    const int c = (int)(i % G) * 8;
    const int64_t q = i / G;
    const int x = q % Wd, y = (q / Wd) % H, b = q / ((int64_t)Wd * H);
    const V8 g = ld8(dout + ((int64_t)(b * (H / 2) + y / 2) * (Wd / 2) + x / 2) * d_s + d_o + c);
    bf* p = din + ((int64_t)(b * H + y) * Wd + x) * i_s + i_o + c;
    V8 t = ld8(p);
#pragma unroll
    for (int e = 0; e < 8; ++e) t.v[e] += 0.25f * g.v[e];
    st8(p, t);
  }
}

// nearest up-sampling x2: out (H x W) from in (H/2 x W/2)
__global__ void k_up(const bf* __restrict__ in, int in_s, int in_o, bf* __restrict__ out, int out_s, int out_o, int C,
                     int B, int H, int Wd) {
  const int G = C / 8;
  GRID_STRIDE(i, (int64_t)B * H * Wd * G) {
    const int c = (int)(i % G) * 8;
    const int64_t q = i / G;
    const int x = q % Wd, y = (q / Wd) % H, b = q / ((int64_t)Wd * H);
    *reinterpret_cast<uint4*>(out + ((int64_t)(b * H + y) * Wd + x) * out_s + out_o + c) =
        *reinterpret_cast<const uint4*>(in + ((int64_t)(b * (H / 2) + y / 2) * (Wd / 2) + x / 2) * in_s + in_o + c);
  }
}

// up-sampling backward: din(y, x) = sum of the 4 children of dout, times the
// ReLU' mask of the up-sampled activation's producer (mask view, may be NULL)
__global__ void k_up_bwd(const bf* __restrict__ dout, int d_s, int d_o, bf* __restrict__ din, int i_s, int i_o,
                         const bf* __restrict__ mask, int m_s, int m_o, int C, int B, int H, int Wd) {
  const int h = H / 2, w = Wd / 2, G = C / 8;
  GRID_STRIDE(i, (int64_t)B * h * w * G) {
    const int c = (int)(i % G) * 8;
    const int64_t q = i / G;
    const int x = q % w, y = (q / w) % h, b = q / ((int64_t)w * h);
    V8 s;
#pragma unroll
    for (int e = 0; e < 8; ++e) s.v[e] = 0.f;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const V8 t = ld8(dout + ((int64_t)(b * H + 2 * y + dy) * Wd + 2 * x + dx) * d_s + d_o + c);
#pragma unroll
        for (int e = 0; e < 8; ++e) s.v[e] += t.v[e];
      }
    const int64_t pix = (int64_t)(b * h + y) * w + x;
    if (mask) {
      const V8 m = ld8(mask + pix * m_s + m_o + c);
#pragma unroll
      for (int e = 0; e < 8; ++e) s.v[e] = (m.v[e] > 0.f) ? s.v[e] : 0.f;
    }
    st8(din + pix * i_s + i_o + c, s);
  }
}

// g *= (act > 0) in place
__global__ void k_relu_mask(bf* __restrict__ g, int g_s, int g_o, const bf* __restrict__ act, int a_s, int a_o, int C,
                            int64_t npix) {
  const int G = C / 8;
  GRID_STRIDE(i, npix * G) {
    const int c = (int)(i % G) * 8;
    const int64_t p = i / G;
    bf* gp = g + p * g_s + g_o + c;
    V8 t = ld8(gp);
    const V8 m = ld8(act + p * a_s + a_o + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) t.v[e] = (m.v[e] > 0.f) ? t.v[e] : 0.f;
    st8(gp, t);
  }
}

// input: channel 0 = r * inv_scale[b], channels 1..7 = 0 (C == 8)
__global__ void k_pack_input(const float* __restrict__ r, const float* __restrict__ inv_scale, bf* __restrict__ out,
                             int C, int64_t npix_img, int B) {
  GRID_STRIDE(p, npix_img * B) {
    const int b = (int)(p / npix_img);
    const uint32_t lo = __builtin_bit_cast(uint16_t, f2b(r[p] * inv_scale[b]));
    *reinterpret_cast<uint4*>(out + p * C) = make_uint4(lo, 0u, 0u, 0u);
  }
}


// loss = mean (y - e * inv_scale)^2 over pixels; dy = 2 (y - t) / npix into a
// bf16 gradient view (channel 0; the other channels are zeroed)
__global__ void __launch_bounds__(256)
k_loss(const float* __restrict__ y, int y_s, const float* __restrict__ e, const float* __restrict__ inv_scale,
       bf* __restrict__ dy, int d_s, int C, int64_t npix_img, int B, double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t N = npix_img * B;
  double l = 0.0;
  GRID_STRIDE(p, N) {
    const float t = e[p] * inv_scale[(int)(p / npix_img)];
    const float d = y[p * y_s] - t;
    l += (double)d * d;
    dy[p * d_s] = f2b(2.f * d / (float)N);
    for (int c = 1; c < C; ++c) dy[p * d_s + c] = f2b(0.f);
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] / (double)N;
}

// Adam on FP32 master parameters
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// pack FP32 master weights [cout][cin][3][3] (real channel counts) into the
// MFMA operand [COUTP][KPAD] (k = tap * CINP + ci); transpose = 1 packs the
// data-gradient operand: W'[ci][co] with the taps flipped (tap' = 8 - tap)
__global__ void k_pack_w(const float* __restrict__ w, int cout, int cin, bf* __restrict__ out, int rows, int cinp,
                         int kpad, int transpose) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * kpad) return;
  const int row = i / kpad, k = i % kpad;
  float v = 0.f;
  if (k < 9 * cinp) {
    const int tap = k / cinp, c = k % cinp;
    if (!transpose) {
      if (row < cout && c < cin) v = w[((row * cin) + c) * 9 + tap];
    } else {  // row = input channel of the layer, c = its output channel
      if (row < cin && c < cout) v = w[((c * cin) + row) * 9 + (8 - tap)];
    }
  }
  out[i] = f2b(v);
}

// gradient [COUTP][KPAD] (k = tap * CINP + ci) -> FP32 [cout][cin][3][3]
__global__ void k_unpack_wgrad(const float* __restrict__ g, int cout, int cin, int cinp, int kpad, float* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= cout * cin * 9) return;
  const int tap = i % 9, c = (i / 9) % cin, co = i / (9 * cin);
  out[i] = g[(int64_t)co * kpad + tap * cinp + c];
}

// ============================================================ launchers

// blocks for n elements of a grid-stride kernel (at most 2^20 blocks)
static inline unsigned nb(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, (int64_t)1 << 20); }

#define CONV_CASES(X) X(8, 16) X(16, 16) X(16, 32) X(32, 32) X(32, 64) X(64, 64) X(96, 32) X(48, 16) X(32, 16) \
  X(64, 32) X(32, 96) X(16, 48)

hipError_t conv(int cin, int cout, const bf* in, int in_s, int in_o, const bf* W, const float* bias, int relu,
                bf* out_b, float* out_f, int out_s, int out_o, int cstore, const bf* mask, int mask_s, int mask_o,
                int B, int H, int Wd, hipStream_t st, const bf* in2, int in2_s, int in2_o, int cup,
                const float* rin, const float* rscale, const float* oscale) {
  if (Wd % 64 || (in2 && (cup % 8 || cup <= 0 || cup >= cin || H % 2)) || (rin && (cin != 8 || !rscale)))
    return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((int64_t)B * ((H + CONV_RB - 1) / CONV_RB) * (Wd / 64));
  if (rin) {
    if (cin != 8 || cout != 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_conv3x3<8, 16, true>), dim3(grid), dim3(256), 0, st, in, in_s, in_o, W, bias, relu, out_b,
                       out_f, out_s, out_o, cstore, mask, mask_s, mask_o, H, Wd, in2, in2_s, in2_o, cup, rin, rscale,
                       oscale);
    return hipGetLastError();
  }
#define X(CI, CO)                                                                                              \
  if (cin == CI && cout == CO) {                                                                               \
    hipLaunchKernelGGL((k_conv3x3<CI, CO, false>), dim3(grid), dim3(256), 0, st, in, in_s, in_o, W, bias, relu, \
                       out_b, out_f, out_s, out_o, cstore, mask, mask_s, mask_o, H, Wd, in2, in2_s, in2_o, cup,  \
                       rin, rscale, oscale);                                                                   \
    return hipGetLastError();                                                                                  \
  }
  CONV_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

int wgrad_groups(int cin, int cout) {
  const int kpad = (9 * cin + 31) / 32 * 32;
  return ((cout / 16) * (kpad / 16) + 31) / 32;
}

hipError_t wgrad(int cin, int cout, const bf* in, int in_s, int in_o, const bf* dout, int d_s, int d_o,
                 float* partial, int B, int H, int Wd, int R, hipStream_t st) {
  if (Wd % 64) return hipErrorInvalidValue;
  const int chunks = B * ((H + R - 1) / R);
  const unsigned grid = (unsigned)(chunks * wgrad_groups(cin, cout));
#define X(CI, CO)                                                                                            \
  if (cin == CI && cout == CO) {                                                                             \
    hipLaunchKernelGGL((k_conv3x3_wgrad<CI, CO>), dim3(grid), dim3(256), 0, st, in, in_s, in_o, dout, d_s,   \
                       d_o, partial, H, Wd, R);                                                              \
    return hipGetLastError();                                                                                \
  }
  CONV_CASES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t sum_chunks(const float* partial, int nchunks, int n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_chunks, dim3(nb(n)), dim3(256), 0, st, partial, nchunks, n, out);
  return hipGetLastError();
}
hipError_t bias_grad(const bf* dout, int d_s, int d_o, int cout, int64_t npix, float* partial, int nblocks,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_bias_grad, dim3(nblocks), dim3(256), 0, st, dout, d_s, d_o, cout, npix, partial);
  return hipGetLastError();
}
hipError_t pool(const bf* in, int in_s, int in_o, bf* out, int out_s, int out_o, int C, int B, int H, int Wd,
                hipStream_t st) {
  hipLaunchKernelGGL(k_pool, dim3(nb((int64_t)B * (H / 2) * (Wd / 2) * (C / 8))), dim3(256), 0, st, in, in_s, in_o, out,
                     out_s, out_o, C, B, H, Wd);
  return hipGetLastError();
}
hipError_t pool_bwd_acc(const bf* dout, int d_s, int d_o, bf* din, int i_s, int i_o, int C, int B, int H, int Wd,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_pool_bwd_acc, dim3(nb((int64_t)B * H * Wd * (C / 8))), dim3(256), 0, st, dout, d_s, d_o, din, i_s,
                     i_o, C, B, H, Wd);
  return hipGetLastError();
}
hipError_t up(const bf* in, int in_s, int in_o, bf* out, int out_s, int out_o, int C, int B, int H, int Wd,
              hipStream_t st) {
  hipLaunchKernelGGL(k_up, dim3(nb((int64_t)B * H * Wd * (C / 8))), dim3(256), 0, st, in, in_s, in_o, out, out_s, out_o, C,
                     B, H, Wd);
  return hipGetLastError();
}
hipError_t up_bwd(const bf* dout, int d_s, int d_o, bf* din, int i_s, int i_o, const bf* mask, int m_s, int m_o, int C,
                  int B, int H, int Wd, hipStream_t st) {
  hipLaunchKernelGGL(k_up_bwd, dim3(nb((int64_t)B * (H / 2) * (Wd / 2) * (C / 8))), dim3(256), 0, st, dout, d_s, d_o, din,
                     i_s, i_o, mask, m_s, m_o, C, B, H, Wd);
  return hipGetLastError();
}
hipError_t relu_mask(bf* g, int g_s, int g_o, const bf* act, int a_s, int a_o, int C, int64_t npix, hipStream_t st) {
  hipLaunchKernelGGL(k_relu_mask, dim3(nb(npix * (C / 8))), dim3(256), 0, st, g, g_s, g_o, act, a_s, a_o, C, npix);
  return hipGetLastError();
}
hipError_t pack_input(const float* r, const float* inv_scale, bf* out, int C, int64_t npix_img, int B,
                      hipStream_t st) {
  if (C != 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_input, dim3(nb(npix_img * B)), dim3(256), 0, st, r, inv_scale, out, C, npix_img, B);
  return hipGetLastError();
}
hipError_t loss(const float* y, int y_s, const float* e, const float* inv_scale, bf* dy, int d_s, int C,
                int64_t npix_img, int B, double* partial, int* nblocks, hipStream_t st) {
  *nblocks = (int)nb(npix_img * B);
  hipLaunchKernelGGL(k_loss, dim3(*nblocks), dim3(256), 0, st, y, y_s, e, inv_scale, dy, d_s, C, npix_img, B, partial);
  return hipGetLastError();
}
hipError_t adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t pack_w(const float* w, int cout, int cin, bf* out, int rows, int cinp, int kpad, int transpose,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_pack_w, dim3(nb((int64_t)rows * kpad)), dim3(256), 0, st, w, cout, cin, out, rows, cinp, kpad,
                     transpose);
  return hipGetLastError();
}
hipError_t unpack_wgrad(const float* g, int cout, int cin, int cinp, int kpad, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_unpack_wgrad, dim3(nb((int64_t)cout * cin * 9)), dim3(256), 0, st, g, cout, cin, cinp, kpad, out);
  return hipGetLastError();
}

}  // namespace net
}  // namespace gd
