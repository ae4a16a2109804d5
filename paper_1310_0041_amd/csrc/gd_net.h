// Launchers of the learned-preconditioner kernels (net.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace gd {
namespace net {

typedef __hip_bfloat16 bf;

// 3x3 convolution, zero padding; cin/cout are the padded channel counts of a
// supported layer shape.  out_b (bf16) or out_f (fp32) receives channels
// [0, cstore); relu applies max(0, .); mask (may be NULL) zeroes outputs
// where the mask view is <= 0.
hipError_t conv(int cin, int cout, const bf* in, int in_s, int in_o, const bf* W, const float* bias, int relu,
                bf* out_b, float* out_f, int out_s, int out_o, int cstore, const bf* mask, int mask_s, int mask_o,
                int B, int H, int Wd, hipStream_t st, const bf* in2 = nullptr, int in2_s = 0, int in2_o = 0,
                int cup = 0, const float* rin = nullptr, const float* rscale = nullptr,
                const float* oscale = nullptr);
int wgrad_groups(int cin, int cout);
hipError_t wgrad(int cin, int cout, const bf* in, int in_s, int in_o, const bf* dout, int d_s, int d_o,
                 float* partial, int B, int H, int Wd, int R, hipStream_t st);
hipError_t sum_chunks(const float* partial, int nchunks, int n, float* out, hipStream_t st);
hipError_t bias_grad(const bf* dout, int d_s, int d_o, int cout, int64_t npix, float* partial, int nblocks,
                     hipStream_t st);
hipError_t pool(const bf* in, int in_s, int in_o, bf* out, int out_s, int out_o, int C, int B, int H, int Wd,
                hipStream_t st);
hipError_t pool_bwd_acc(const bf* dout, int d_s, int d_o, bf* din, int i_s, int i_o, int C, int B, int H, int Wd,
                        hipStream_t st);
hipError_t up(const bf* in, int in_s, int in_o, bf* out, int out_s, int out_o, int C, int B, int H, int Wd,
              hipStream_t st);
hipError_t up_bwd(const bf* dout, int d_s, int d_o, bf* din, int i_s, int i_o, const bf* mask, int m_s, int m_o, int C,
                  int B, int H, int Wd, hipStream_t st);
hipError_t relu_mask(bf* g, int g_s, int g_o, const bf* act, int a_s, int a_o, int C, int64_t npix, hipStream_t st);
hipError_t pack_input(const float* r, const float* inv_scale, bf* out, int C, int64_t npix_img, int B,
                      hipStream_t st);
hipError_t loss(const float* y, int y_s, const float* e, const float* inv_scale, bf* dy, int d_s, int C,
                int64_t npix_img, int B, double* partial, int* nblocks, hipStream_t st);
hipError_t adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, float c1,
                float c2, hipStream_t st);
hipError_t pack_w(const float* w, int cout, int cin, bf* out, int rows, int cinp, int kpad, int transpose,
                  hipStream_t st);
hipError_t unpack_wgrad(const float* g, int cout, int cin, int cinp, int kpad, float* out, hipStream_t st);

}  // namespace net
}  // namespace gd
