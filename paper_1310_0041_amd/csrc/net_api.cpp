// Host side of the learned preconditioner: a 3-level U-Net of 3x3
// convolutions (16 / 32 / 64 channels, average-pool down, nearest up,
// concatenated skips), BF16 weights and activations, FP32 accumulation and
// FP32 master weights with Adam.  It maps a residual r (normalised to unit
// RMS per image) to an estimate of the multigrid error e, and is used as a
// preconditioner z = N(r / s) * s inside flexible CG.
//
// Layers (input -> output channels; level = resolution / 2^level):
//   0 L1a 1->16  (relu)   level 0       5 L3b 64->64 (relu)  level 2
//   1 L1b 16->16 (relu)   level 0, skip  6 L4  96->32 (relu)  level 1 (up(L3b) ++ skip L2b)
//   2 L2a 16->32 (relu)   level 1        7 L5  48->16 (relu)  level 0 (up(L4) ++ skip L1b)
//   3 L2b 32->32 (relu)   level 1, skip  8 L6  16->1  (linear) level 0
//   4 L3a 32->64 (relu)   level 2
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gd.h"
#include "gd_net.h"

using gd::net::bf;

namespace {

thread_local std::string t_err;
gd_status nfail(gd_status s, const std::string& m) {
  t_err = m;
  return s;
}

struct HipErr {
  hipError_t e;
  const char* what;
};
#define NT_TRY(call)                                 \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) throw HipErr{e_, #call};   \
  } while (0)

struct LayerSpec {
  int cin, cout, cinp, coutp;
};
const LayerSpec kLayers[9] = {{1, 16, 8, 16},  {16, 16, 16, 16}, {16, 32, 16, 32},
                              {32, 32, 32, 32}, {32, 64, 32, 64}, {64, 64, 64, 64},
                              {96, 32, 96, 32}, {48, 16, 48, 16}, {16, 1, 16, 16}};

int kpad_of(int cinp) { return (9 * cinp + 31) / 32 * 32; }

// splitmix64 for the initial weights
uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

struct Buf {  // device allocation owned by the net
  void* p = nullptr;
  size_t n = 0;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  void ensure(size_t bytes) {
    if (bytes <= n) return;
    if (p) NT_TRY(hipFree(p));
    p = nullptr;
    NT_TRY(hipMalloc(&p, bytes));
    n = bytes;
  }
  template <typename T> T* as() { return (T*)p; }
};

}  // namespace

struct gd_net {
  int64_t nparam = 0;
  size_t woff[9], boff[9];
  Buf master, grad, m, v, wpk[9], wpkT[9];
  int step = 0;
  // per-shape activations / gradients
  int B = 0, H = 0, W = 0;
  Buf X0, A1, C1, P1, A2, C2, P2, A3, A3b, A4, A5, Y;
  Buf S1, S2;  // forward-only: the skip activations L1b / L2b, contiguous
  Buf dY, dA5, dC1, dA4, dC2, dA3b, dA3, dP2, dA2, dP1, dA1;
  Buf part, bpart, gpk, scale, lpart;
  std::vector<double> hl;
  // optional HIP-event timing of the forward convolutions, per layer
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> ev_layer;
  std::vector<double> ev_flops;
  size_t ev_used = 0;
  double t_ms[9] = {}, t_flops[9] = {};
  int64_t t_cnt[9] = {};
  ~gd_net() {
    for (auto& p : ev) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  }
  void harvest() {  // after the stream has been synchronised
    for (size_t i = 0; i < ev_used; ++i) {
      float ms = 0.f;
      NT_TRY(hipEventElapsedTime(&ms, ev[i].first, ev[i].second));
      t_ms[ev_layer[i]] += ms;
      t_flops[ev_layer[i]] += ev_flops[i];
      t_cnt[ev_layer[i]] += 1;
    }
    ev_used = 0;
  }

  void layout() {
    size_t o = 0;
    for (int l = 0; l < 9; ++l) {
      woff[l] = o;
      o += (size_t)kLayers[l].cout * kLayers[l].cin * 9;
    }
    for (int l = 0; l < 9; ++l) {
      boff[l] = o;
      o += kLayers[l].cout;
    }
    nparam = (int64_t)o;
  }
  void alloc_params() {
    master.ensure(nparam * 4);
    grad.ensure(nparam * 4);
    m.ensure(nparam * 4);
    v.ensure(nparam * 4);
    NT_TRY(hipMemset(m.p, 0, nparam * 4));
    NT_TRY(hipMemset(v.p, 0, nparam * 4));
    for (int l = 0; l < 9; ++l) {
      const LayerSpec& L = kLayers[l];
      wpk[l].ensure((size_t)L.coutp * kpad_of(L.cinp) * 2);
      const int rows = (L.cin + 15) / 16 * 16;
      wpkT[l].ensure((size_t)rows * kpad_of(L.coutp) * 2);
    }
  }
  void pack(hipStream_t st) {
    for (int l = 0; l < 9; ++l) {
      const LayerSpec& L = kLayers[l];
      const float* w = master.as<float>() + woff[l];
      NT_TRY(gd::net::pack_w(w, L.cout, L.cin, wpk[l].as<bf>(), L.coutp, L.cinp, kpad_of(L.cinp), 0, st));
      const int rows = (L.cin + 15) / 16 * 16;
      NT_TRY(gd::net::pack_w(w, L.cout, L.cin, wpkT[l].as<bf>(), rows, L.coutp, kpad_of(L.coutp), 1, st));
    }
  }
  void shape(int b, int h, int w) {
    if (b == B && h == H && w == W) return;
    const size_t p0 = (size_t)b * h * w, p1 = p0 / 4, p2 = p0 / 16;
    auto bfb = [](size_t px, int c) { return px * c * 2; };
    X0.ensure(bfb(p0, 8)); A1.ensure(bfb(p0, 16)); C1.ensure(bfb(p0, 48)); P1.ensure(bfb(p1, 16));
    A2.ensure(bfb(p1, 32)); C2.ensure(bfb(p1, 96)); P2.ensure(bfb(p2, 32)); A3.ensure(bfb(p2, 64));
    A3b.ensure(bfb(p2, 64)); A4.ensure(bfb(p1, 32)); A5.ensure(bfb(p0, 16)); Y.ensure(p0 * 4);
    S1.ensure(bfb(p0, 16)); S2.ensure(bfb(p1, 32));
    dY.ensure(bfb(p0, 16)); dA5.ensure(bfb(p0, 16)); dC1.ensure(bfb(p0, 48)); dA4.ensure(bfb(p1, 32));
    dC2.ensure(bfb(p1, 96)); dA3b.ensure(bfb(p2, 64)); dA3.ensure(bfb(p2, 64)); dP2.ensure(bfb(p2, 32));
    dA2.ensure(bfb(p1, 32)); dP1.ensure(bfb(p1, 16)); dA1.ensure(bfb(p0, 16));
    scale.ensure((size_t)b * 2 * 4);
    B = b; H = h; W = w;
  }
};

namespace {

using namespace gd::net;

// rows per weight-gradient chunk: about 128 chunks over the batch
int wgrad_rows(int B, int h) { return std::max(1, (B * h + 127) / 128); }

void conv_fwd(gd_net& N, int l, const bf* in, int in_s, int in_o, bf* out, int out_s, int out_o, int h, int w,
              hipStream_t st, float* out_f = nullptr, const bf* in2 = nullptr, int in2_s = 0, int cup = 0,
              const float* rin = nullptr, const float* rscale = nullptr, const float* oscale = nullptr) {
  const LayerSpec& L = kLayers[l];
  const float* bias = N.master.as<float>() + N.boff[l];
  if (N.timing) {
    if (N.ev_used == N.ev.size()) {
      hipEvent_t a, b;
      NT_TRY(hipEventCreate(&a));
      NT_TRY(hipEventCreate(&b));
      N.ev.push_back({a, b});
      N.ev_layer.push_back(0);
      N.ev_flops.push_back(0.0);
    }
    N.ev_layer[N.ev_used] = l;
    N.ev_flops[N.ev_used] = 2.0 * 9.0 * L.cin * L.cout * (double)N.B * h * w;  // real channels, not padding
    NT_TRY(hipEventRecord(N.ev[N.ev_used].first, st));
  }
  NT_TRY(conv(L.cinp, L.coutp, in, in_s, in_o, N.wpk[l].as<bf>(), bias, l != 8, out, out_f, out_s, out_o,
              L.cout, nullptr, 0, 0, N.B, h, w, st, in2, in2_s, 0, cup, rin, rscale, oscale));
  if (N.timing) NT_TRY(hipEventRecord(N.ev[N.ev_used++].second, st));
}

// weight and bias gradients of layer l into N.grad
void conv_wgrad(gd_net& N, int l, const bf* in, int in_s, int in_o, const bf* dout, int d_s, int d_o, int h, int w,
                hipStream_t st) {
  const LayerSpec& L = kLayers[l];
  const int kpad = kpad_of(L.cinp);
  const int R = wgrad_rows(N.B, h);
  const int chunks = N.B * ((h + R - 1) / R);
  const int n = L.coutp * kpad;
  N.part.ensure((size_t)chunks * n * 4);
  N.gpk.ensure((size_t)n * 4);
  NT_TRY(wgrad(L.cinp, L.coutp, in, in_s, in_o, dout, d_s, d_o, N.part.as<float>(), N.B, h, w, R, st));
  NT_TRY(sum_chunks(N.part.as<float>(), chunks, n, N.gpk.as<float>(), st));
  NT_TRY(unpack_wgrad(N.gpk.as<float>(), L.cout, L.cin, L.cinp, kpad, N.grad.as<float>() + N.woff[l], st));
  const int nb = 256;
  N.bpart.ensure((size_t)nb * 64 * 4);
  NT_TRY(bias_grad(dout, d_s, d_o, L.cout, (int64_t)N.B * h * w, N.bpart.as<float>(), nb, st));
  NT_TRY(sum_chunks(N.bpart.as<float>(), nb, 64, N.gpk.as<float>(), st));
  NT_TRY(hipMemcpyAsync(N.grad.as<float>() + N.boff[l], N.gpk.as<float>(), L.cout * 4, hipMemcpyDeviceToDevice, st));
}

// data gradient of layer l: din = conv(dout, W^T flipped) [* (mask > 0)]
void conv_dgrad(gd_net& N, int l, const bf* dout, int d_s, int d_o, bf* din, int i_s, int i_o, const bf* mask,
                int m_s, int m_o, int h, int w, hipStream_t st) {
  const LayerSpec& L = kLayers[l];
  const int rows = (L.cin + 15) / 16 * 16;
  NT_TRY(conv(L.coutp, rows, dout, d_s, d_o, N.wpkT[l].as<bf>(), nullptr, 0, din, nullptr, i_s, i_o, L.cin, mask, m_s,
              m_o, N.B, h, w, st));
}

// per-image RMS of r -> scale (s) and inverse (1/s) on the device
void image_scale(gd_net& N, const float* r, hipStream_t st);

// train: the activations back-propagation needs are kept and the output
// is the net's FP32 value; otherwise z = net * scale is written to z_out
void forward(gd_net& N, const float* r, hipStream_t st, bool train = true, float* z_out = nullptr) {
  const int H = N.H, W = N.W, h1 = H / 2, w1 = W / 2, h2 = H / 4, w2 = W / 4;
  const int64_t npix = (int64_t)H * W;
  image_scale(N, r, st);
  if (!train) {
    // forward only: the first convolution reads the residual itself, the
    // skip activations stay contiguous, the decoder convolutions read their
    // concatenated inputs in place, up-sampling on the fly, and the last one
    // writes z scaled back
    conv_fwd(N, 0, nullptr, 8, 0, N.A1.as<bf>(), 16, 0, H, W, st, nullptr, nullptr, 0, 0, r,
             N.scale.as<float>() + N.B);
    conv_fwd(N, 1, N.A1.as<bf>(), 16, 0, N.S1.as<bf>(), 16, 0, H, W, st);
    NT_TRY(pool(N.S1.as<bf>(), 16, 0, N.P1.as<bf>(), 16, 0, 16, N.B, H, W, st));
    conv_fwd(N, 2, N.P1.as<bf>(), 16, 0, N.A2.as<bf>(), 32, 0, h1, w1, st);
    conv_fwd(N, 3, N.A2.as<bf>(), 32, 0, N.S2.as<bf>(), 32, 0, h1, w1, st);
    NT_TRY(pool(N.S2.as<bf>(), 32, 0, N.P2.as<bf>(), 32, 0, 32, N.B, h1, w1, st));
    conv_fwd(N, 4, N.P2.as<bf>(), 32, 0, N.A3.as<bf>(), 64, 0, h2, w2, st);
    conv_fwd(N, 5, N.A3.as<bf>(), 64, 0, N.A3b.as<bf>(), 64, 0, h2, w2, st);
    conv_fwd(N, 6, N.A3b.as<bf>(), 64, 0, N.A4.as<bf>(), 32, 0, h1, w1, st, nullptr, N.S2.as<bf>(), 32, 64);
    conv_fwd(N, 7, N.A4.as<bf>(), 32, 0, N.A5.as<bf>(), 16, 0, H, W, st, nullptr, N.S1.as<bf>(), 16, 32);
    conv_fwd(N, 8, N.A5.as<bf>(), 16, 0, nullptr, 1, 0, H, W, st, z_out, nullptr, 0, 0, nullptr, nullptr,
             N.scale.as<float>());
    return;
  }
  NT_TRY(pack_input(r, N.scale.as<float>() + N.B, N.X0.as<bf>(), 8, npix, N.B, st));
  conv_fwd(N, 0, N.X0.as<bf>(), 8, 0, N.A1.as<bf>(), 16, 0, H, W, st);
  conv_fwd(N, 1, N.A1.as<bf>(), 16, 0, N.C1.as<bf>(), 48, 32, H, W, st);
  NT_TRY(pool(N.C1.as<bf>(), 48, 32, N.P1.as<bf>(), 16, 0, 16, N.B, H, W, st));
  conv_fwd(N, 2, N.P1.as<bf>(), 16, 0, N.A2.as<bf>(), 32, 0, h1, w1, st);
  conv_fwd(N, 3, N.A2.as<bf>(), 32, 0, N.C2.as<bf>(), 96, 64, h1, w1, st);
  NT_TRY(pool(N.C2.as<bf>(), 96, 64, N.P2.as<bf>(), 32, 0, 32, N.B, h1, w1, st));
  conv_fwd(N, 4, N.P2.as<bf>(), 32, 0, N.A3.as<bf>(), 64, 0, h2, w2, st);
  conv_fwd(N, 5, N.A3.as<bf>(), 64, 0, N.A3b.as<bf>(), 64, 0, h2, w2, st);
  NT_TRY(up(N.A3b.as<bf>(), 64, 0, N.C2.as<bf>(), 96, 0, 64, N.B, h1, w1, st));
  conv_fwd(N, 6, N.C2.as<bf>(), 96, 0, N.A4.as<bf>(), 32, 0, h1, w1, st);
  NT_TRY(up(N.A4.as<bf>(), 32, 0, N.C1.as<bf>(), 48, 0, 32, N.B, H, W, st));
  conv_fwd(N, 7, N.C1.as<bf>(), 48, 0, N.A5.as<bf>(), 16, 0, H, W, st);
  conv_fwd(N, 8, N.A5.as<bf>(), 16, 0, nullptr, 1, 0, H, W, st, N.Y.as<float>());
}

double backward(gd_net& N, const float* e, hipStream_t st) {
  const int H = N.H, W = N.W, h1 = H / 2, w1 = W / 2, h2 = H / 4, w2 = W / 4;
  const int64_t npix = (int64_t)H * W;
  int nblk = 0;
  N.lpart.ensure((size_t)((npix * N.B + 255) / 256) * 8);
  NT_TRY(loss(N.Y.as<float>(), 1, e, N.scale.as<float>() + N.B, N.dY.as<bf>(), 16, 16, npix, N.B,
              N.lpart.as<double>(), &nblk, st));
  // L6 and L5
  conv_wgrad(N, 8, N.A5.as<bf>(), 16, 0, N.dY.as<bf>(), 16, 0, H, W, st);
  conv_dgrad(N, 8, N.dY.as<bf>(), 16, 0, N.dA5.as<bf>(), 16, 0, N.A5.as<bf>(), 16, 0, H, W, st);
  conv_wgrad(N, 7, N.C1.as<bf>(), 48, 0, N.dA5.as<bf>(), 16, 0, H, W, st);
  conv_dgrad(N, 7, N.dA5.as<bf>(), 16, 0, N.dC1.as<bf>(), 48, 0, nullptr, 0, 0, H, W, st);
  // up(L4) part of concat 1 -> L4
  NT_TRY(up_bwd(N.dC1.as<bf>(), 48, 0, N.dA4.as<bf>(), 32, 0, N.A4.as<bf>(), 32, 0, 32, N.B, H, W, st));
  conv_wgrad(N, 6, N.C2.as<bf>(), 96, 0, N.dA4.as<bf>(), 32, 0, h1, w1, st);
  conv_dgrad(N, 6, N.dA4.as<bf>(), 32, 0, N.dC2.as<bf>(), 96, 0, nullptr, 0, 0, h1, w1, st);
  // up(L3b) part of concat 2 -> L3b, L3a
  NT_TRY(up_bwd(N.dC2.as<bf>(), 96, 0, N.dA3b.as<bf>(), 64, 0, N.A3b.as<bf>(), 64, 0, 64, N.B, h1, w1, st));
  conv_wgrad(N, 5, N.A3.as<bf>(), 64, 0, N.dA3b.as<bf>(), 64, 0, h2, w2, st);
  conv_dgrad(N, 5, N.dA3b.as<bf>(), 64, 0, N.dA3.as<bf>(), 64, 0, N.A3.as<bf>(), 64, 0, h2, w2, st);
  conv_wgrad(N, 4, N.P2.as<bf>(), 32, 0, N.dA3.as<bf>(), 64, 0, h2, w2, st);
  conv_dgrad(N, 4, N.dA3.as<bf>(), 64, 0, N.dP2.as<bf>(), 32, 0, nullptr, 0, 0, h2, w2, st);
  // pool 2 backward joins the skip gradient of L2b
  NT_TRY(pool_bwd_acc(N.dP2.as<bf>(), 32, 0, N.dC2.as<bf>(), 96, 64, 32, N.B, h1, w1, st));
  NT_TRY(relu_mask(N.dC2.as<bf>(), 96, 64, N.C2.as<bf>(), 96, 64, 32, (int64_t)N.B * h1 * w1, st));
  conv_wgrad(N, 3, N.A2.as<bf>(), 32, 0, N.dC2.as<bf>(), 96, 64, h1, w1, st);
  conv_dgrad(N, 3, N.dC2.as<bf>(), 96, 64, N.dA2.as<bf>(), 32, 0, N.A2.as<bf>(), 32, 0, h1, w1, st);
  conv_wgrad(N, 2, N.P1.as<bf>(), 16, 0, N.dA2.as<bf>(), 32, 0, h1, w1, st);
  conv_dgrad(N, 2, N.dA2.as<bf>(), 32, 0, N.dP1.as<bf>(), 16, 0, nullptr, 0, 0, h1, w1, st);
  // pool 1 backward joins the skip gradient of L1b
  NT_TRY(pool_bwd_acc(N.dP1.as<bf>(), 16, 0, N.dC1.as<bf>(), 48, 32, 16, N.B, H, W, st));
  NT_TRY(relu_mask(N.dC1.as<bf>(), 48, 32, N.C1.as<bf>(), 48, 32, 16, (int64_t)N.B * H * W, st));
  conv_wgrad(N, 1, N.A1.as<bf>(), 16, 0, N.dC1.as<bf>(), 48, 32, H, W, st);
  conv_dgrad(N, 1, N.dC1.as<bf>(), 48, 32, N.dA1.as<bf>(), 16, 0, N.A1.as<bf>(), 16, 0, H, W, st);
  conv_wgrad(N, 0, N.X0.as<bf>(), 8, 0, N.dA1.as<bf>(), 16, 0, H, W, st);
  // loss (block partials summed in order on the host)
  N.hl.resize(nblk);
  NT_TRY(hipMemcpyAsync(N.hl.data(), N.lpart.p, nblk * 8, hipMemcpyDeviceToHost, st));
  NT_TRY(hipStreamSynchronize(st));
  double L = 0.0;
  for (double v : N.hl) L += v;
  return L;
}

gd_status guard(const std::function<gd_status()>& f) {
  try {
    return f();
  } catch (const HipErr& e) {
    if (e.e == hipErrorOutOfMemory) return nfail(GD_ERR_NOMEM, std::string("out of device memory in ") + e.what);
    return nfail(GD_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return nfail(GD_ERR_NOMEM, "host allocation failed");
  }
}

gd_status check_shape(int64_t nx, int64_t ny, int64_t batch, bool training) {
  if (nx <= 0 || ny <= 0 || batch <= 0 || nx % 256 || ny % 4 || nx > (1 << 14) || ny > (1 << 14) || batch > (1 << 16))
    return nfail(GD_ERR_INVALID, "net: images must be nx % 256 == 0, ny % 4 == 0 (pooling twice, 64-pixel rows), "
                                 "at most 16384 x 16384");
  if (nx * ny > ((int64_t)1 << 26) || (training && nx * ny * batch > ((int64_t)1 << 28)))
    return nfail(GD_ERR_INVALID, "net: at most 2^26 pixels per image and 2^28 per training batch");
  return GD_OK;
}

}  // namespace

// per-image RMS: small reduction kernels live in kernels of net.hip via loss()'s
// machinery would mix concerns; a dedicated kernel is defined here
namespace {
__global__ void k_img_sumsq(const float* __restrict__ r, int64_t npix_img, int nblk_img, double* __restrict__ part) {
  __shared__ double red[256];
  const int b = blockIdx.x / nblk_img, k = blockIdx.x % nblk_img;
  double s = 0.0;
  for (int64_t p = (int64_t)k * 256 + threadIdx.x; p < npix_img; p += (int64_t)nblk_img * 256) {
    const double v = r[(int64_t)b * npix_img + p];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_img_scale(const double* __restrict__ part, int nblk_img, int64_t npix_img, int B,
                            float* __restrict__ scale) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int k = 0; k < nblk_img; ++k) s += part[b * nblk_img + k];
  double rms = std::sqrt(s / (double)npix_img);
  if (!(rms > 0.0)) rms = 1.0;
  scale[b] = (float)rms;
  scale[B + b] = (float)(1.0 / rms);
}
}  // namespace

namespace {
void image_scale(gd_net& N, const float* r, hipStream_t st) {
  const int64_t npix = (int64_t)N.H * N.W;
  const int nblk = 64;
  N.lpart.ensure(std::max<size_t>(N.lpart.n, (size_t)N.B * nblk * 8));
  hipLaunchKernelGGL(k_img_sumsq, dim3(N.B * nblk), dim3(256), 0, st, r, npix, nblk, N.lpart.as<double>());
  NT_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_img_scale, dim3((N.B + 255) / 256), dim3(256), 0, st, N.lpart.as<double>(), nblk, npix, N.B,
                     N.scale.as<float>());
  NT_TRY(hipGetLastError());
}
}  // namespace

extern "C" {

const char* gd_net_last_error(void) { return t_err.c_str(); }

gd_status gd_net_create(gd_net** out, const float* weights, int64_t count, uint64_t seed) {
  if (!out) return nfail(GD_ERR_INVALID, "gd_net_create: null handle pointer");
  *out = nullptr;
  return guard([&]() -> gd_status {
    auto N = std::make_unique<gd_net>();
    N->layout();
    if (weights && count != N->nparam)
      return nfail(GD_ERR_INVALID, "gd_net_create: weight count " + std::to_string(count) + " != " +
                                       std::to_string(N->nparam));
    N->alloc_params();
    if (weights) {  // the caller's FP32 master weights (gd_net_get_params layout)
      NT_TRY(hipMemcpy(N->master.p, weights, N->nparam * 4, hipMemcpyHostToDevice));
      N->pack(nullptr);
      NT_TRY(hipDeviceSynchronize());
      *out = N.release();
      return GD_OK;
    }
    // He-normal weights (Box-Muller on splitmix64), zero biases
    std::vector<float> h(N->nparam, 0.f);
    uint64_t c = seed * 0x2545F4914F6CDD1Dull + 1;
    for (int l = 0; l < 9; ++l) {
      const LayerSpec& L = kLayers[l];
      const double sd = std::sqrt(2.0 / (9.0 * L.cin)) * (l == 8 ? 0.1 : 1.0);
      const size_t n = (size_t)L.cout * L.cin * 9;
      for (size_t i = 0; i < n; ++i) {
        const double u1 = ((mix64(c++) >> 11) + 0.5) / 9007199254740992.0;
        const double u2 = ((mix64(c++) >> 11) + 0.5) / 9007199254740992.0;
        h[N->woff[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
      }
    }
    NT_TRY(hipMemcpy(N->master.p, h.data(), N->nparam * 4, hipMemcpyHostToDevice));
    N->pack(nullptr);
    NT_TRY(hipDeviceSynchronize());
    *out = N.release();
    return GD_OK;
  });
}

gd_status gd_net_destroy(gd_net* n) {
  delete n;
  return GD_OK;
}

int64_t gd_net_num_params(const gd_net* n) { return n ? n->nparam : 0; }

gd_status gd_net_get_params(gd_net* n, float* host, int64_t count) {
  if (!n || !host || count != n->nparam) return nfail(GD_ERR_INVALID, "gd_net_get_params: bad arguments");
  return guard([&]() -> gd_status {
    NT_TRY(hipMemcpy(host, n->master.p, count * 4, hipMemcpyDeviceToHost));
    return GD_OK;
  });
}

gd_status gd_net_set_params(gd_net* n, const float* host, int64_t count) {
  if (!n || !host || count != n->nparam) return nfail(GD_ERR_INVALID, "gd_net_set_params: bad arguments");
  return guard([&]() -> gd_status {
    NT_TRY(hipMemcpy(n->master.p, host, count * 4, hipMemcpyHostToDevice));
    n->pack(nullptr);
    NT_TRY(hipDeviceSynchronize());
    return GD_OK;
  });
}

gd_status gd_net_forward(gd_net* n, const float* r, float* z, int64_t nx, int64_t ny, int64_t batch, void* stream) {
  if (!n || !r || !z) return nfail(GD_ERR_INVALID, "gd_net_forward: null pointer");
  if (r == z) return nfail(GD_ERR_INVALID, "gd_net_forward: output aliases input");
  gd_status s = check_shape(nx, ny, batch, false);
  if (s != GD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  return guard([&]() -> gd_status {
    // batches of images of at most 2^25 pixels bound the activation memory
    const int64_t npix = nx * ny, bc = std::max<int64_t>(1, ((int64_t)1 << 25) / npix);
    for (int64_t b0 = 0; b0 < batch; b0 += bc) {
      const int64_t nbat = std::min(bc, batch - b0);
      n->shape((int)nbat, (int)ny, (int)nx);
      forward(*n, r + b0 * npix, st, false, z + b0 * npix);
    }
    NT_TRY(hipStreamSynchronize(st));
    n->harvest();
    return GD_OK;
  });
}

gd_status gd_net_gradients(gd_net* n, const float* r, const float* e, int64_t nx, int64_t ny, int64_t batch,
                           float* grad_host, double* loss_out, void* stream) {
  if (!n || !r || !e) return nfail(GD_ERR_INVALID, "gd_net_gradients: null pointer");
  gd_status s = check_shape(nx, ny, batch, true);
  if (s != GD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  return guard([&]() -> gd_status {
    n->shape((int)batch, (int)ny, (int)nx);
    forward(*n, r, st);
    const double L = backward(*n, e, st);
    n->harvest();
    if (loss_out) *loss_out = L;
    if (grad_host) NT_TRY(hipMemcpy(grad_host, n->grad.p, n->nparam * 4, hipMemcpyDeviceToHost));
    return GD_OK;
  });
}

gd_status gd_net_train_step(gd_net* n, const float* r, const float* e, int64_t nx, int64_t ny, int64_t batch, float lr,
                            double* loss_out, void* stream) {
  if (!n || !r || !e) return nfail(GD_ERR_INVALID, "gd_net_train_step: null pointer");
  if (!(lr > 0.f)) return nfail(GD_ERR_INVALID, "gd_net_train_step: lr must be > 0");
  gd_status s = check_shape(nx, ny, batch, true);
  if (s != GD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  return guard([&]() -> gd_status {
    n->shape((int)batch, (int)ny, (int)nx);
    forward(*n, r, st);
    const double L = backward(*n, e, st);
    n->harvest();
    if (loss_out) *loss_out = L;
    if (!std::isfinite(L)) return nfail(GD_ERR_NUMERIC, "gd_net_train_step: non-finite loss");
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    NT_TRY(adam(n->master.as<float>(), n->grad.as<float>(), n->m.as<float>(), n->v.as<float>(), (int)n->nparam, lr,
                b1, b2, 1e-8f, c1, c2, st));
    n->pack(st);
    NT_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_net_set_timing(gd_net* n, int on) {
  if (!n) return nfail(GD_ERR_INVALID, "gd_net_set_timing: null handle");
  n->timing = on != 0;
  n->ev_used = 0;
  for (int l = 0; l < 9; ++l) {
    n->t_ms[l] = 0.0;
    n->t_flops[l] = 0.0;
    n->t_cnt[l] = 0;
  }
  return GD_OK;
}

gd_status gd_net_kernel_time(const gd_net* n, int layer, double* ms, int64_t* launches, double* flops) {
  if (!n || layer < 0 || layer >= 9) return nfail(GD_ERR_INVALID, "gd_net_kernel_time: bad handle or layer");
  if (ms) *ms = n->t_ms[layer];
  if (launches) *launches = n->t_cnt[layer];
  if (flops) *flops = n->t_flops[layer];
  return GD_OK;
}

}  // extern "C"
