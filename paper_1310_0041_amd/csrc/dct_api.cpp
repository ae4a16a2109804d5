// C ABI of the spectral (DCT) solver: exact solves of the constant-
// coefficient systems of Sec. 4 by DCT-II diagonalisation (Sec. 3.2), a
// competitor and verifier of the multigrid path on power-of-two grids.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "gd.h"
#include "gd_dct.h"

namespace gd {
gd_status set_error(gd_status s, const std::string& msg);  // gd_api.cpp
}

namespace {

std::mutex g_mu;
std::map<int, std::pair<double*, size_t>> g_ws;  // device -> FP64 workspace
struct Tab {
  double2 *W = nullptr, *Q = nullptr;
  double* lam = nullptr;
};
std::map<std::pair<int, int>, Tab> g_tabs;  // (device, length) -> twiddle and eigenvalue tables

bool pow2_le(int64_t n, int64_t cap) { return n >= 1 && n <= cap && (n & (n - 1)) == 0; }

gd_status check_grid(const char* who, int64_t nx, int64_t ny, int64_t nz) {
  if (nx <= 0 || ny <= 0 || nz <= 0) return gd::set_error(GD_ERR_INVALID, std::string(who) + ": bad size");
  if (!pow2_le(nx, 4096) || !pow2_le(ny, 4096) || !pow2_le(nz, 4096))
    return gd::set_error(GD_ERR_UNSUPPORTED, std::string(who) + ": every axis must be a power of two <= 4096");
  return GD_OK;
}

bool valid(gd_dtype t) { return t == GD_F64 || t == GD_F32 || t == GD_F16 || t == GD_BF16; }

// FP64 work array of n values on the current device (kept between calls)
hipError_t workspace(int dev, int64_t n, double** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto& w = g_ws[dev];
  const size_t bytes = (size_t)n * sizeof(double);
  if (w.second < bytes) {
    if (w.first) (void)hipFree(w.first);
    w.first = nullptr;
    w.second = 0;
    hipError_t e = hipMalloc(&w.first, bytes);
    if (e != hipSuccess) return e;
    w.second = bytes;
  }
  *out = w.first;
  return hipSuccess;
}

hipError_t tables(int dev, int n, Tab* out, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tabs.find({dev, n});
  if (it != g_tabs.end()) { *out = it->second; return hipSuccess; }
  Tab t;
  void* p = nullptr;
  const size_t bytes = (size_t)n * (sizeof(double2) * 2 + sizeof(double));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return e;
  t.W = (double2*)p;
  t.Q = t.W + n;
  t.lam = (double*)(t.Q + n);
  e = gd::dct_tables(n, t.W, t.Q, t.lam, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { (void)hipFree(p); return e; }
  g_tabs[{dev, n}] = t;
  *out = t;
  return hipSuccess;
}

// forward DCT along x, y, z (the z pass also scales), inverse along z, y, x;
// the first pass reads the caller's input and the last writes the output.
// Long y-lines (ny >= 512, nx > 1) are transposed into contiguous lines
// first (a y pass over lines ny values apart reads short runs), and back
// before the last x pass.
gd_status spectral(const char* who, const void* in, gd_dtype it, void* out, gd_dtype ot, int64_t nx, int64_t ny,
                   int64_t nz, int mode, double alpha, double wx, double wy, double wz, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = nx * ny * nz;
  const bool tr = ny >= 512 && nx > 1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  double* w = nullptr;
  Tab tb[3];
  const int len[3] = {(int)nx, (int)ny, (int)nz};
  auto ok = [&](hipError_t r) { return r == hipSuccess; };
  if (ok(e)) e = workspace(dev, tr ? 2 * n : n, &w);
  double* w2 = w + n;
  for (int a = 0; a < 3 && ok(e); ++a) e = tables(dev, len[a], &tb[a], st);
  // a pass over a volume of dims d[3] (x, y, z) along `axis`; tabs / weights
  // of the volume's own x and y axes
  auto pass = [&](const int d[3], const Tab* tx, const Tab* ty, double ax_w, double ay_w, int a, bool inv,
                  const void* src, gd_dtype ts, void* dst, gd_dtype td, int scale) {
    const Tab& ta = a == 0 ? *tx : (a == 1 ? *ty : tb[2]);
    gd::DctPass p{d[0], d[1], d[2], a, inv, src, ts, dst, td, ta.W, ta.Q, scale, tx->lam, ty->lam, tb[2].lam,
                  alpha, ax_w, ay_w, wz};
    return gd::dct_pass(p, st);
  };
  if (tr) {
    const int dn[3] = {(int)nx, (int)ny, (int)nz}, dt[3] = {(int)ny, (int)nx, (int)nz};
    const bool zt = nz > 1;
    if (ok(e)) e = pass(dn, &tb[0], &tb[1], wx, wy, 0, false, in, it, w, GD_F64, -1);
    if (ok(e)) e = gd::dct_transpose_xy(w, w2, (int)nx, (int)ny, (int)nz, st);
    if (ok(e)) e = pass(dt, &tb[1], &tb[0], wy, wx, 0, false, w2, GD_F64, w2, GD_F64, -1);
    if (ok(e) && zt) e = pass(dt, &tb[1], &tb[0], wy, wx, 2, false, w2, GD_F64, w2, GD_F64, mode);
    if (ok(e) && !zt)
      e = gd::dct_scale(w2, (int)ny, (int)nx, (int)nz, mode, tb[1].lam, tb[0].lam, tb[2].lam, alpha, wy, wx, wz, st);
    if (ok(e) && zt) e = pass(dt, &tb[1], &tb[0], wy, wx, 2, true, w2, GD_F64, w2, GD_F64, -1);
    if (ok(e)) e = pass(dt, &tb[1], &tb[0], wy, wx, 0, true, w2, GD_F64, w2, GD_F64, -1);
    if (ok(e)) e = gd::dct_transpose_xy(w2, w, (int)ny, (int)nx, (int)nz, st);
    if (ok(e)) e = pass(dn, &tb[0], &tb[1], wx, wy, 0, true, w, GD_F64, out, ot, -1);
  } else {
    int axes[3], na = 0;
    for (int a = 0; a < 3; ++a)
      if (len[a] > 1) axes[na++] = a;
    const int dn[3] = {(int)nx, (int)ny, (int)nz};
    const bool fused = na > 0 && axes[na - 1] == 2;  // the z pass exists and is the last forward pass
    if (ok(e) && na == 0) e = gd::dct_convert(in, it, w, n, true, nullptr, st);
    for (int q = 0; q < na && ok(e); ++q)
      e = pass(dn, &tb[0], &tb[1], wx, wy, axes[q], false, q == 0 ? in : w, q == 0 ? it : GD_F64, w, GD_F64,
               (fused && q == na - 1) ? mode : -1);
    if (ok(e) && !fused)
      e = gd::dct_scale(w, (int)nx, (int)ny, (int)nz, mode, tb[0].lam, tb[1].lam, tb[2].lam, alpha, wx, wy, wz, st);
    for (int q = na - 1; q >= 0 && ok(e); --q)
      e = pass(dn, &tb[0], &tb[1], wx, wy, axes[q], true, w, GD_F64, q == 0 ? out : w, q == 0 ? ot : GD_F64, -1);
    if (ok(e) && na == 0) e = gd::dct_convert(w, ot, nullptr, n, false, out, st);
  }
  if (ok(e)) e = hipStreamSynchronize(st);
  if (e == hipErrorOutOfMemory) return gd::set_error(GD_ERR_NOMEM, std::string(who) + ": out of device memory");
  if (!ok(e)) return gd::set_error(GD_ERR_HIP, std::string(who) + ": " + hipGetErrorString(e));
  return GD_OK;
}

}  // namespace

namespace gd {
void dct_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ws)
    if (kv.second.first) (void)hipFree(kv.second.first);
  g_ws.clear();
  for (auto& kv : g_tabs) (void)hipFree(kv.second.W);
  g_tabs.clear();
}
}  // namespace gd

extern "C" {

gd_status gd_dct_solve(const void* b, gd_dtype bt, void* x, gd_dtype xt, int64_t nx, int64_t ny, int64_t nz,
                       double alpha, double beta_x, double beta_y, double beta_z, void* stream) {
  if (!b || !x) return gd::set_error(GD_ERR_INVALID, "gd_dct_solve: null pointer");
  if (!valid(bt) || !valid(xt)) return gd::set_error(GD_ERR_INVALID, "gd_dct_solve: bad dtype");
  if (!(alpha >= 0.0) || !(beta_x >= 0.0) || !(beta_y >= 0.0) || !(beta_z >= 0.0) || !std::isfinite(alpha) ||
      !std::isfinite(beta_x) || !std::isfinite(beta_y) || !std::isfinite(beta_z))
    return gd::set_error(GD_ERR_INVALID, "gd_dct_solve: need alpha, beta >= 0");
  gd_status s = check_grid("gd_dct_solve", nx, ny, nz);
  if (s != GD_OK) return s;
  return spectral("gd_dct_solve", b, bt, x, xt, nx, ny, nz, 0, alpha, beta_x, beta_y, beta_z, stream);
}

gd_status gd_dct_smooth_z(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny,
                          int64_t nz, double beta_x, double beta_y, double beta_z, void* stream) {
  if (!I0 || !I1) return gd::set_error(GD_ERR_INVALID, "gd_dct_smooth_z: null pointer");
  if (!valid(in_t) || !valid(out_t)) return gd::set_error(GD_ERR_INVALID, "gd_dct_smooth_z: bad dtype");
  if (!(beta_x >= 0.0) || !(beta_y >= 0.0) || !(beta_z > 0.0) || !std::isfinite(beta_x) ||
      !std::isfinite(beta_y) || !std::isfinite(beta_z))
    return gd::set_error(GD_ERR_INVALID, "gd_dct_smooth_z: need beta_x, beta_y >= 0 and beta_z > 0");
  gd_status s = check_grid("gd_dct_smooth_z", nx, ny, nz);
  if (s != GD_OK) return s;
  return spectral("gd_dct_smooth_z", I0, in_t, I1, out_t, nx, ny, nz, 1, 0.0, beta_x, beta_y, beta_z, stream);
}

}  // extern "C"
