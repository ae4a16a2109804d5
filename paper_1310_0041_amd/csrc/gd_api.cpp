// Host orchestration and C ABI of the gradient-domain multigrid solver
// (Kazhdan et al., "Gradient-Domain Processing for Large EM Image Stacks").
//
// The hierarchy: a level holds one grid (3-D stack, anisotropic diffusion)
// or many (independent 2-D slices, screened Poisson).  Each grid is coarsened
// on its own: an axis is halved when it still has more than one cell and its
// coupling weight is at least half of the strongest remaining one, so a
// strongly coupled axis (beta_z = 4 > beta_x = beta_y) is coarsened first and
// the coarse operators become isotropic.  A coarse operator re-discretises
// the fine one on the doubled cells: with cell-volume ratio V = prod f_a,
// alpha_c = V alpha and w_a,c = V / f_a^2 * w_a (face area over length).
// Grids end at one cell, whose relaxation is an exact solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gd.h"
#include "gd_launch.h"

namespace gd {

static thread_local std::string t_err;

static gd_status fail(gd_status s, const std::string& msg) {
  t_err = msg;
  return s;
}
// the same, for the library's other translation units
gd_status set_error(gd_status s, const std::string& msg) { return fail(s, msg); }
void dct_release();  // dct_api.cpp

struct HipFail {
  hipError_t e;
  const char* what;
};

#define HIP_TRY(call)                                         \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) throw HipFail{e_, #call};           \
  } while (0)

static size_t dsize(gd_dtype t) {
  switch (t) {
    case GD_F64: return 8;
    case GD_F32: return 4;
    case GD_F16: return 2;
    case GD_BF16: return 2;
  }
  return 0;
}

static bool valid_dtype(int t) { return t >= GD_F64 && t <= GD_BF16; }

// ------------------------------------------------------------- timing

// finest-level relaxation launches by kind: 0 stack grid, 1 stack with the
// correction added on load, 2 slices, 3 slices with the correction, 4 stack
// starting from zero, 5 slices starting from zero
constexpr int kTimerKinds = 6;
struct KernelTimer {
  std::mutex mu;
  double total_ms[kTimerKinds] = {};
  int64_t launches[kTimerKinds] = {};
  double bytes[kTimerKinds] = {};  // summed over the launches (grids the kernels worked on)
};
static KernelTimer g_timer;

// --------------------------------------------------------------- hierarchy

struct GridSpec {  // finest-level grid in the kernels' view
  int64_t nx, ny, nz;
  double alpha, wx, wy, wz;
  int64_t ioff, ipy, ipz;
  int zin = 0;  // a 2-D slice seen as nz rows of one line
};

static int32_t pitch_of(int64_t nx) { return (int32_t)((nx + 3) & ~(int64_t)3); }

// Block order of relaxation launches (0 plain, 1 a contiguous run of tiles
// per XCD): GD_SWEEP_ORDER=0/1 fixes it, otherwise -1 here and the slice
// autotuner times both (3-D grids keep the plain order unless it is set).
static int sweep_order_env() {
  static const int v = [] {
    const char* e = std::getenv("GD_SWEEP_ORDER");
    const int o = e ? std::atoi(e) : -1;
    return o == 0 || o == 1 ? o : -1;
  }();
  return v;
}

// The quad relaxation of a one-grid 3-D level runs as two launches, its
// interior tiles (uniform weights) and its edge tiles (GD_SWEEP_SPLIT=0: one
// launch over all tiles).  Counts as in the kernels' decode.
static bool split_on() {
  static const bool v = [] {
    const char* e = std::getenv("GD_SWEEP_SPLIT");
    return !(e && std::atoi(e) == 0);
  }();
  return v;
}
static void set_split(Geom& g, const GridDesc& G) {
  g.n_int = g.n_edge = 0;
  if (!split_on()) return;
  const int TX = SWEEP_TILE_TX[g.tile], TY = SWEEP_TILE_TY[g.tile];
  const int64_t ntx = (G.nx + TX - 1) / TX, nty = (G.ny + TY - 1) / TY;
  const int64_t nix = std::max<int64_t>(0, (G.nx - 4) / TX - 1), niy = std::max<int64_t>(0, (G.ny - 2) / TY - 1);
  const int64_t chunks = (G.nz + g.zlen - 1) / g.zlen;
  if (nix * niy == 0) return;
  g.n_int = nix * niy * chunks;
  // the edge tiles are few: shorter z-chunks give their launch enough blocks
  // to fill the chip instead of a tail of long columns (values do not depend
  // on the chunking)
  const int64_t et = ntx * nty - nix * niy;
  const int64_t ce = std::min<int64_t>(G.nz, std::max<int64_t>(chunks, (4096 + et - 1) / et));
  g.zlen_edge = (int)((G.nz + ce - 1) / ce);
  g.n_edge = et * ((G.nz + g.zlen_edge - 1) / g.zlen_edge);
}

struct Tab {  // launch geometry of one kernel family on one level
  int64_t* d_b0 = nullptr;
  std::vector<int64_t> h_b0;
  int zlen = 1;
  int tile = 0;   // relaxation tile variant (3-D grids)
  int order = 0;  // relaxation block order (see xcd_block)
  Geom geom(const GridDesc* d_grids, int ngrids, bool row) const {
    Geom g;
    g.grids = d_grids;
    g.block0 = d_b0;
    g.ngrids = ngrids;
    g.nblocks = h_b0.back();
    g.zlen = zlen;
    g.etx = row ? EWR_TX : EW_TX;
    g.row = row;
    g.tile = tile;
    g.order = order;
    g.quad = true;  // level arrays: pitch and offsets multiples of 4
    return g;
  }
};

struct Level {
  std::vector<GridDesc> h;
  GridDesc* d = nullptr;
  int64_t total = 0;
  bool row = false;  // every grid has ny == 1
  bool keep_x = false;  // every grid keeps x on the way to the next level (f_x == 1)
  Tab sw, ew, rc, rz, pp;  // relaxation, per-voxel, child-cell, z-marching restriction, prolongation tiles
  Tab cs;                  // quad-form finest-level stencil passes (3-D grids)
  void* x = nullptr;
  void* xt = nullptr;
  void* b = nullptr;
};

struct Hier {
  int device = 0;
  gd_dtype s = GD_F32;
  int ngrids = 0;
  std::vector<Level> lv;
  std::vector<void*> allocs;
  size_t bytes = 0;  // device bytes held through alloc()
  double* partials = nullptr;
  double* dred = nullptr;    // ngrids * 2
  double* dscal = nullptr;   // ngrids * 4: scale, inv_scale, shift, spare
  double* hpin = nullptr;    // pinned host, ngrids * 4
  double* x64 = nullptr;     // FP64 iterate of the refinement path
  double* x64b = nullptr;    // its next value (the fused update writes here)
  std::vector<int64_t> cells;  // finest cells per grid
  std::vector<double> lcells;  // cells of every level (the grids the kernels work on)
  std::vector<double> lcells_all;  // the same with every grid
  double act = 1.0;  // share of the finest level's cells in grids the kernels work on
  // Algorithmic HBM bytes of the kernels launched through this hierarchy
  // (host-side count: the bytes each kernel must read and write per cell,
  // times the cells it covers; replayed graphs add what their capture counted)
  double acct = 0.0;
  void count(int l, double per_cell) { acct += per_cell * lcells[l]; }
  // Hybrid discretisation: per-level table blocks (levels >= 1) on the device
  // Hybrid (hyb) and Linear (lin) discretisations: per-level table blocks on
  // the device (Hybrid: levels >= 1; Linear: every level)
  std::vector<HybTables> hyb, lin;
  double* hyb_part = nullptr;   // per-block r^2 of a finest-level residual
  int64_t* hyb_b0 = nullptr;    // {0, block count} of the 7-point residual
  int64_t* tab_b0 = nullptr;    // {0, block count} of the table residual

  // Captured V-cycle segments (see CycleGraphs): two executables that map
  // the level buffers' ping-pong state A -> B and B -> A.
  struct Graph {
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<void*, void*>> from, to;  // (x, xt) of every level before / after
    double bytes = 0.0;  // algorithmic bytes of one replay
    double act = 1.0;    // Hier::act when it was captured (replays scale by the share now)
  };
  hipStream_t cap = nullptr;  // private capture stream (default priority)
  std::map<std::string, std::vector<Graph>> graphs;

  ~Hier() {
    for (auto& kv : graphs)
      for (auto& g : kv.second)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (cap) (void)hipStreamDestroy(cap);
    for (void* p : allocs) (void)hipFree(p);
    if (hpin && host_pin.empty()) (void)hipHostFree(hpin);
  }
  std::vector<std::pair<void*, void*>> xstate() const {
    std::vector<std::pair<void*, void*>> v;
    for (const auto& L : lv) v.push_back({L.x, L.xt});
    return v;
  }
  void set_xstate(const std::vector<std::pair<void*, void*>>& v) {
    for (size_t i = 0; i < lv.size(); ++i) { lv[i].x = v[i].first; lv[i].xt = v[i].second; }
  }
  // Arena mode (the no-allocation entry point): device arrays are carved out
  // of a caller-provided region instead of hipMalloc, and the host side of
  // the norm read-back is ordinary memory.  measure: only count the bytes.
  char* arena = nullptr;
  size_t arena_cap = 0;
  bool measure = false;
  std::vector<double> host_pin;
  void* alloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    if (arena || measure) {
      const size_t at = (this->bytes + 255) & ~(size_t)255;
      if (!measure && at + bytes > arena_cap) throw std::logic_error("scratch arena overflow");
      this->bytes = at + bytes;
      return measure ? nullptr : (void*)(arena + at);
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
    allocs.push_back(p);
    this->bytes += bytes;
    return p;
  }
  Geom g_sw(int l) const {
    Geom g = lv[l].sw.geom(lv[l].d, ngrids, lv[l].row);
    if (ngrids == 1 && !lv[l].row) set_split(g, lv[l].h[0]);
    return g;
  }
  Geom g_ew(int l) const { return lv[l].ew.geom(lv[l].d, ngrids, lv[l].row); }
  Geom g_rc(int l) const { return lv[l].rc.geom(lv[l].d, ngrids, lv[l].row); }
  Geom g_rz(int l) const { return lv[l].rz.geom(lv[l].d, ngrids, lv[l].row); }
  Geom g_pp(int l) const { return lv[l].pp.geom(lv[l].d, ngrids, lv[l].row); }
  Geom g_cs(int l) const { return lv[l].cs.geom(lv[l].d, ngrids, lv[l].row); }
  bool quad_opt = true;  // the caller's sweep_quad option of the running solve
  // A stack of equal, independent slices solved as one 3-D grid with w_z = 0:
  // the norms of the stencil passes are taken per plane (one plane per block)
  struct PlaneNorms {
    Tab tab[2];              // one-plane tiles of the pair (0) and quad (1) stencil forms
    int64_t* seg[2] = {};    // device: nz + 1 block offsets of the planes
    double* part = nullptr;  // device: 2 sums per block
    int64_t part_blocks = 0;
    double* red = nullptr;   // device: 2 sums per plane
    std::vector<double> host;  // 2 sums per plane
    int64_t* tseg = nullptr;   // device: nz + 1 block offsets of the table residual's planes
  };
  std::unique_ptr<PlaneNorms> planes;
  bool stack_z = false;  // z indexes independent slices: the table operators have M_z = Id, K_z = 0
  bool flags_set = false;  // some grid descriptor carries a skip / alt flag
  // level l (>= 1) holds a stale x that counts as zero: the restriction into
  // it did not clear x, and its next relaxation starts from zero (kept here,
  // not in a Cycler, because captured cycle pieces end with that restriction)
  std::vector<char> czero;
};

static void coarsen_factors(const GridDesc& g, int f[3]) {
  const int64_t n[3] = {g.nx, g.ny, g.nz};
  const double w[3] = {g.wx, g.wy, g.wz};
  double wmax = 0.0;
  for (int a = 0; a < 3; ++a)
    if (n[a] > 1 && w[a] > 0.0) wmax = std::max(wmax, w[a]);
  for (int a = 0; a < 3; ++a) f[a] = (n[a] > 1 && w[a] > 0.0 && w[a] >= 0.5 * wmax) ? 2 : 1;
}

static void build_tab(Tab& t, const std::vector<GridDesc>& grids, int TX, int TY, bool child, int64_t target,
                      bool even = false) {
  int64_t nzmax = 1, tiles_sum = 0;
  for (const auto& g : grids) {
    const int64_t nx = child ? g.cnx : g.nx, ny = child ? g.cny : g.ny, nz = child ? g.cnz : g.nz;
    nzmax = std::max(nzmax, nz);
    tiles_sum += ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY);
  }
  int64_t chunks = std::max<int64_t>(1, (target + tiles_sum - 1) / std::max<int64_t>(tiles_sum, 1));
  chunks = std::min(chunks, nzmax);
  t.zlen = (int)((nzmax + chunks - 1) / chunks);
  if (even && (t.zlen & 1)) t.zlen += 1;
  t.h_b0.assign(1, 0);
  for (const auto& g : grids) {
    const int64_t nx = child ? g.cnx : g.nx, ny = child ? g.cny : g.ny, nz = child ? g.cnz : g.nz;
    const int64_t nb = ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + t.zlen - 1) / t.zlen);
    t.h_b0.push_back(t.h_b0.back() + nb);
  }
}

// Relaxation tile variant of 3-D grids when the autotuner does not choose
// (GD_SWEEP_TILE, 0..5, the wide ones 4 and 5 where the quad form applies;
// 64 x 16 by default).
static int sweep_tile() {
  static int v = [] {
    const char* e = std::getenv("GD_SWEEP_TILE");
    const int t = e ? std::atoi(e) : 2;
    return (t >= 0 && t < kSweepTiles) ? t : 2;
  }();
  return v;
}

// Tile of the quad-form stencil passes (GD_STENCIL_TILE: 0 128 x 8, the
// default; 1 64 x 16).
static int stencil4_tile() {
  static const int v = [] {
    const char* e = std::getenv("GD_STENCIL_TILE");
    return (e && std::atoi(e) == 1) ? 1 : 0;
  }();
  return v;
}

// Blocks a finest-level relaxation launch aims for (z-chunks are cut until
// reached): GD_SWEEP_BLOCKS for 3-D grids (default 4096), GD_SWEEP_BLOCKS_ROW
// for one-line grids (2-D slices, default 8192).
static int64_t env_blocks(const char* name, int64_t dflt) {
  const char* e = std::getenv(name);
  return e ? std::max<int64_t>(1, std::atoll(e)) : dflt;
}
static int64_t sweep_target(bool row = false) {
  static int64_t v3 = env_blocks("GD_SWEEP_BLOCKS", 4096), vr = env_blocks("GD_SWEEP_BLOCKS_ROW", 8192);
  return row ? vr : v3;
}

// Levels below first_arrays get launch tables but no x / xt / b (their
// data lives elsewhere); max_levels > 0 stops the hierarchy after that many.
// arena / arena_cap: carve the device arrays out of that region (no
// allocation); measure: only count the device bytes (nothing is touched).
static std::unique_ptr<Hier> build_hier(const std::vector<GridSpec>& specs, gd_dtype s, bool mixed,
                                        hipStream_t st, int tile_force = -1, int first_arrays = 0,
                                        int max_levels = 0, char* arena = nullptr, size_t arena_cap = 0,
                                        bool measure = false) {
  auto H = std::make_unique<Hier>();
  H->arena = arena;
  H->arena_cap = arena_cap;
  H->measure = measure;
  HIP_TRY(hipGetDevice(&H->device));
  H->s = s;
  H->ngrids = (int)specs.size();
  // level descriptors
  std::vector<GridDesc> cur(specs.size());
  for (size_t i = 0; i < specs.size(); ++i) {
    GridDesc g{};
    g.nx = (int32_t)specs[i].nx;
    g.ny = (int32_t)specs[i].ny;
    g.nz = (int32_t)specs[i].nz;
    g.alpha = specs[i].alpha;
    g.wx = specs[i].wx;
    g.wy = specs[i].wy;
    g.wz = specs[i].wz;
    g.ioff = specs[i].ioff;
    g.ipy = specs[i].ipy;
    g.ipz = specs[i].ipz;
    g.zin = specs[i].zin;
    cur[i] = g;
    H->cells.push_back(specs[i].nx * specs[i].ny * specs[i].nz);
  }
  for (;;) {
    Level L;
    int64_t off = 0;
    bool more = false;
    L.row = true;
    L.keep_x = true;
    for (auto& g : cur) {
      g.off = off;
      g.px = pitch_of(g.nx);
      off += (int64_t)g.px * g.ny * g.nz;
      if (g.ny != 1) L.row = false;
      int f[3];
      coarsen_factors(g, f);
      g.fx = f[0]; g.fy = f[1]; g.fz = f[2];
      if (g.fx != 1) L.keep_x = false;
      g.cnx = (g.nx + f[0] - 1) / f[0];
      g.cny = (g.ny + f[1] - 1) / f[1];
      g.cnz = (g.nz + f[2] - 1) / f[2];
      g.cpx = pitch_of(g.cnx);
      if (f[0] * f[1] * f[2] > 1) more = true;
    }
    L.h = cur;
    L.total = off;
    double lc = 0.0;
    for (const auto& g : cur) lc += (double)g.nx * g.ny * g.nz;
    H->lcells.push_back(lc);
    H->lcells_all.push_back(lc);
    H->lv.push_back(std::move(L));
    if (!more || (max_levels > 0 && (int)H->lv.size() >= max_levels)) break;
    std::vector<GridDesc> nxt(cur.size());
    int64_t coff = 0;
    for (size_t i = 0; i < cur.size(); ++i) {
      GridDesc& g = H->lv.back().h[i];
      g.coff = coff;
      GridDesc c{};
      c.nx = g.cnx; c.ny = g.cny; c.nz = g.cnz;
      const double V = (double)g.fx * g.fy * g.fz;
      c.alpha = g.alpha * V;
      c.wx = g.wx * V / (g.fx * g.fx);
      c.wy = g.wy * V / (g.fy * g.fy);
      c.wz = g.wz * V / (g.fz * g.fz);
      nxt[i] = c;
      coff += (int64_t)pitch_of(c.nx) * c.ny * c.nz;
    }
    cur = nxt;
  }
  // last level: no child
  for (auto& g : H->lv.back().h) {
    g.cnx = g.nx; g.cny = g.ny; g.cnz = g.nz; g.cpx = g.px; g.fx = g.fy = g.fz = 1; g.coff = 0;
  }

  // launch tables, device copies, arrays
  const size_t es = dsize(s);
  int64_t maxblocks = 1;
  std::vector<char> stage;
  for (size_t li = 0; li < H->lv.size(); ++li) {
    Level& L = H->lv[li];
    // the finest level aims for more blocks than the coarser ones (its
    // launches are then told apart by their grid size in kernel traces)
    const int64_t tgt = li == 0 ? sweep_target(L.row) : std::max<int64_t>(1, sweep_target(L.row) / 2);
    if (L.row) {
      build_tab(L.sw, L.h, SWR_TX, 1, false, tgt);
      L.sw.order = sweep_order_env() == 1 ? 1 : 0;
      build_tab(L.ew, L.h, EWR_TX, 1, false, 8192);
      build_tab(L.rc, L.h, EWR_TX, 1, true, 8192);
      build_tab(L.rz, L.h, SWR_TX, 1, false, 4096, true);
      build_tab(L.pp, L.h, SWR_TX, 1, false, li == 0 ? 8192 : 4096);
      build_tab(L.cs, L.h, SWR_TX, 1, false, 4096);  // not used: rows take the pair form
    } else {
      int v = tile_force >= 0 ? tile_force : sweep_tile();
      if (v >= kPairTiles && !sweep_wide_tiles_ok(s, true)) v = kPairTiles - 1;  // a quad-only tile
      build_tab(L.sw, L.h, SWEEP_TILE_TX[v], SWEEP_TILE_TY[v], false, tgt);
      L.sw.tile = v;
      L.sw.order = sweep_order_env() == 1 ? 1 : 0;
      build_tab(L.ew, L.h, EW_TX, EW_TY, false, 8192);
      build_tab(L.rc, L.h, EW_TX, EW_TY, true, 8192);
      build_tab(L.rz, L.h, SW_TX, SW_TY, false, 2048, true);
      build_tab(L.pp, L.h, SW_TX, SW_TY, false, li == 0 ? 4096 : 2048);
      const int c4 = stencil4_tile();
      build_tab(L.cs, L.h, CS4_TX[c4], CS4_TY[c4], false, 2048);
      L.cs.tile = c4;
    }
    maxblocks = std::max({maxblocks, L.sw.h_b0.back(), L.ew.h_b0.back(), L.rc.h_b0.back(), L.rz.h_b0.back(),
                          L.pp.h_b0.back(), L.cs.h_b0.back()});
    const size_t nb = (size_t)H->ngrids + 1;
    const size_t gbytes = L.h.size() * sizeof(GridDesc);
    const size_t bytes = gbytes + 6 * nb * sizeof(int64_t);
    char* dev = (char*)H->alloc(bytes);
    L.d = (GridDesc*)dev;
    L.sw.d_b0 = (int64_t*)(dev + gbytes);
    L.ew.d_b0 = L.sw.d_b0 + nb;
    L.rc.d_b0 = L.ew.d_b0 + nb;
    L.rz.d_b0 = L.rc.d_b0 + nb;
    L.pp.d_b0 = L.rz.d_b0 + nb;
    L.cs.d_b0 = L.pp.d_b0 + nb;
    stage.resize(bytes);
    std::memcpy(stage.data(), L.h.data(), gbytes);
    const Tab* tabs[6] = {&L.sw, &L.ew, &L.rc, &L.rz, &L.pp, &L.cs};
    for (int k = 0; k < 6; ++k)
      std::memcpy(stage.data() + gbytes + k * nb * sizeof(int64_t), tabs[k]->h_b0.data(), nb * sizeof(int64_t));
    if (!measure) HIP_TRY(hipMemcpy(dev, stage.data(), bytes, hipMemcpyHostToDevice));
    if ((int)li >= first_arrays) {
      L.x = H->alloc(L.total * es);
      L.xt = H->alloc(L.total * es);
      L.b = H->alloc(L.total * es);
    }
  }
  H->partials = (double*)H->alloc(maxblocks * 2 * sizeof(double));
  H->dred = (double*)H->alloc(H->ngrids * 2 * sizeof(double));
  H->dscal = (double*)H->alloc(H->ngrids * 4 * sizeof(double));
  if (arena || measure) {
    H->host_pin.assign((size_t)H->ngrids * 4, 0.0);
    H->hpin = H->host_pin.data();
  } else {
    HIP_TRY(hipHostMalloc((void**)&H->hpin, H->ngrids * 4 * sizeof(double), hipHostMallocDefault));
  }
  if (mixed) {
    H->x64 = (double*)H->alloc(H->lv[0].total * sizeof(double));
    H->x64b = (double*)H->alloc(H->lv[0].total * sizeof(double));
  }
  (void)st;
  return H;
}

// ------------------------------------------------------------ autotuning
//
// The relaxation of a large finest 3-D level is timed once per (size,
// storage type) for every tile variant and block target; the fastest is
// kept for this and later hierarchies of that size.  Any tile computes the
// same values (each cell's update depends on its neighbours only), so the
// choice changes time, not results.  GD_AUTOTUNE=0, or a GD_SWEEP_TILE /
// GD_SWEEP_BLOCKS setting, keeps the fixed choice.
struct TuneChoice {
  int tile = 2;
  int order = 0;
  int64_t target = 4096;
  double ms = 0.0;
  bool tuned = false;
};
static std::mutex g_tune_mu;
static std::map<std::tuple<int64_t, int64_t, int64_t, int>, TuneChoice> g_tune;

static bool autotune_on() {
  static bool v = [] {
    const char* e = std::getenv("GD_AUTOTUNE");
    if (e && std::atoi(e) == 0) return false;
    return !std::getenv("GD_SWEEP_TILE") && !std::getenv("GD_SWEEP_BLOCKS") && !std::getenv("GD_SWEEP_BLOCKS_ROW");
  }();
  return v;
}

static void set_sweep_tabs(Hier& H, int tile, int64_t target) {
  for (size_t li = 0; li < H.lv.size(); ++li) {
    Level& L = H.lv[li];
    if (L.row) continue;
    const int64_t tgt = li == 0 ? target : std::max<int64_t>(1, target / 2);
    int64_t* d = L.sw.d_b0;
    build_tab(L.sw, L.h, SWEEP_TILE_TX[tile], SWEEP_TILE_TY[tile], false, tgt);
    L.sw.d_b0 = d;
    L.sw.tile = tile;
    HIP_TRY(hipMemcpy(d, L.sw.h_b0.data(), L.sw.h_b0.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
}

static void set_row_tabs(Hier& H, int64_t target, int order) {
  for (size_t li = 0; li < H.lv.size(); ++li) {
    Level& L = H.lv[li];
    if (!L.row) continue;
    const int64_t tgt = li == 0 ? target : std::max<int64_t>(1, target / 2);
    int64_t* d = L.sw.d_b0;
    build_tab(L.sw, L.h, SWR_TX, 1, false, tgt);
    L.sw.d_b0 = d;
    L.sw.order = order;
    HIP_TRY(hipMemcpy(d, L.sw.h_b0.data(), L.sw.h_b0.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  }
}

// One-line grids (2-D slices): the row tile is fixed; the block target of the
// finest level (2048 .. 16384) and the block order (plain, or a contiguous
// run per XCD: faster for some batches, slower for others) are timed and
// the fastest kept, per set of slice sizes (total cells and count; tile -1
// in the cache key).
static void autotune_rows(Hier& H, hipStream_t st) {
  Level& L = H.lv[0];
  int64_t cells = 0;
  for (const auto& g : L.h) cells += (int64_t)g.nx * g.ny * g.nz;
  if (cells < ((int64_t)1 << 22)) return;
  const auto key = std::make_tuple(cells, (int64_t)H.ngrids, (int64_t)-1, (int)H.s);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      set_row_tabs(H, it->second.target, it->second.order);
      return;
    }
  }
  const size_t es = dsize(H.s);
  HIP_TRY(hipMemsetAsync(L.x, 0, L.total * es, st));
  HIP_TRY(hipMemsetAsync(L.b, 0, L.total * es, st));
  const size_t nb = (size_t)H.ngrids + 1;
  int64_t* d_b0 = nullptr;
  HIP_TRY(hipMalloc(&d_b0, nb * sizeof(int64_t)));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  TuneChoice best;
  best.ms = 1e30;
  best.tile = -1;
  for (int order = 0; order < 2; ++order) {
    if (sweep_order_env() >= 0 && order != sweep_order_env()) continue;
    for (int64_t target : {2048, 4096, 8192, 16384}) {
      Tab t;
      build_tab(t, L.h, SWR_TX, 1, false, target);
      HIP_TRY(hipMemcpyAsync(d_b0, t.h_b0.data(), nb * sizeof(int64_t), hipMemcpyHostToDevice, st));
      t.d_b0 = d_b0;
      t.order = order;
      const Geom geo = t.geom(L.d, H.ngrids, true);
      HIP_TRY(launch_rb_sweep(H.s, geo, L.x, L.xt, L.b, nullptr, 0, st));
      HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) HIP_TRY(launch_rb_sweep(H.s, geo, L.x, L.xt, L.b, nullptr, 0, st));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms / 3.0 < best.ms) {
        best.ms = ms / 3.0;
        best.target = target;
        best.order = order;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_b0);
  best.tuned = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  set_row_tabs(H, best.target, best.order);
}

// wide: the quad form's wide tiles (4, 5) are candidates
static void autotune(Hier& H, hipStream_t st, bool wide) {
  Level& L = H.lv[0];
  if (!autotune_on()) return;
  if (L.row) {
    autotune_rows(H, st);
    return;
  }
  if (H.ngrids != 1) return;
  const GridDesc& g = L.h[0];
  if ((int64_t)g.nx * g.ny * g.nz < ((int64_t)1 << 22)) return;
  const auto key = std::make_tuple((int64_t)g.nx, (int64_t)g.ny, (int64_t)g.nz, (int)H.s);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      set_sweep_tabs(H, it->second.tile, it->second.target);
      return;
    }
  }
  const size_t es = dsize(H.s);
  HIP_TRY(hipMemsetAsync(L.x, 0, L.total * es, st));
  HIP_TRY(hipMemsetAsync(L.b, 0, L.total * es, st));
  int64_t* d_b0 = nullptr;
  HIP_TRY(hipMalloc(&d_b0, 2 * sizeof(int64_t)));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  TuneChoice best;
  best.ms = 1e30;
  const int64_t targets[4] = {1024, 2048, 4096, 8192};
  for (int tile = 0; tile < (wide ? kSweepTiles : kPairTiles); ++tile) {
    for (int64_t target : targets) {
      Tab t;
      build_tab(t, L.h, SWEEP_TILE_TX[tile], SWEEP_TILE_TY[tile], false, target);
      t.tile = tile;
      t.order = L.sw.order;
      HIP_TRY(hipMemcpyAsync(d_b0, t.h_b0.data(), 2 * sizeof(int64_t), hipMemcpyHostToDevice, st));
      t.d_b0 = d_b0;
      Geom geo = t.geom(L.d, 1, false);
      set_split(geo, g);
      HIP_TRY(launch_rb_sweep(H.s, geo, L.x, L.xt, L.b, nullptr, 0, st));  // warm-up
      HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) HIP_TRY(launch_rb_sweep(H.s, geo, L.x, L.xt, L.b, nullptr, 0, st));
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms / 3.0 < best.ms) {
        best.ms = ms / 3.0;
        best.tile = tile;
        best.target = target;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_b0);
  best.tuned = true;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  set_sweep_tabs(H, best.tile, best.target);
}

// -------------------------------------------------------------- workspace

// Cached hierarchies, keyed by what fixes their structure: the grids'
// sizes and coupling weights (the weights decide which axes are halved),
// the storage type and the path.  The screening weight alpha of each grid
// only scales the level operators, so a new alpha (a new batch of slices
// with freshly drawn alphas) is written into the cached level descriptors
// instead of building another hierarchy.  At most kCacheMax hierarchies are
// kept; the least recently used one is freed first (and all idle ones when
// a build runs out of device memory).  A lease holds the hierarchy's lock
// while a solve uses it, so calls of one shape from several threads run one
// after the other.
constexpr size_t kCacheMax = 6;
struct CacheEntry {
  std::unique_ptr<Hier> H;
  std::unique_ptr<std::mutex> mu;
  uint64_t used = 0;
};
static std::mutex g_cache_mu;
static std::map<std::string, CacheEntry> g_cache;
static uint64_t g_cache_tick = 0;

struct HierLease {
  Hier* H = nullptr;
  std::unique_lock<std::mutex> lk;
  Hier* operator->() const { return H; }
  Hier& operator*() const { return *H; }
};

static uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  return h;
}

// free idle cached hierarchies (least recently used first) until at most
// `keep` remain; entries in use are skipped
static void evict_idle(size_t keep) {
  while (g_cache.size() > keep) {
    auto victim = g_cache.end();
    for (auto it = g_cache.begin(); it != g_cache.end(); ++it) {
      if (!it->second.mu->try_lock()) continue;
      it->second.mu->unlock();
      if (victim == g_cache.end() || it->second.used < victim->second.used) victim = it;
    }
    if (victim == g_cache.end()) return;
    g_cache.erase(victim);
  }
}

// Write each grid's alpha into every level (alpha_c = V alpha per level, as
// build_hier derives it) and drop captured graphs, which hold launch
// arguments by value.
static void set_alphas(Hier& H, const std::vector<GridSpec>& specs, hipStream_t st) {
  bool changed = false;
  for (size_t i = 0; i < specs.size(); ++i)
    if (H.lv[0].h[i].alpha != specs[i].alpha) changed = true;
  if (!changed) return;
  HIP_TRY(hipStreamSynchronize(st));
  for (size_t i = 0; i < specs.size(); ++i) {
    double a = specs[i].alpha;
    for (auto& L : H.lv) {
      GridDesc& g = L.h[i];
      g.alpha = a;
      a *= (double)g.fx * g.fy * g.fz;
    }
  }
  for (auto& L : H.lv) HIP_TRY(hipMemcpy(L.d, L.h.data(), L.h.size() * sizeof(GridDesc), hipMemcpyHostToDevice));
  for (auto* T : {&H.hyb, &H.lin})
    for (auto& t : *T) t.alpha = H.lv[0].h[0].alpha;
  for (auto& kv : H.graphs)
    for (auto& g : kv.second)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
  H.graphs.clear();
}

static HierLease get_hier(const char* kind, const std::vector<GridSpec>& specs, gd_dtype s, bool mixed,
                          hipStream_t st, int tile_force, bool quad) {
  const bool wide = sweep_wide_tiles_ok(s, quad);  // the autotuner may pick a quad-only tile
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  // sizes and weights decide the hierarchy; alpha and the caller's layout are updated in place
  std::vector<double> sig;
  for (const auto& g : specs) sig.insert(sig.end(), {(double)g.nx, (double)g.ny, (double)g.nz, g.wx, g.wy, g.wz});
  char key[256];
  std::snprintf(key, sizeof key, "%s|d%d|s%d|m%d|t%d|w%d|n%zu|h%016llx", kind, dev, (int)s, (int)mixed, tile_force,
                (int)wide, specs.size(), (unsigned long long)fnv(sig.data(), sig.size() * sizeof(double)));
  HierLease lease;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
      evict_idle(kCacheMax - 1);
      std::unique_ptr<Hier> H;
      try {
        H = build_hier(specs, s, mixed, st, tile_force);
      } catch (const HipFail& e) {
        if (e.e != hipErrorOutOfMemory) throw;
        evict_idle(0);  // free every idle hierarchy and try once more
        H = build_hier(specs, s, mixed, st, tile_force);
      }
      if (tile_force < 0) autotune(*H, st, wide);
      CacheEntry ce;
      ce.H = std::move(H);
      ce.mu = std::make_unique<std::mutex>();
      it = g_cache.emplace(key, std::move(ce)).first;
    }
    it->second.used = ++g_cache_tick;
    lease.H = it->second.H.get();
    lease.lk = std::unique_lock<std::mutex>(*it->second.mu);
  }
  Hier* H = lease.H;
  set_alphas(*H, specs, st);
  // the caller's layout may differ between calls of the same shape
  auto& L0 = H->lv[0];
  bool changed = false;
  for (size_t i = 0; i < specs.size(); ++i) {
    if (L0.h[i].ioff != specs[i].ioff || L0.h[i].ipy != specs[i].ipy || L0.h[i].ipz != specs[i].ipz) {
      L0.h[i].ioff = specs[i].ioff;
      L0.h[i].ipy = specs[i].ipy;
      L0.h[i].ipz = specs[i].ipz;
      changed = true;
    }
  }
  if (changed) {
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpy(L0.d, L0.h.data(), L0.h.size() * sizeof(GridDesc), hipMemcpyHostToDevice));
  }
  return lease;
}

// --------------------------------------------------------------- V-cycle

// A valid request this library does not build (reported as GD_ERR_UNSUPPORTED).
struct Unsupported : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Hybrid discretisation (Sec. 4.2): per-axis Galerkin tables of every level
// >= 1.  Along one axis the finest level has M_0 = Id and K_0 = L (Neumann
// 3-point); M_{l+1} = P^T M_l P, K_{l+1} = P^T K_l P with P the B-spline
// nesting of the axis (identity when the axis is kept), all tridiagonal.
struct Tri {
  std::vector<double> lo, di, up;  // T[i][i-1], T[i][i], T[i][i+1]
};

static Tri galerkin_1d(const Tri& T, int n, bool halved) {
  const int nc = halved ? (n + 1) / 2 : n;
  Tri C{std::vector<double>(nc, 0.0), std::vector<double>(nc, 0.0), std::vector<double>(nc, 0.0)};
  auto parents = [&](int f, int* c, double* w) -> int {
    if (!halved) { c[0] = f; w[0] = 1.0; return 1; }
    if ((f & 1) == 0) { c[0] = f / 2; w[0] = 1.0; return 1; }
    const int lo = (f - 1) / 2, hi = (f + 1) / 2;
    if (hi < nc) { c[0] = lo; w[0] = 0.5; c[1] = hi; w[1] = 0.5; return 2; }
    c[0] = lo; w[0] = 1.0;
    return 1;
  };
  for (int f = 0; f < n; ++f) {
    int pc[2], qc[2];
    double pw[2], qw[2];
    const int np = parents(f, pc, pw);
    for (int d = -1; d <= 1; ++d) {
      const int g = f + d;
      if (g < 0 || g >= n) continue;
      const double t = d < 0 ? T.lo[f] : (d == 0 ? T.di[f] : T.up[f]);
      if (t == 0.0) continue;
      const int nq = parents(g, qc, qw);
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < nq; ++b) {
          const double v = pw[a] * t * qw[b];
          const int dc = qc[b] - pc[a];
          if (dc == -1) C.lo[pc[a]] += v;
          else if (dc == 0) C.di[pc[a]] += v;
          else if (dc == 1) C.up[pc[a]] += v;
          else throw std::logic_error("Galerkin product left the tridiagonal band");
        }
    }
  }
  return C;
}

// Per-block partial sums of the finest-level residual kernels (one grid).
static void alloc_partials(Hier& H) {
  const GridDesc& g0 = H.lv[0].h[0];
  const int64_t n7 = hyb_residual7_blocks(g0), nt = hyb_residual_blocks(g0);
  H.hyb_part = (double*)H.alloc(std::max(n7, nt) * sizeof(double));
  H.hyb_b0 = (int64_t*)H.alloc(2 * sizeof(int64_t));
  H.tab_b0 = (int64_t*)H.alloc(2 * sizeof(int64_t));
  const int64_t b7[2] = {0, n7}, bt[2] = {0, nt};
  HIP_TRY(hipMemcpy(H.hyb_b0, b7, sizeof b7, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(H.tab_b0, bt, sizeof bt, hipMemcpyHostToDevice));
}

// Tables of the Hybrid (disc 1) or Linear (disc 2) discretisation.  Along
// one axis level 0 has K_0 = L (Neumann 3-point, also the B-spline stiffness
// matrix) and M_0 = Id (Hybrid: the 7-point finest operator) or the B-spline
// mass matrix (1/6, 4/6, 1/6; ends 2/6, 1/6) (Linear).
static void ensure_tables(Hier& H, int disc) {
  std::vector<HybTables>& out = disc == 2 ? H.lin : H.hyb;
  if (!out.empty()) return;
  if (H.ngrids != 1) throw Unsupported("the Hybrid and Linear discretisations are built for single-grid solves only");
  const int nl = (int)H.lv.size();
  const GridDesc& g0 = H.lv[0].h[0];
  if (g0.ny > 65535 * 4 || g0.nz > 65535 * 4)
    throw Unsupported("the Hybrid and Linear discretisations need ny and nz <= 262140");
  Tri M[3], K[3];
  const int n0[3] = {g0.nx, g0.ny, g0.nz};
  for (int a = 0; a < 3; ++a) {
    const int n = n0[a];
    M[a] = Tri{std::vector<double>(n, 0.0), std::vector<double>(n, 1.0), std::vector<double>(n, 0.0)};
    K[a] = Tri{std::vector<double>(n, 0.0), std::vector<double>(n, 0.0), std::vector<double>(n, 0.0)};
    for (int i = 0; i < n; ++i) {
      if (i > 0) { K[a].lo[i] = -1.0; K[a].di[i] += 1.0; }
      if (i + 1 < n) { K[a].up[i] = -1.0; K[a].di[i] += 1.0; }
    }
    if (a == 2 && H.stack_z) {  // a stack of slices: no coupling along z
      std::fill(K[a].lo.begin(), K[a].lo.end(), 0.0);
      std::fill(K[a].di.begin(), K[a].di.end(), 0.0);
      std::fill(K[a].up.begin(), K[a].up.end(), 0.0);
      continue;
    }
    if (disc == 2 && n > 1)
      for (int i = 0; i < n; ++i) {
        M[a].lo[i] = i > 0 ? 1.0 / 6.0 : 0.0;
        M[a].up[i] = i + 1 < n ? 1.0 / 6.0 : 0.0;
        M[a].di[i] = (i > 0 ? 2.0 / 6.0 : 0.0) + (i + 1 < n ? 2.0 / 6.0 : 0.0);
      }
  }
  std::vector<double> host;
  std::vector<size_t> at(3 * nl, 0);
  auto push = [&](int l) {
    for (int a = 0; a < 3; ++a) {
      at[3 * l + a] = host.size();
      for (const auto* v : {&M[a].lo, &M[a].di, &M[a].up, &K[a].lo, &K[a].di, &K[a].up})
        host.insert(host.end(), v->begin(), v->end());
    }
  };
  if (disc == 2) push(0);
  for (int l = 1; l < nl; ++l) {
    const GridDesc& p = H.lv[l - 1].h[0];
    const GridDesc& g = H.lv[l].h[0];
    const int fa[3] = {p.fx, p.fy, p.fz}, np_[3] = {p.nx, p.ny, p.nz}, nn[3] = {g.nx, g.ny, g.nz};
    for (int a = 0; a < 3; ++a) {
      M[a] = galerkin_1d(M[a], np_[a], fa[a] == 2);
      K[a] = galerkin_1d(K[a], np_[a], fa[a] == 2);
      if ((int)M[a].di.size() != nn[a]) throw std::logic_error("discretisation tables: level size mismatch");
    }
    push(l);
  }
  double* dev = (double*)H.alloc(std::max<size_t>(host.size(), 1) * sizeof(double));
  if (!host.empty()) HIP_TRY(hipMemcpy(dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
  if (!H.hyb_part) alloc_partials(H);
  out.assign(nl, HybTables{});
  for (int l = 0; l < nl; ++l) {
    HybTables& T = out[l];
    T.alpha = g0.alpha;
    T.w[0] = g0.wx; T.w[1] = g0.wy; T.w[2] = g0.wz;
    const bool has = disc == 2 || l > 0;
    for (int a = 0; a < 3; ++a) T.t[a] = has ? dev + at[3 * l + a] : nullptr;
  }
}

static void upload_flags(Hier& H, const std::vector<char>& skip, const std::vector<char>& alt, hipStream_t st);

// How a table level is relaxed: eight in-place colour launches, or two
// plane-parity launches (the same values bit for bit).  The parity form
// reads the level once per sweep instead of eight times but runs its four
// in-plane colours one after another in each block, which costs more than
// it saves on small grids and on one-line slice grids: it is used on levels
// of at least 8 rows and 2^20 samples (measured on 1024^2 x 128: level 0
// 2.3 against 3.2 ms per sweep; one-block grids 15 against 11 us).
// GD_HYB_COLOURS=1 / 2 forces the colour / parity form (read at every
// sweep, so one process can compare them).
static int hyb_relax_mode() {
  const char* e = std::getenv("GD_HYB_COLOURS");
  const int v = e ? std::atoi(e) : 0;
  return v == 1 || v == 2 ? v : 0;
}
static bool hyb_parity_launches(const GridDesc& g) {
  const int m = hyb_relax_mode();
  if (m != 0) return m == 2;
  return g.ny >= 8 && (double)g.nx * g.ny * g.nz >= (double)(1 << 20);
}

static void prep(Hier& H, const gd_solve_opts& o) {
  if (o.discretization == 1 || o.discretization == 2) ensure_tables(H, o.discretization);
  H.quad_opt = o.sweep_quad != 0;
  if (H.flags_set) upload_flags(H, {}, {}, nullptr);  // left by a solve that ended in an error
}

static void read_dred(Hier& H, int ncomp, hipStream_t st);

struct Cycler {
  Hier& H;
  hipStream_t st;
  int pre, post, pmode;
  int post0 = -1;  // post-smoothing sweeps of the finest level (-1: as the others)
  bool timing;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> ev_kind;
  std::vector<double> ev_cells;  // finest-level cells the timed launch worked on
  size_t ev_used = 0;

  bool fuse;
  bool quad;  // the relaxation's quad form on the level arrays (FP32 and 16-bit storage)
  int disc;  // 0 Constant; 1 Hybrid (table levels >= 1), 2 Linear (all table levels); B-spline transfers
  bool hyb;  // disc != 0
  const std::vector<HybTables>* T = nullptr;
  Cycler(Hier& h, hipStream_t s, const gd_solve_opts& o)
      : H(h), st(s), pre(o.pre_smooth), post(o.post_smooth), pmode(o.prolong), timing(o.timing != 0),
        fuse(o.fuse_prolong != 0), quad(o.sweep_quad != 0), disc(o.discretization), hyb(o.discretization != 0) {
    if (hyb) {
      T = disc == 2 ? &H.lin : &H.hyb;
      if (T->empty()) throw std::logic_error("discretisation tables not built before the cycle");
    }
  }
  bool table_level(int l) const { return disc == 2 || (disc == 1 && l > 0); }
  // ||b - A x|| of level 0 (FP64 accumulation), r left in the level's spare buffer
  double level0_residual() {
    Level& L = H.lv[0];
    H.count(0, 3.0 * P());
    if (table_level(0)) {
      HIP_TRY(launch_hyb_residual(H.s, L.h[0], (*T)[0], L.x, L.b, L.xt, st, H.hyb_part));
      HIP_TRY(launch_reduce(H.hyb_part, H.tab_b0, 1, 1, H.dred, st));
      read_dred(H, 1, st);
    } else {  // 7-point level (one grid): the fast residual with its own block partials
      if (!H.hyb_part) alloc_partials(H);
      HIP_TRY(launch_hyb_residual7(H.s, L.h[0], L.x, L.b, L.xt, H.hyb_part, st));
      HIP_TRY(launch_reduce(H.hyb_part, H.hyb_b0, 1, 1, H.dred, st));
      read_dred(H, 1, st);
    }
    return std::sqrt(H.hpin[0]);
  }
  ~Cycler() {
    for (auto& p : ev) { (void)hipEventDestroy(p.first); (void)hipEventDestroy(p.second); }
  }

  double P() const { return (double)dsize(H.s); }
  bool x0_zero = false;  // level 0's x is zero before its next sweep (which then does not read it)
  void sweep(int l, const void* ec) {
    Level& L = H.lv[l];
    if (H.czero.size() < H.lv.size()) H.czero.assign(H.lv.size(), 0);
    const bool xz = l == 0 ? x0_zero : H.czero[l] != 0;
    if (l == 0) x0_zero = false;
    else H.czero[l] = 0;
    H.count(l, (xz ? 2.0 : 3.0) * P());  // read x and b, write x
    if (ec) H.count(l + 1, P());
    if (hyb && table_level(l)) {  // 27-point level: 8-colour Gauss-Seidel
      if (!hyb_parity_launches(L.h[0])) {  // one launch per colour, in place
        for (int c = 0; c < 8; ++c) HIP_TRY(launch_hyb_gs8(H.s, L.h[0], (*T)[l], c, L.x, L.b, st));
        return;
      }
      HIP_TRY(launch_hyb_gs8z(H.s, L.h[0], (*T)[l], L.x, L.xt, L.b, st));  // one launch per plane parity
      std::swap(L.x, L.xt);
      return;
    }
    const bool t = timing && l == 0;
    if (t) {
      if (ev_used == ev.size()) {
        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        ev.push_back({a, b});
      }
      HIP_TRY(hipEventRecord(ev[ev_used].first, st));
      if (ev_kind.size() < ev.size()) ev_kind.resize(ev.size());
      if (ev_cells.size() < ev.size()) ev_cells.resize(ev.size());
      ev_kind[ev_used] = xz ? 4 + (L.row ? 1 : 0) : (L.row ? 2 : 0) + (ec ? 1 : 0);
      ev_cells[ev_used] = H.lcells[0];
    }
    Geom g = H.g_sw(l);
    g.quad = quad;
    HIP_TRY(launch_rb_sweep(H.s, g, L.x, L.xt, L.b, ec, pmode, st, xz));
    if (t) HIP_TRY(hipEventRecord(ev[ev_used++].second, st));
    std::swap(L.x, L.xt);
  }
  void smooth(int l, int n, const void* ec = nullptr) {
    for (int i = 0; i < n; ++i) sweep(l, i == 0 ? ec : nullptr);
  }
  // residual of level l restricted into level l + 1 (its x zeroed);
  // with `norm`, per-grid sum r^2 lands in H.dred.  lazy: level l + 1 is
  // relaxed next (a V-cycle's descent), so where that relaxation can start
  // from zero without reading x, x is left as it is and flagged instead
  void restrict_to(int l, bool norm, bool lazy = true) {
    Level& L = H.lv[l];
    Level& C = H.lv[l + 1];
    if (H.czero.size() < H.lv.size()) H.czero.assign(H.lv.size(), 0);
    const int last = (int)H.lv.size() - 1;
    bool lz = false;
    if (lazy && !hyb && (pre > 0 || l + 1 == last)) {
      Geom gc = H.g_sw(l + 1);
      gc.quad = quad;
      lz = sweep_starts_from_zero_ok(H.s, gc);
    }
    H.czero[l + 1] = lz ? 1 : 0;
    H.count(l, 2.0 * P());                   // read x and b
    H.count(l + 1, (lz ? 1.0 : 2.0) * P());  // write coarse b (and x)
    if (hyb) H.count(l, 2.0 * P());  // r written and read again
    if (hyb) {  // residual into the level's spare buffer, then P^T
      if (!table_level(l)) {
        HIP_TRY(launch_hyb_residual7(H.s, L.h[0], L.x, L.b, L.xt, H.hyb_part, st));
        if (norm) HIP_TRY(launch_reduce(H.hyb_part, H.hyb_b0, 1, 1, H.dred, st));
      } else {
        HIP_TRY(launch_hyb_residual(H.s, L.h[0], (*T)[l], L.x, L.b, L.xt, st, norm ? H.hyb_part : nullptr));
        if (norm) HIP_TRY(launch_reduce(H.hyb_part, H.tab_b0, 1, 1, H.dred, st));
      }
      HIP_TRY(launch_hyb_restrict(H.s, L.h[0], L.xt, C.b, C.x, st));
      return;
    }
    HIP_TRY(launch_restrict_z(H.s, H.g_rz(l), L.x, L.b, C.b, lz ? nullptr : C.x, norm ? H.partials : nullptr, st));
    if (norm) HIP_TRY(launch_reduce(H.partials, L.rz.d_b0, H.ngrids, 1, H.dred, st));
  }
  // coarse-grid correction of level l (levels l+1 .. bottom), then post-smoothing
  void correct(int l) {
    below(l + 1);
    Level& C = H.lv[l + 1];
    const int np = (l == 0 && post0 >= 0) ? post0 : post;
    if (hyb) {
      H.count(l, 2.0 * P());
      H.count(l + 1, P());
      HIP_TRY(launch_hyb_prolong(H.s, H.lv[l].h[0], C.x, H.lv[l].x, st));
      smooth(l, np);
    } else if (fuse && np > 0 && H.lv[l].sw.tile == 0) {
      smooth(l, np, C.x);  // prolongation fused into the first sweep's loads
    } else {
      H.count(l, 2.0 * P());
      H.count(l + 1, P());
      HIP_TRY(launch_prolong_pair(H.s, H.g_pp(l), C.x, H.lv[l].x, pmode, H.lv[l].keep_x, st));
      smooth(l, np);
    }
  }
  void below(int l) {
    const int last = (int)H.lv.size() - 1;
    if (l == last) {
      smooth(l, 1);  // one-cell grids: one relaxation is the exact solve
      return;
    }
    smooth(l, pre);
    restrict_to(l, false);
    correct(l);
  }
  // full multigrid start (x of level 0 is zero): the right-hand side
  // restricted to every level, the coarsest solved, then level by level the
  // coarse solution interpolated as the initial guess and one V-cycle run
  void fmg() {
    const int last = (int)H.lv.size() - 1;
    for (int l = 0; l < last; ++l) restrict_to(l, false, false);  // x = 0: r = b
    smooth(last, 1);
    for (int l = last - 1; l >= 0; --l) {
      if (hyb) HIP_TRY(launch_hyb_prolong(H.s, H.lv[l].h[0], H.lv[l + 1].x, H.lv[l].x, st));
      else HIP_TRY(launch_prolong_pair(H.s, H.g_pp(l), H.lv[l + 1].x, H.lv[l].x, pmode, H.lv[l].keep_x, st));
      full(l);
    }
  }
  void full(int l) {  // one V-cycle from level l
    if (l == (int)H.lv.size() - 1) { smooth(l, 1); return; }
    smooth(l, pre);
    restrict_to(l, false);
    correct(l);
  }
  // collect HIP-event times of finest-level sweeps (after a stream sync)
  void harvest() {
    if (!timing || ev_used == 0) return;
    double tot[kTimerKinds] = {}, byt[kTimerKinds] = {};
    int64_t cnt[kTimerKinds] = {};
    for (size_t i = 0; i < ev_used; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev[i].first, ev[i].second));
      const int k = ev_kind[i];
      tot[k] += ms;
      cnt[k] += 1;
      byt[k] += (k >= 4 ? 2.0 : 3.0) * (double)dsize(H.s) * ev_cells[i];
    }
    std::lock_guard<std::mutex> lk(g_timer.mu);
    for (int k = 0; k < kTimerKinds; ++k) {
      if (!cnt[k]) continue;
      g_timer.total_ms[k] += tot[k];
      g_timer.launches[k] += cnt[k];
      g_timer.bytes[k] += byt[k];
    }
    ev_used = 0;
  }
};

// A repeated piece of the solve (e.g. "coarse-grid correction of level 0,
// post-smoothing, next pre-smoothing, restriction with norm") captured once
// into a HIP graph per buffer state and replayed: the launch sequence and
// every argument are fixed by the hierarchy and the options, except which of
// a level's two x buffers is current, so one graph is kept per state.  The
// host's view of the buffers is set to the state the replayed graph leaves.
// No memset or host synchronisation is inside a captured piece.
struct CycleGraphs {
  Hier& H;
  std::string key;
  CycleGraphs(Hier& h, const std::string& k) : H(h), key(k) {}
  // run `piece` (which launches on the stream it is given) on st, through a graph
  template <typename F>
  void run(hipStream_t st, F&& piece) {
    auto& gs = H.graphs[key];
    const auto now = H.xstate();
    for (auto& g : gs) {
      if (g.from == now) {
        HIP_TRY(hipGraphLaunch(g.exec, st));
        H.set_xstate(g.to);
        H.acct += g.bytes * (H.act / g.act);
        return;
      }
    }
    if (!H.cap) HIP_TRY(hipStreamCreateWithFlags(&H.cap, hipStreamNonBlocking));
    // order the capture stream after the caller's work, capture, then launch
    HIP_TRY(hipStreamSynchronize(st));
    Hier::Graph g;
    g.from = now;
    g.act = H.act;
    hipGraph_t graph = nullptr;
    const double a0 = H.acct;
    HIP_TRY(hipStreamBeginCapture(H.cap, hipStreamCaptureModeThreadLocal));
    piece(H.cap);
    g.bytes = H.acct - a0;  // the first replay below runs what the capture counted
    HIP_TRY(hipStreamEndCapture(H.cap, &graph));
    g.to = H.xstate();
    hipError_t e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(e);
    H.set_xstate(g.from);
    HIP_TRY(hipGraphLaunch(g.exec, st));
    H.set_xstate(g.to);
    gs.push_back(std::move(g));
  }
};

static bool graphs_on(const gd_solve_opts& o) { return o.use_graph != 0 && o.timing == 0; }

static std::string graph_key(const char* what, const gd_solve_opts& o) {
  char k[128];
  std::snprintf(k, sizeof k, "%s|%d|%d|%d|%d|%d|%d|%d", what, o.pre_smooth, o.post_smooth, o.prolong, o.fuse_prolong,
                o.discretization, o.sweep_quad, hyb_relax_mode());
  return k;
}

static void read_dred(Hier& H, int ncomp, hipStream_t st) {
  HIP_TRY(hipMemcpyAsync(H.hpin, H.dred, H.ngrids * ncomp * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
}

// ---------------------------------------------------------- AD / SP solves

struct Problem {
  const void* I0;
  const void* I1;  // SP value target (NULL for AD)
  void* out;
  gd_dtype tin, tout;
  bool gauge;        // AD: mean(x) = mean(I0)
  gd_dtype t1 = GD_F32;  // I1's type (tin, or F32 / F64)
};

struct Outcome {
  int cycles = 0, steps = 0;
  std::vector<int> gcycles;  // per grid, when grids of a batch retire at different cycles
  double bytes = 0.0;  // algorithmic HBM bytes of the solve's kernels
  std::vector<double> rel, bnorm;
  bool converged = false, numeric = false;
};

// Launch geometry of the finest-level stencil passes: the quad form on 3-D
// grids when the caller's inputs allow aligned 4-element accesses (offsets
// and pitches multiples of 4, base addresses aligned) and the solve asks
// for quad forms; otherwise the pair form on the restriction's tiles.
static Geom stencil_geom(const Hier& H, const Problem& P) {
  const Level& L = H.lv[0];
  auto aligned = [](const void* p, gd_dtype t) { return ((uintptr_t)p % (4 * dsize(t))) == 0; };
  const char* env = std::getenv("GD_STENCIL_QUAD");  // 0: the pair form (same values)
  bool q = H.quad_opt && !(env && std::atoi(env) == 0) && !L.row && aligned(P.I0, P.tin) &&
           (!P.I1 || (P.t1 == P.tin && aligned(P.I1, P.t1)));
  for (const auto& g : L.h) q = q && ((g.ioff | g.ipy | g.ipz) & 3) == 0;
  Geom g = q ? H.g_cs(0) : H.g_rz(0);
  g.stencil4 = q;
  return g;
}

// ||b|| of the canonical system per grid (and the correction-form rhs when b_out)
// bytes per cell of reading the caller's inputs (I0, and I1 when given)
static double in_bytes(const Problem& P) { return (double)dsize(P.tin) + (P.I1 ? (double)dsize(P.t1) : 0.0); }

// (one pass; r0, when given, receives the norm of the correction-form
// right-hand side, which is the canonical residual of x = I0)
// Stencil geometry with one plane per block and the plane segments (plane mode).
static Geom plane_geom(Hier& H, const Problem& P, const int64_t*& seg) {
  Geom g = stencil_geom(H, P);
  auto& pn = *H.planes;
  const int f = g.stencil4 ? 1 : 0;
  const Level& L = H.lv[0];
  const GridDesc& G = L.h[0];
  Tab& t = pn.tab[f];
  const int TX = f ? CS4_TX[L.cs.tile] : SW_TX, TY = f ? CS4_TY[L.cs.tile] : SW_TY;
  if (!t.d_b0) {
    const int64_t txy = (int64_t)((G.nx + TX - 1) / TX) * ((G.ny + TY - 1) / TY);
    build_tab(t, L.h, TX, TY, false, txy * G.nz);  // as many blocks as tiles: one plane each
    t.tile = L.cs.tile;
    t.d_b0 = (int64_t*)H.alloc(2 * sizeof(int64_t));
    HIP_TRY(hipMemcpy(t.d_b0, t.h_b0.data(), 2 * sizeof(int64_t), hipMemcpyHostToDevice));
    std::vector<int64_t> sg(G.nz + 1);
    for (int z = 0; z <= G.nz; ++z) sg[z] = (int64_t)z * txy;
    pn.seg[f] = (int64_t*)H.alloc(sg.size() * sizeof(int64_t));
    HIP_TRY(hipMemcpy(pn.seg[f], sg.data(), sg.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (t.h_b0.back() > pn.part_blocks) {
      pn.part = (double*)H.alloc(2 * t.h_b0.back() * sizeof(double));
      pn.part_blocks = t.h_b0.back();
    }
    if (!pn.red) {
      pn.red = (double*)H.alloc(2 * (size_t)G.nz * sizeof(double));
      pn.host.resize(2 * (size_t)G.nz);
    }
  }
  Geom q = t.geom(L.d, 1, false);
  q.stencil4 = g.stencil4;
  seg = pn.seg[f];
  return q;
}

// per-plane sums (ncomp per plane) of the partials of a plane-mode pass
static void read_planes(Hier& H, const int64_t* seg, int ncomp, hipStream_t st) {
  auto& pn = *H.planes;
  const int nz = H.lv[0].h[0].nz;
  HIP_TRY(launch_reduce(pn.part, seg, nz, ncomp, pn.red, st));
  HIP_TRY(hipMemcpyAsync(pn.host.data(), pn.red, (size_t)nz * ncomp * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
}

static void canonical_norms(Hier& H, const Problem& P, void* b_out, void* x_zero, std::vector<double>& bn,
                            hipStream_t st, std::vector<double>* r0 = nullptr, const double* inv_scale = nullptr) {
  H.count(0, in_bytes(P) + (b_out ? dsize(H.s) : 0) + (x_zero ? dsize(H.s) : 0));
  if (H.planes) {  // per plane of the stack
    const int64_t* seg = nullptr;
    const Geom g = plane_geom(H, P, seg);
    HIP_TRY(launch_rhs_corr(P.tin, P.t1, H.s, g, P.I0, P.I1, b_out, x_zero, H.planes->part, st, inv_scale));
    read_planes(H, seg, 2, st);
    const int nz = H.lv[0].h[0].nz;
    bn.resize(nz);
    for (int z = 0; z < nz; ++z) bn[z] = std::sqrt(H.planes->host[2 * z]);
    if (r0) {
      r0->resize(nz);
      for (int z = 0; z < nz; ++z) (*r0)[z] = std::sqrt(H.planes->host[2 * z + 1]);
    }
    return;
  }
  const Geom g = stencil_geom(H, P);
  HIP_TRY(launch_rhs_corr(P.tin, P.t1, H.s, g, P.I0, P.I1, b_out, x_zero, H.partials, st, inv_scale));
  HIP_TRY(launch_reduce(H.partials, g.block0, H.ngrids, 2, H.dred, st));
  read_dred(H, 2, st);
  bn.resize(H.ngrids);
  for (int g = 0; g < H.ngrids; ++g) bn[g] = std::sqrt(H.hpin[2 * g]);
  if (r0) {
    r0->resize(H.ngrids);
    for (int g = 0; g < H.ngrids; ++g) (*r0)[g] = std::sqrt(H.hpin[2 * g + 1]);
  }
}

static std::vector<double> canon_residual(Hier& H, const Problem& P, int mode, void* rout, hipStream_t st) {
  H.count(0, in_bytes(P) + (mode == 0 ? dsize(H.s) : 8.0) + (rout ? dsize(H.s) : 0));
  if (H.planes) {  // per plane of the stack
    const int64_t* seg = nullptr;
    const Geom g = plane_geom(H, P, seg);
    HIP_TRY(launch_canon_residual(P.tin, P.t1, H.s, mode, g, P.I0, P.I1, H.lv[0].x, H.x64, rout,
                                  H.dscal + H.ngrids, H.planes->part, st));
    read_planes(H, seg, 1, st);
    const int nz = H.lv[0].h[0].nz;
    std::vector<double> r(nz);
    for (int z = 0; z < nz; ++z) r[z] = std::sqrt(H.planes->host[z]);
    return r;
  }
  const Geom g = stencil_geom(H, P);
  HIP_TRY(launch_canon_residual(P.tin, P.t1, H.s, mode, g, P.I0, P.I1, H.lv[0].x, H.x64, rout, H.dscal + H.ngrids,
                                H.partials, st));
  HIP_TRY(launch_reduce(H.partials, g.block0, H.ngrids, 1, H.dred, st));
  read_dred(H, 1, st);
  std::vector<double> r(H.ngrids);
  for (int g = 0; g < H.ngrids; ++g) r[g] = std::sqrt(H.hpin[g]);
  return r;
}

static double denom(double bn) { return bn > 0.0 ? bn : 1.0; }

static void finish(Hier& H, const Problem& P, int mode, hipStream_t st) {
  const double* shift = nullptr;
  const double xb = mode == 0 ? (double)dsize(H.s) : 8.0;
  H.count(0, dsize(P.tin) + xb + dsize(P.tout));
  if (P.gauge) {
    H.count(0, dsize(P.tin) + xb);
    HIP_TRY(launch_sum_shift(P.tin, H.s, mode, H.g_ew(0), P.I0, H.lv[0].x, H.x64, H.partials, st, H.lv[0].xt));
    HIP_TRY(launch_reduce(H.partials, H.lv[0].ew.d_b0, H.ngrids, 1, H.dred, st));
    read_dred(H, 1, st);
    for (int g = 0; g < H.ngrids; ++g) H.hpin[g] = H.hpin[g] / (double)H.cells[g];
    HIP_TRY(hipMemcpyAsync(H.dscal + 2 * H.ngrids, H.hpin, H.ngrids * sizeof(double), hipMemcpyHostToDevice, st));
    shift = H.dscal + 2 * H.ngrids;
  }
  HIP_TRY(launch_finalize(P.tin, H.s, P.tout, mode, H.g_ew(0), P.I0, H.lv[0].x, H.x64, shift, P.out, st,
                          H.lv[0].xt));
  HIP_TRY(hipStreamSynchronize(st));
}

// Per-grid flags of the level descriptors (every level; host copy and device).
static void upload_flags(Hier& H, const std::vector<char>& skip, const std::vector<char>& alt, hipStream_t st) {
  if (st) HIP_TRY(hipStreamSynchronize(st));
  else HIP_TRY(hipDeviceSynchronize());  // no stream known: nothing may still read the descriptors
  for (auto& L : H.lv) {
    for (int g = 0; g < H.ngrids; ++g) {
      L.h[g].skip = skip.empty() ? 0 : skip[g];
      L.h[g].alt = alt.empty() ? 0 : alt[g];
    }
    HIP_TRY(hipMemcpy(L.d, L.h.data(), L.h.size() * sizeof(GridDesc), hipMemcpyHostToDevice));
  }
  H.flags_set = !(skip.empty() && alt.empty());
  // byte accounting: only the grids the kernels work on
  for (size_t l = 0; l < H.lv.size(); ++l) {
    double c = 0.0;
    for (const auto& g : H.lv[l].h)
      if (!g.skip) c += (double)g.nx * g.ny * g.nz;
    H.lcells[l] = c;
  }
  H.act = H.lcells_all[0] > 0.0 ? H.lcells[0] / H.lcells_all[0] : 1.0;
}

static bool all_below(const std::vector<double>& r, const std::vector<double>& bn, double tol, bool& bad) {
  bool ok = true;
  for (size_t g = 0; g < r.size(); ++g) {
    if (!std::isfinite(r[g])) bad = true;
    if (!(r[g] <= tol * denom(bn[g]))) ok = false;
  }
  return ok;
}

// Plain path: V-cycles on the correction E = x - I0 in the storage type.
// The convergence test after each pre-smoothing uses the storage-precision
// residual against half the tolerance; a pass is confirmed with the FP64
// canonical residual of x = I0 + E before returning.  The storage precision
// bounds how small the residual of a stored E can be (its rounding error
// times the operator); when three successive cycles gain less than 30 %, the
// solve stops there and reports the FP64 residual it reached.
// In a batch of grids (slices) each grid is retired once its FP64 residual
// meets the tolerance: the cycle kernels then leave it alone (its flag in
// the level descriptors), and the output pass reads its correction from
// whichever of the level's two buffers held it then.
static Outcome solve_plain(Hier& H, const Problem& P, const gd_solve_opts& o, hipStream_t st) {
  prep(H, o);
  Outcome R;
  const double a0 = H.acct;
  const int n = H.ngrids;
  canonical_norms(H, P, H.lv[0].b, H.lv[0].x, R.bnorm, st);
  Cycler cy(H, st, o);
  const bool single = H.lv.size() == 1;
  const bool retire = n > 1 && !single;
  // Per grid: retired, the level-0 buffer that held it then (1: the second),
  // its inner threshold, and whether its own storage residual asked for the
  // FP64 check.  A grid leaves only on a check it asked for, so when it
  // leaves depends on that grid alone, not on the others in the batch.
  std::vector<char> done(n, 0), park(n, 0), asked(n, 0);
  std::vector<double> inner(n, 0.5), rr(n), best(n, INFINITY);
  int ndone = 0;
  void* const buf0 = H.lv[0].x;
  auto which = [&]() { return H.lv[0].x == buf0 ? 0 : 1; };
  R.rel.assign(n, 0.0);
  int stall = 0;
  bool pre_done = false;  // the graph has already run this cycle's pre-smoothing and restriction
  if (o.fmg && !single) {
    cy.fmg();
    R.cycles++;
  }
  for (;;) {
    if (single) {
      cy.smooth(0, 1);
      R.cycles++;
    } else if (!pre_done) {
      cy.smooth(0, o.pre_smooth);
    }
    bool check_final = R.cycles >= o.max_cycles || single;
    bool stop_after = check_final;
    if (!single) {
      if (!pre_done) cy.restrict_to(0, true);
      pre_done = false;
      read_dred(H, 1, st);
      bool bad = false, gained = false, all = true, any = false;
      for (int g = 0; g < n; ++g) {
        if (done[g]) continue;
        rr[g] = std::sqrt(H.hpin[g]);
        if (!std::isfinite(rr[g])) bad = true;
        if (rr[g] < 0.7 * best[g]) gained = true;
        best[g] = std::min(best[g], rr[g]);
        asked[g] = rr[g] <= inner[g] * o.rel_tol * denom(R.bnorm[g]);
        all = all && asked[g];
        any = any || asked[g];
      }
      if (all || (retire && any)) check_final = true;
      if (bad) { R.numeric = true; break; }
      stall = gained ? 0 : stall + 1;
      if (stall >= 3) check_final = stop_after = true;
    } else {
      asked.assign(n, 1);
    }
    if (check_final) {
      std::vector<double> c = canon_residual(H, P, 0, nullptr, st);
      bool bad = false, all = true;
      std::vector<int> leave;
      for (int g = 0; g < n; ++g) {
        if (done[g]) continue;
        if (!std::isfinite(c[g])) bad = true;
        R.rel[g] = c[g] / denom(R.bnorm[g]);
        const bool ok = c[g] <= o.rel_tol * denom(R.bnorm[g]);
        if (!ok) all = false;
        if (asked[g]) {
          if (ok) leave.push_back(g);
          else inner[g] *= 0.25;
        }
      }
      if (bad) { R.numeric = true; break; }
      const bool last = ndone + (int)leave.size() == n;  // every grid has left
      if (last || (!retire && all)) R.converged = true;
      if (R.converged || stop_after) {
        if (!R.converged && all) R.converged = true;  // stopped with every grid below the tolerance
        break;
      }
      if (retire && !leave.empty()) {
        if (R.gcycles.empty()) R.gcycles.assign(n, 0);
        for (int g : leave) {
          done[g] = 1;
          park[g] = (char)which();
          R.gcycles[g] = R.cycles;
        }
        ndone += (int)leave.size();
        upload_flags(H, done, {}, st);
      }
    }
    if (graphs_on(o) && !single) {
      // the correction of this cycle and the next cycle's pre-smoothing and
      // restriction (with its norm), replayed as one graph
      CycleGraphs(H, graph_key("plain", o)).run(st, [&](hipStream_t cs) {
        Cycler c(H, cs, o);
        c.correct(0);
        c.smooth(0, o.pre_smooth);
        c.restrict_to(0, true);
      });
      R.cycles++;
      pre_done = true;
    } else {
      cy.correct(0);
      R.cycles++;
    }
  }
  cy.harvest();
  for (int g = 0; g < (int)R.gcycles.size(); ++g)
    if (!done[g]) R.gcycles[g] = R.cycles;
  if (ndone > 0) {  // every grid back in the kernels' view; retired ones read where they were left
    std::vector<char> alt(n, 0);
    for (int g = 0; g < n; ++g) alt[g] = done[g] && park[g] != which();
    upload_flags(H, {}, alt, st);
  }
  finish(H, P, 0, st);
  if (ndone > 0) upload_flags(H, {}, {}, st);
  cy.harvest();
  R.bytes = H.acct - a0;
  return R;
}

// Plain V-cycles of a stack of equal, independent slices held as one 3-D
// grid with w_z = 0 (z is never coarsened, so every level keeps the slices
// apart): the storage-precision residual of the whole stack decides when to
// look, and the FP64 canonical residual of every slice against its own
// right-hand side decides convergence (each slice to the tolerance).
static Outcome solve_planes(Hier& H, const Problem& P, const gd_solve_opts& o, hipStream_t st) {
  prep(H, o);
  Outcome R;
  const double a0 = H.acct;
  canonical_norms(H, P, H.lv[0].b, H.lv[0].x, R.bnorm, st);
  const int nz = (int)R.bnorm.size();
  double bglob = 0.0;
  for (double b : R.bnorm) bglob += b * b;
  bglob = std::sqrt(bglob);
  Cycler cy(H, st, o);
  // Once the stack's storage residual is below half the tolerance (or stops
  // falling), every cycle checks the slices in FP64; the slices' floors in
  // the storage precision differ (a slice with a small right-hand side has
  // a relatively higher one), so the worst slice decides when to stop.
  bool checking = false, pre_done = false;
  double best = INFINITY, best_worst = INFINITY;
  int stall = 0, stall_c = 0;
  R.rel.assign(nz, 0.0);
  for (;;) {
    if (!pre_done) {
      cy.smooth(0, o.pre_smooth);
      cy.restrict_to(0, true);
    }
    pre_done = false;
    read_dred(H, 1, st);
    const double rr = std::sqrt(H.hpin[0]);
    if (!std::isfinite(rr)) { R.numeric = true; break; }
    stall = rr < 0.7 * best ? 0 : stall + 1;
    best = std::min(best, rr);
    if (rr <= 0.5 * o.rel_tol * denom(bglob) || stall >= 3) checking = true;
    const bool last = R.cycles >= o.max_cycles;
    if (checking || last) {
      std::vector<double> c = canon_residual(H, P, 0, nullptr, st);
      bool bad = false;
      R.converged = all_below(c, R.bnorm, o.rel_tol, bad);
      double worst = 0.0;
      for (int z = 0; z < nz; ++z) {
        R.rel[z] = c[z] / denom(R.bnorm[z]);
        worst = std::max(worst, R.rel[z]);
      }
      if (bad) { R.numeric = true; break; }
      if (R.converged || last) break;
      stall_c = worst < 0.7 * best_worst ? 0 : stall_c + 1;
      best_worst = std::min(best_worst, worst);
      if (stall_c >= 3) break;  // the worst slice has reached its floor
    }
    if (graphs_on(o)) {
      CycleGraphs(H, graph_key("plain", o)).run(st, [&](hipStream_t cs) {
        Cycler c(H, cs, o);
        c.correct(0);
        c.smooth(0, o.pre_smooth);
        c.restrict_to(0, true);
      });
      pre_done = true;
    } else {
      cy.correct(0);
    }
    R.cycles++;
  }
  cy.harvest();
  finish(H, P, 0, st);
  R.bytes = H.acct - a0;
  return R;
}

// Mixed path: FP64 iterate x64 (starting at I0), V-cycles in the storage
// type on the residual scaled to unit RMS (by a power of two).  The
// right-hand-side pass writes the correction-form b, which is the residual
// of x64 = I0, and its norm (in FP16 storage, whose range is narrow, a first
// pass takes the norm and a second writes b already scaled).  One fused pass
// per refinement step applies the update x64 + s e (into the second FP64
// buffer; the first update reads I0 in place of x64), computes the FP64
// canonical residual of the result and writes it, scaled by the RMS of the
// residual before it (so that it is of order one), as the next right-hand
// side.
static Outcome solve_mixed(Hier& H, const Problem& P, const gd_solve_opts& o, hipStream_t st) {
  prep(H, o);
  Outcome R;
  const double a0 = H.acct;
  Cycler cy(H, st, o);
  const size_t es = dsize(H.s);
  const int n = H.ngrids;
  // the power of two nearest the RMS of a residual: scaling by it is exact,
  // so the stored right-hand side does not depend on the last bits of the
  // norm (which depend on the order of its sums)
  auto rms = [&](int g, const std::vector<double>& v) {
    const double q = v[g] / std::sqrt((double)H.cells[g]);
    return (q > 0.0 && std::isfinite(q)) ? std::ldexp(1.0, (int)std::lround(std::log2(q))) : 1.0;
  };
  std::vector<double> r;
  std::vector<double> scale(n, 1.0);  // scale of the right-hand side in L0.b
  if (H.s == GD_F16) {
    canonical_norms(H, P, nullptr, nullptr, R.bnorm, st, &r);
    for (int g = 0; g < n; ++g) {
      scale[g] = rms(g, r);
      H.hpin[3 * n + g] = 1.0 / scale[g];  // a slot the steps below leave alone
    }
    HIP_TRY(hipMemcpyAsync(H.dscal + 3 * n, H.hpin + 3 * n, n * sizeof(double), hipMemcpyHostToDevice, st));
    canonical_norms(H, P, H.lv[0].b, nullptr, R.bnorm, st, &r, H.dscal + 3 * n);
  } else {
    canonical_norms(H, P, H.lv[0].b, nullptr, R.bnorm, st, &r);
  }
  Geom g0sw = H.g_sw(0);
  g0sw.quad = o.sweep_quad != 0;
  const bool zstart = o.pre_smooth > 0 && o.discretization == 0 && sweep_starts_from_zero_ok(H.s, g0sw);
  for (;;) {
    bool bad = false;
    R.converged = all_below(r, R.bnorm, o.rel_tol, bad);
    R.rel.resize(n);
    for (int g = 0; g < n; ++g) R.rel[g] = r[g] / denom(R.bnorm[g]);
    if (bad) { R.numeric = true; break; }
    if (R.converged || R.steps >= o.max_cycles) break;
    // the V-cycles start from zero: the first level-0 sweep skips reading x
    // where its form allows (otherwise x is cleared)
    if (!zstart) {
      H.count(0, (double)es);
      HIP_TRY(hipMemsetAsync(H.lv[0].x, 0, H.lv[0].total * es, st));
    }
    for (int c = 0; c < o.inner_cycles; ++c) {
      const bool z = zstart && c == 0;
      if (graphs_on(o)) {
        CycleGraphs(H, graph_key(z ? "full-zero" : "full", o)).run(st, [&](hipStream_t cs) {
          Cycler c2(H, cs, o);
          c2.x0_zero = z;
          c2.full(0);
        });
      } else {
        cy.x0_zero = z;
        cy.full(0);
      }
      R.cycles++;
    }
    // x64' = x64 + scale e (x64 = I0 before the first update); r = b - A x64';
    // L0.b = r / rms(previous r)
    for (int g = 0; g < n; ++g) {
      H.hpin[g] = scale[g];
      scale[g] = rms(g, r);
      H.hpin[n + g] = 1.0 / scale[g];
    }
    HIP_TRY(hipMemcpyAsync(H.dscal, H.hpin, 2 * n * sizeof(double), hipMemcpyHostToDevice, st));
    const int mode = R.steps == 0 ? 3 : 2;
    H.count(0, in_bytes(P) + (mode == 2 ? 8.0 : 0.0) + es + 8.0 + es);  // read x64, e; write x64', scaled r
    const Geom gs = stencil_geom(H, P);
    HIP_TRY(launch_canon_residual(P.tin, P.t1, H.s, mode, gs, P.I0, P.I1, H.lv[0].x, H.x64, H.lv[0].b,
                                  H.dscal + n, H.partials, st, H.x64b, H.dscal));
    HIP_TRY(launch_reduce(H.partials, gs.block0, n, 1, H.dred, st));
    read_dred(H, 1, st);
    for (int g = 0; g < n; ++g) r[g] = std::sqrt(H.hpin[g]);
    std::swap(H.x64, H.x64b);
    R.steps++;
  }
  if (R.steps == 0) {  // x64 = I0 for the output
    H.count(0, dsize(P.tin) + 8.0);
    HIP_TRY(launch_refine_init(P.tin, H.g_ew(0), P.I0, H.x64, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  cy.harvest();
  finish(H, P, 1, st);
  R.bytes = H.acct - a0;
  return R;
}

// Plain V-cycles on a correction system A E = b already in level 0 (E = 0
// at the start; the gradient-modulation filter and the Linear AD solve)
// until the residual, accumulated in FP64, is at most rel_tol times the
// canonical ||b||.  The residual of E equals the canonical residual of
// I0 + E.
static Outcome solve_corr(Hier& H, const gd_solve_opts& o, double bnorm, hipStream_t st) {
  prep(H, o);
  Outcome R;
  const double a0 = H.acct;
  R.bnorm = {bnorm};
  Cycler cy(H, st, o);
  const bool single = H.lv.size() == 1;
  const double den = denom(bnorm);
  double best = INFINITY, inner = 0.5;
  int stall = 0;
  auto full_residual = [&]() { return cy.level0_residual(); };
  for (;;) {
    bool check_final = R.cycles >= o.max_cycles || single, stop_after = check_final;
    if (single) {
      cy.smooth(0, 1);
      R.cycles++;
    } else {
      cy.smooth(0, o.pre_smooth);
      cy.restrict_to(0, true);
      read_dred(H, 1, st);
      const double rr = std::sqrt(H.hpin[0]);
      if (!std::isfinite(rr)) { R.numeric = true; break; }
      stall = rr < 0.7 * best ? 0 : stall + 1;
      best = std::min(best, rr);
      if (rr <= inner * o.rel_tol * den) check_final = true;
      if (stall >= 3) check_final = stop_after = true;
    }
    if (check_final) {
      const double rr = full_residual();
      R.rel = {rr / den};
      if (!std::isfinite(rr)) { R.numeric = true; break; }
      R.converged = rr <= o.rel_tol * den;
      if (R.converged || stop_after) break;
      inner *= 0.25;
    }
    if (!single) {
      cy.correct(0);
      R.cycles++;
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  cy.harvest();
  R.bytes = H.acct - a0;
  return R;
}

// AD (Eq. (1)) with the Linear discretisation: b = (b_x Kx My Mz + b_y Mx Ky
// Mz) I0 (canonical, its norm only); in correction form E = I1 - I0 the
// system is A E = -b_z Mx My Kz I0.  Both come from the table residual
// against a zero right-hand side, with I0 loaded into level 0.  Then plain
// V-cycles on every table level, and the output I0 + E shifted to the mean
// of I0 (the constants are the null space).
static Outcome solve_linear_ad(Hier& H, const Problem& P, const gd_solve_opts& o, double bx, double by, double bz,
                               hipStream_t st) {
  prep(H, o);
  Level& L0 = H.lv[0];
  const GridDesc& g0 = L0.h[0];
  const size_t es = dsize(H.s);
  HIP_TRY(launch_load_input(P.tin, H.s, g0, P.I0, L0.x, st));
  HIP_TRY(hipMemsetAsync(L0.b, 0, L0.total * es, st));
  HybTables Tb = H.lin[0], Tz = H.lin[0];
  Tb.alpha = 0.0; Tb.w[0] = bx; Tb.w[1] = by; Tb.w[2] = 0.0;
  Tz.alpha = 0.0; Tz.w[0] = 0.0; Tz.w[1] = 0.0; Tz.w[2] = bz;
  HIP_TRY(launch_hyb_residual(H.s, g0, Tb, L0.x, L0.b, L0.xt, st, H.hyb_part));  // -b
  HIP_TRY(launch_reduce(H.hyb_part, H.tab_b0, 1, 1, H.dred, st));
  read_dred(H, 1, st);
  const double bnorm = std::sqrt(H.hpin[0]);
  HIP_TRY(launch_hyb_residual(H.s, g0, Tz, L0.x, L0.b, L0.xt, st));  // -b_z Mx My Kz I0
  HIP_TRY(hipMemcpyAsync(L0.b, L0.xt, L0.total * es, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * es, st));
  Outcome R = solve_corr(H, o, bnorm, st);
  finish(H, P, 0, st);
  HIP_TRY(hipStreamSynchronize(st));
  return R;
}

// SP (Eq. (2)) of one slice with the Linear discretisation: A = alpha Mx My +
// b_x Kx My + b_y Mx Ky on the slice's hat functions.  In correction form
// E = I2 - I0 the system is A E = alpha Mx My (I1 - I0); the canonical
// right-hand side (for the residual's denominator) is alpha Mx My I1 +
// (b_x Kx My + b_y Mx Ky) I0 = A I0 + alpha Mx My (I1 - I0).  Every product
// comes from the table residual r = b - A x of suitable x and b.
static Outcome solve_linear_sp(Hier& H, const Problem& P, const gd_solve_opts& o, hipStream_t st) {
  prep(H, o);
  Level& L0 = H.lv[0];
  const GridDesc& g0 = L0.h[0];
  const size_t es = dsize(H.s);
  HybTables Ta = H.lin[0], Tf = H.lin[0];  // alpha Mx My only; the whole operator
  Ta.w[0] = Ta.w[1] = Ta.w[2] = 0.0;
  // -alpha M (I1 - I0): x = I1 - I0 against b = 0
  HIP_TRY(hipMemsetAsync(L0.b, 0, L0.total * es, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, P.I1, -1.0, 1.0, L0.x, st));
  HIP_TRY(launch_hyb_residual(H.s, g0, Ta, L0.x, L0.b, L0.xt, st));
  // with b = -alpha M (I1 - I0) and x = I0: r = -(canonical right-hand side)
  HIP_TRY(hipMemcpyAsync(L0.b, L0.xt, L0.total * es, hipMemcpyDeviceToDevice, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, nullptr, 1.0, 0.0, L0.x, st));
  HIP_TRY(launch_hyb_residual(H.s, g0, Tf, L0.x, L0.b, L0.xt, st, H.hyb_part));
  HIP_TRY(launch_reduce(H.hyb_part, H.tab_b0, 1, 1, H.dred, st));
  read_dred(H, 1, st);
  const double bnorm = std::sqrt(H.hpin[0]);
  // the correction's right-hand side alpha M (I1 - I0): x = I0 - I1 against b = 0
  HIP_TRY(hipMemsetAsync(L0.b, 0, L0.total * es, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, P.I1, 1.0, -1.0, L0.x, st));
  HIP_TRY(launch_hyb_residual(H.s, g0, Ta, L0.x, L0.b, L0.xt, st));
  HIP_TRY(hipMemcpyAsync(L0.b, L0.xt, L0.total * es, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * es, st));
  H.count(0, 3.0 * (double)dsize(P.tin) + 2.0 * (double)dsize(P.t1) + 14.0 * (double)es);
  Outcome R = solve_corr(H, o, bnorm, st);
  finish(H, P, 0, st);
  HIP_TRY(hipStreamSynchronize(st));
  return R;
}

// ||b - A x|| of every plane of level 0 (table operator T), r left in r
// (a stack of independent slices: one norm per slice)
static std::vector<double> table_planes(Hier& H, const HybTables& T, const void* x, const void* b, void* r,
                                        hipStream_t st) {
  auto& pn = *H.planes;
  const GridDesc& g0 = H.lv[0].h[0];
  const int nz = g0.nz;
  const int64_t nb = hyb_residual_blocks(g0, true);
  if (!pn.tseg) {
    std::vector<int64_t> sg(nz + 1);
    for (int z = 0; z <= nz; ++z) sg[z] = (int64_t)z * (nb / nz);
    pn.tseg = (int64_t*)H.alloc(sg.size() * sizeof(int64_t));
    HIP_TRY(hipMemcpy(pn.tseg, sg.data(), sg.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (nb > pn.part_blocks) {
      pn.part = (double*)H.alloc(2 * nb * sizeof(double));
      pn.part_blocks = nb;
    }
    if (!pn.red) {
      pn.red = (double*)H.alloc(2 * (size_t)nz * sizeof(double));
      pn.host.resize(2 * (size_t)nz);
    }
  }
  HIP_TRY(launch_hyb_residual(H.s, g0, T, x, b, r, st, pn.part, true));
  HIP_TRY(launch_reduce(pn.part, pn.tseg, nz, 1, pn.red, st));
  HIP_TRY(hipMemcpyAsync(pn.host.data(), pn.red, (size_t)nz * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<double> out(nz);
  for (int z = 0; z < nz; ++z) out[z] = std::sqrt(pn.host[z]);
  return out;
}

// The Linear SP of a stack of equal slices as one grid (z indexes the
// slices: M_z = Id, w_z = 0, z never coarsened): the right-hand side and
// the residuals of solve_linear_sp with norms per slice; every slice must
// meet the tolerance against its own right-hand side.
static Outcome solve_linear_sp_stack(Hier& H, const Problem& P, const gd_solve_opts& o, hipStream_t st) {
  prep(H, o);
  Level& L0 = H.lv[0];
  const GridDesc& g0 = L0.h[0];
  const size_t es = dsize(H.s);
  const double a0 = H.acct;
  HybTables Ta = H.lin[0];  // alpha Mx My only
  Ta.w[0] = Ta.w[1] = Ta.w[2] = 0.0;
  Outcome R;
  HIP_TRY(hipMemsetAsync(L0.b, 0, L0.total * es, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, P.I1, -1.0, 1.0, L0.x, st));
  HIP_TRY(launch_hyb_residual(H.s, g0, Ta, L0.x, L0.b, L0.xt, st));
  HIP_TRY(hipMemcpyAsync(L0.b, L0.xt, L0.total * es, hipMemcpyDeviceToDevice, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, nullptr, 1.0, 0.0, L0.x, st));
  R.bnorm = table_planes(H, H.lin[0], L0.x, L0.b, L0.xt, st);  // the canonical right-hand side per slice
  HIP_TRY(hipMemsetAsync(L0.b, 0, L0.total * es, st));
  HIP_TRY(launch_load_comb(P.tin, P.t1, H.s, g0, P.I0, P.I1, 1.0, -1.0, L0.x, st));
  HIP_TRY(launch_hyb_residual(H.s, g0, Ta, L0.x, L0.b, L0.xt, st));
  HIP_TRY(hipMemcpyAsync(L0.b, L0.xt, L0.total * es, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * es, st));
  H.count(0, 3.0 * (double)dsize(P.tin) + 2.0 * (double)dsize(P.t1) + 14.0 * (double)es);
  const int nz = g0.nz;
  double bglob = 0.0;
  for (double v : R.bnorm) bglob += v * v;
  bglob = std::sqrt(bglob);
  Cycler cy(H, st, o);
  const bool single = H.lv.size() == 1;
  // the stack's residual triggers the per-slice checks, as in solve_planes
  bool checking = single;
  double best = INFINITY, best_worst = INFINITY;
  int stall = 0, stall_c = 0;
  R.rel.assign(nz, 0.0);
  for (;;) {
    if (single) {
      cy.smooth(0, 1);
      R.cycles++;
    } else {
      cy.smooth(0, o.pre_smooth);
      cy.restrict_to(0, true);
      read_dred(H, 1, st);
      const double rr = std::sqrt(H.hpin[0]);
      if (!std::isfinite(rr)) { R.numeric = true; break; }
      stall = rr < 0.7 * best ? 0 : stall + 1;
      best = std::min(best, rr);
      if (rr <= 0.5 * o.rel_tol * denom(bglob) || stall >= 3) checking = true;
    }
    const bool last = R.cycles >= o.max_cycles;
    if (checking || last) {
      const std::vector<double> c = table_planes(H, H.lin[0], L0.x, L0.b, L0.xt, st);
      bool bad = false;
      R.converged = all_below(c, R.bnorm, o.rel_tol, bad);
      double worst = 0.0;
      for (int z = 0; z < nz; ++z) {
        R.rel[z] = c[z] / denom(R.bnorm[z]);
        worst = std::max(worst, R.rel[z]);
      }
      if (bad) { R.numeric = true; break; }
      if (R.converged || last) break;
      stall_c = worst < 0.7 * best_worst ? 0 : stall_c + 1;
      best_worst = std::min(best_worst, worst);
      if (stall_c >= 3) break;  // the worst slice has reached its floor
    }
    if (!single) {
      cy.correct(0);
      R.cycles++;
    }
  }
  cy.harvest();
  finish(H, P, 0, st);
  R.bytes = H.acct - a0;
  return R;
}

static void fill_report(gd_solve_report* rep, const Outcome& R, int g, double secs, int levels,
                        double share = 1.0) {
  rep->fallback_used = 0;
  rep->bytes = R.bytes * share;
  rep->cycles = (g < (int)R.gcycles.size()) ? R.gcycles[g] : R.cycles;
  rep->refine_steps = R.steps;
  rep->rel_residual = R.rel.empty() ? 0.0 : R.rel[g];
  rep->b_norm = R.bnorm.empty() ? 0.0 : R.bnorm[g];
  rep->seconds = secs;
  rep->levels = levels;
}

// Standalone single steps: a one-grid level description in a small cached
// device buffer.
struct StepBuf {
  int device = -1;
  char* dev = nullptr;
  size_t cap = 0;
  double* part = nullptr;
  size_t pcap = 0;
};
static std::mutex g_step_mu;
static std::map<int, StepBuf> g_step;

// Kernels address a cell inside one x-y plane with a 32-bit offset (bytes,
// up to 8 per value): planes are limited to 2^28 cells (16384^2).
constexpr int64_t MAX_PLANE = (int64_t)1 << 28;

static gd_status run_guarded(const std::function<gd_status()>& f) {
  try {
    return f();
  } catch (const HipFail& e) {
    if (e.e == hipErrorOutOfMemory) return fail(GD_ERR_NOMEM, std::string("out of device memory in ") + e.what);
    return fail(GD_ERR_HIP, std::string(e.what) + ": " + hipGetErrorString(e.e));
  } catch (const std::bad_alloc&) {
    return fail(GD_ERR_NOMEM, "host allocation failed");
  } catch (const Unsupported& e) {
    return fail(GD_ERR_UNSUPPORTED, e.what());
  } catch (const std::exception& e) {
    return fail(GD_ERR_HIP, e.what());
  }
}

// Scratch of the no-allocation entry point: one file-scope device array per
// GPU (loaded with the library's code object and held until the process
// ends).  In host code the array's name only stands for it; its device
// address on the current device comes from hipGetSymbolAddress, taken once
// per device and kept.  Every call on a device shares that device's array.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static char* scratch_ptr() {
  static std::mutex mu;
  static std::map<int, char*> per_dev;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = per_dev.find(dev);
  if (it != per_dev.end()) return it->second;
  void* p = nullptr;
  HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw std::logic_error("no device address for the scratch array");
  per_dev[dev] = (char*)p;
  return (char*)p;
}

}  // namespace gd

using namespace gd;

// =================================================================== C ABI

extern "C" {

void gd_default_opts(gd_solve_opts* o) {
  if (!o) return;
  o->rel_tol = 1e-6;
  o->max_cycles = 50;
  o->pre_smooth = -1;  // automatic (auto_smooth)
  o->post_smooth = -1;
  o->storage = GD_F32;
  o->fp64_refine = 0;
  o->inner_cycles = 1;
  o->prolong = 0;
  o->timing = 0;
  o->fuse_prolong = 0;
  o->sweep_tile = -1;
  o->use_graph = 1;
  o->fmg = 0;
  o->discretization = 0;
  o->sweep_quad = 1;
}

const char* gd_last_error(void) { return t_err.c_str(); }
const char* gd_version(void) { return "gdstack 0.1 gfx950"; }

// Sweeps per V-cycle left automatic (-1): V(2, 3) for 16-bit storage with
// FP64 refinement (a stronger cycle saves refinement passes, which cost an
// FP64 pass over the finest level each), V(1, 2) otherwise; the fastest
// splits to 1e-6 measured on the 4096^2 x 256 stack.
static void auto_smooth(gd_solve_opts& o) {
  const bool mixed16 = o.fp64_refine && (o.storage == GD_F16 || o.storage == GD_BF16);
  if (o.pre_smooth == -1) o.pre_smooth = mixed16 ? 2 : 1;
  if (o.post_smooth == -1) o.post_smooth = mixed16 ? 3 : 2;
}

static gd_status check_opts(const gd_solve_opts& o) {
  if (!(o.rel_tol > 0.0) || o.max_cycles < 0 || o.pre_smooth < 0 || o.post_smooth < 0 ||
      o.pre_smooth + o.post_smooth < 1 || !valid_dtype(o.storage) || o.inner_cycles < 1 ||
      (o.prolong != 0 && o.prolong != 1) || o.sweep_tile < -1 || o.sweep_tile >= kSweepTiles ||
      o.discretization < 0 || o.discretization > 2 || o.sweep_quad < 0 || o.sweep_quad > 1)
    return fail(GD_ERR_INVALID, "invalid solver options");
  if (o.sweep_tile >= kPairTiles && !sweep_wide_tiles_ok(o.storage, o.sweep_quad != 0))
    return fail(GD_ERR_INVALID, "sweep_tile 4 and 5 need the quad relaxation (FP32/FP16/BF16 storage, sweep_quad = 1)");
  if (!o.fp64_refine && (o.storage == GD_F16 || o.storage == GD_BF16))
    return fail(GD_ERR_UNSUPPORTED, "16-bit storage needs fp64_refine = 1 (its rounding floor is far above 1e-6)");
  return GD_OK;
}

static gd_status smooth_z_args(const std::string& who, const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t,
                               int64_t nx, int64_t ny, int64_t nz, double bx, double by, double bz,
                               const gd_solve_opts* opts, gd_solve_opts& o) {
  if (!I0 || !I1) return fail(GD_ERR_INVALID, who + ": null pointer");
  if ((const void*)I0 == (const void*)I1) return fail(GD_ERR_INVALID, who + ": output aliases input");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX)
    return fail(GD_ERR_INVALID, who + ": bad size");
  if (nx * ny > MAX_PLANE) return fail(GD_ERR_UNSUPPORTED, who + ": x-y plane above 2^28 cells");
  if (!valid_dtype(in_t) || !valid_dtype(out_t)) return fail(GD_ERR_INVALID, who + ": bad dtype");
  if (!(bx >= 0.0) || !(by >= 0.0) || !(bz > 0.0) || !std::isfinite(bx) || !std::isfinite(by) || !std::isfinite(bz))
    return fail(GD_ERR_INVALID, who + ": need beta_x, beta_y >= 0 and beta_z > 0");
  gd_default_opts(&o);
  if (opts) o = *opts;
  auto_smooth(o);
  gd_status s = check_opts(o);
  if (s != GD_OK) return s;
  if (o.discretization == 2 && o.fp64_refine)
    return fail(GD_ERR_UNSUPPORTED, who + ": FP64 refinement is not built for the Linear discretisation");
  return GD_OK;
}

static Outcome smooth_z_solve(Hier& H, const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, double bx,
                              double by, double bz, const gd_solve_opts& o, hipStream_t st) {
  Problem P{I0, nullptr, I1, in_t, out_t, true, in_t};
  return o.discretization == 2 ? solve_linear_ad(H, P, o, bx, by, bz, st)
         : o.fp64_refine       ? solve_mixed(H, P, o, st)
                               : solve_plain(H, P, o, st);
}

gd_status gd_smooth_z(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny, int64_t nz,
                      double bx, double by, double bz, const gd_solve_opts* opts, gd_solve_report* rep,
                      void* stream) {
  gd_solve_opts o;
  gd_status s = smooth_z_args("gd_smooth_z", I0, in_t, I1, out_t, nx, ny, nz, bx, by, bz, opts, o);
  if (s != GD_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<GridSpec> g{{nx, ny, nz, 0.0, bx, by, bz, 0, nx, nx * ny}};
    HierLease H = get_hier("ad", g, o.storage, o.fp64_refine != 0, st, o.sweep_tile, o.sweep_quad != 0);
    Outcome R = smooth_z_solve(*H, I0, in_t, I1, out_t, bx, by, bz, o, st);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) fill_report(rep, R, 0, secs, (int)H->lv.size());
    if (R.numeric) return fail(GD_ERR_NUMERIC, "gd_smooth_z: non-finite residual");
    if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, "gd_smooth_z: tolerance not reached");
    return GD_OK;
  });
}

gd_status gd_smooth_z_noalloc(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny,
                              int64_t nz, double bx, double by, double bz, const gd_solve_opts* opts,
                              gd_solve_report* rep, void* stream) {
  const char* who = "gd_smooth_z_noalloc";
  gd_solve_opts o;
  gd_status s = smooth_z_args(who, I0, in_t, I1, out_t, nx, ny, nz, bx, by, bz, opts, o);
  if (s != GD_OK) return s;
  if (o.discretization != 0)
    return fail(GD_ERR_UNSUPPORTED, std::string(who) + ": the Constant discretisation only");
  // no graphs and no timing events: neither may be created here
  o.use_graph = 0;
  o.timing = 0;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<GridSpec> g{{nx, ny, nz, 0.0, bx, by, bz, 0, nx, nx * ny}};
    const bool mixed = o.fp64_refine != 0;
    // the device bytes this hierarchy needs, counted without touching the GPU
    const size_t need =
        build_hier(g, o.storage, mixed, st, o.sweep_tile, 0, 0, nullptr, 0, true)->bytes;
    if (need > kScratchBytes)
      return fail(GD_ERR_UNSUPPORTED, std::string(who) + ": needs " + std::to_string(need) +
                                          " bytes of scratch, at most " + std::to_string(kScratchBytes));
    char* arena = scratch_ptr();
    auto H = build_hier(g, o.storage, mixed, st, o.sweep_tile, 0, 0, arena, kScratchBytes);
    Outcome R = smooth_z_solve(*H, I0, in_t, I1, out_t, bx, by, bz, o, st);
    HIP_TRY(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) fill_report(rep, R, 0, secs, (int)H->lv.size());
    if (R.numeric) return fail(GD_ERR_NUMERIC, std::string(who) + ": non-finite residual");
    if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, std::string(who) + ": tolerance not reached");
    return GD_OK;
  });
}

gd_status gd_noalloc_scratch_bytes(int64_t* bytes) {
  if (!bytes) return fail(GD_ERR_INVALID, "gd_noalloc_scratch_bytes: null pointer");
  *bytes = (int64_t)kScratchBytes;
  return GD_OK;
}

gd_status gd_npr_filter(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny, int64_t nz,
                        double alpha, double bx, double by, double bz, double lambda, double sigma,
                        const gd_solve_opts* opts, gd_solve_report* rep, void* stream) {
  if (!I0 || !I1) return fail(GD_ERR_INVALID, "gd_npr_filter: null pointer");
  if ((const void*)I0 == (const void*)I1) return fail(GD_ERR_INVALID, "gd_npr_filter: output aliases input");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX)
    return fail(GD_ERR_INVALID, "gd_npr_filter: bad size");
  if (nx * ny > MAX_PLANE) return fail(GD_ERR_UNSUPPORTED, "gd_npr_filter: x-y plane above 2^28 cells");
  if (!valid_dtype(in_t) || !valid_dtype(out_t)) return fail(GD_ERR_INVALID, "gd_npr_filter: bad dtype");
  if (!(alpha > 0.0) || !std::isfinite(alpha) || !(bx >= 0.0) || !(by >= 0.0) || !(bz >= 0.0) ||
      !std::isfinite(bx) || !std::isfinite(by) || !std::isfinite(bz))
    return fail(GD_ERR_INVALID, "gd_npr_filter: need alpha > 0 and beta >= 0");
  if (!std::isfinite(lambda) || !(sigma > 0.0) || !std::isfinite(sigma))
    return fail(GD_ERR_INVALID, "gd_npr_filter: need a finite lambda and sigma > 0");
  gd_solve_opts o;
  gd_default_opts(&o);
  if (opts) o = *opts;
  auto_smooth(o);
  gd_status s = check_opts(o);
  if (s != GD_OK) return s;
  if (o.fp64_refine) return fail(GD_ERR_UNSUPPORTED, "gd_npr_filter: FP64 refinement is not built for this filter");
  if (o.discretization == 2)
    return fail(GD_ERR_UNSUPPORTED, "gd_npr_filter: the Linear discretisation is built for the AD solve only");
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<GridSpec> g{{nx, ny, nz, alpha, bx, by, bz, 0, nx, nx * ny}};
    HierLease H = get_hier("npr", g, o.storage, false, st, o.sweep_tile, o.sweep_quad != 0);
    Level& L0 = H->lv[0];
    HIP_TRY(launch_npr_rhs(in_t, H->s, H->g_ew(0), I0, lambda, sigma, L0.b, H->partials, st));
    HIP_TRY(launch_reduce(H->partials, L0.ew.d_b0, 1, 2, H->dred, st));
    read_dred(*H, 2, st);
    const double bnorm = std::sqrt(H->hpin[0]);
    HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * dsize(H->s), st));
    Outcome R = solve_corr(*H, o, bnorm, st);
    HIP_TRY(launch_finalize(in_t, H->s, out_t, 0, H->g_ew(0), I0, L0.x, nullptr, nullptr, I1, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) fill_report(rep, R, 0, secs, (int)H->lv.size());
    if (R.numeric) return fail(GD_ERR_NUMERIC, "gd_npr_filter: non-finite residual");
    if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, "gd_npr_filter: tolerance not reached");
    return GD_OK;
  });
}

gd_status gd_screened_poisson_slices(const void* I0, gd_dtype t, const void* I1, gd_dtype t1, void* I2,
                                     gd_dtype tout, const gd_slice_desc* sl, int64_t n, double bx, double by,
                                     const gd_solve_opts* opts, gd_solve_report* rep, gd_solve_report* per,
                                     void* stream) {
  if (n == 0) {  // an empty batch: nothing to solve
    if (rep) std::memset(rep, 0, sizeof *rep);
    return GD_OK;
  }
  if (!I0 || !I1 || !I2 || !sl) return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: null pointer");
  if (I2 == I0 || I2 == I1) return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: output aliases input");
  if (n < 0 || n > (1 << 24)) return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: bad slice count");
  if (!valid_dtype(t) || !valid_dtype(t1) || !valid_dtype(tout))
    return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: bad dtype");
  if (t1 != t && t1 != GD_F32 && t1 != GD_F64)
    return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: I1 must have I0's dtype, F32 or F64");
  if (!(bx >= 0.0) || !(by >= 0.0) || !std::isfinite(bx) || !std::isfinite(by))
    return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: bad beta");
  std::vector<GridSpec> g;
  g.reserve(n);
  for (int64_t i = 0; i < n; ++i) {
    const gd_slice_desc& d = sl[i];
    if (d.nx <= 0 || d.ny <= 0 || d.pitch < d.nx || d.offset < 0 || !(d.alpha > 0.0) || !std::isfinite(d.alpha))
      return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: bad slice descriptor " + std::to_string(i));
    if (d.pitch > MAX_PLANE)
      return fail(GD_ERR_UNSUPPORTED, "gd_screened_poisson_slices: row pitch above 2^28 in slice " + std::to_string(i));
    // the slice's rows become the grid's z axis (one line per plane)
    GridSpec sp{d.nx, 1, d.ny, (double)d.alpha, bx, 0.0, by, d.offset, d.pitch, d.pitch};
    sp.zin = 1;
    g.push_back(sp);
  }
  // slices must not overlap (compare row spans of slices sorted by offset)
  {
    std::vector<std::pair<int64_t, int64_t>> span;
    for (int64_t i = 0; i < n; ++i)
      span.push_back({sl[i].offset, sl[i].offset + (int64_t)sl[i].pitch * (sl[i].ny - 1) + sl[i].nx});
    std::sort(span.begin(), span.end());
    for (size_t i = 1; i < span.size(); ++i)
      if (span[i].first < span[i - 1].second)
        return fail(GD_ERR_INVALID, "gd_screened_poisson_slices: slices overlap");
  }
  gd_solve_opts o;
  gd_default_opts(&o);
  if (opts) o = *opts;
  auto_smooth(o);
  gd_status s = check_opts(o);
  if (s != GD_OK) return s;
  if (o.discretization == 2 && o.fp64_refine)
    return fail(GD_ERR_UNSUPPORTED, "gd_screened_poisson_slices: FP64 refinement is not built for the Linear discretisation");
  hipStream_t st = (hipStream_t)stream;
  // Hybrid (plain V-cycles) or Linear, slices of one size and alpha laid out
  // as a stack (equal pitch, constant stride): one 3-D grid with w_z = 0 (and
  // for Linear M_z = Id), per-slice norms
  bool stack = (o.discretization == 1 || o.discretization == 2) && !o.fp64_refine && n > 1 &&
               (o.discretization != 2 || n <= 65535);  // (Linear: one launch row of blocks per slice)
  for (int64_t i = 1; stack && i < n; ++i)
    stack = sl[i].nx == sl[0].nx && sl[i].ny == sl[0].ny && sl[i].pitch == sl[0].pitch &&
            sl[i].alpha == sl[0].alpha && sl[i].offset - sl[i - 1].offset == sl[1].offset - sl[0].offset &&
            sl[1].offset - sl[0].offset >= (int64_t)sl[0].pitch * sl[0].ny;
  if (stack && (int64_t)sl[0].nx * sl[0].ny <= MAX_PLANE && n <= INT32_MAX) {
    return run_guarded([&]() -> gd_status {
      const auto t0 = std::chrono::steady_clock::now();
      const gd_slice_desc& d = sl[0];
      std::vector<GridSpec> g3{{d.nx, d.ny, n, (double)d.alpha, bx, by, 0.0, d.offset, d.pitch,
                                sl[1].offset - sl[0].offset}};
      HierLease H = get_hier(o.discretization == 2 ? "sp-linear-stack" : "sp-hybrid-stack", g3, o.storage, false, st,
                             o.sweep_tile, o.sweep_quad != 0);
      if (!H->planes) H->planes = std::make_unique<Hier::PlaneNorms>();
      H->stack_z = true;
      Problem P{I0, I1, I2, t, tout, false, t1};
      Outcome R = o.discretization == 2 ? solve_linear_sp_stack(*H, P, o, st) : solve_planes(*H, P, o, st);
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (per)
        for (int64_t i = 0; i < n; ++i) fill_report(&per[i], R, (int)i, secs, (int)H->lv.size(), 1.0 / (double)n);
      if (rep) {
        fill_report(rep, R, 0, secs, (int)H->lv.size());
        double worst = 0.0;
        for (double r : R.rel) worst = std::max(worst, r);
        rep->rel_residual = worst;
        rep->b_norm = 0.0;
      }
      if (R.numeric) return fail(GD_ERR_NUMERIC, "gd_screened_poisson_slices: non-finite residual");
      if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, "gd_screened_poisson_slices: tolerance not reached");
      return GD_OK;
    });
  }
  if (o.discretization != 0) {
    // Hybrid and Linear (Sec. 4.2): each slice is a one-plane grid of its own
    // (the 27-point table levels take one grid per hierarchy), solved in turn;
    // slices of one size share a cached hierarchy
    return run_guarded([&]() -> gd_status {
      const auto t0 = std::chrono::steady_clock::now();
      bool numeric = false, converged = true;
      double worst = 0.0, bytes = 0.0;
      int cycles = 0, steps = 0, levels = 0;
      for (int64_t i = 0; i < n; ++i) {
        const gd_slice_desc& d = sl[i];
        // the slice's rows are the grid's z axis (one line per plane), as in
        // the batched Constant path
        std::vector<GridSpec> g1{{d.nx, 1, d.ny, (double)d.alpha, bx, 0.0, by, d.offset, d.pitch, d.pitch}};
        g1[0].zin = 1;
        HierLease H = get_hier(o.discretization == 1 ? "sp-hybrid" : "sp-linear", g1, o.storage,
                               o.fp64_refine != 0, st, o.sweep_tile, o.sweep_quad != 0);
        Problem P{I0, I1, I2, t, tout, false, t1};
        Outcome R = o.discretization == 2 ? solve_linear_sp(*H, P, o, st)
                    : o.fp64_refine       ? solve_mixed(*H, P, o, st)
                                          : solve_plain(*H, P, o, st);
        if (per) fill_report(&per[i], R, 0, 0.0, (int)H->lv.size());
        numeric = numeric || R.numeric;
        converged = converged && R.converged;
        worst = std::max(worst, R.rel.empty() ? 0.0 : R.rel[0]);
        cycles = std::max(cycles, R.cycles);
        steps = std::max(steps, R.steps);
        levels = std::max(levels, (int)H->lv.size());
        bytes += R.bytes;
      }
      const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (per)
        for (int64_t i = 0; i < n; ++i) per[i].seconds = secs;
      if (rep) {
        std::memset(rep, 0, sizeof *rep);
        rep->cycles = cycles;
        rep->refine_steps = steps;
        rep->rel_residual = worst;
        rep->seconds = secs;
        rep->levels = levels;
        rep->bytes = bytes;
      }
      if (numeric) return fail(GD_ERR_NUMERIC, "gd_screened_poisson_slices: non-finite residual");
      if (!converged) return fail(GD_ERR_NOT_CONVERGED, "gd_screened_poisson_slices: tolerance not reached");
      return GD_OK;
    });
  }
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    HierLease H = get_hier("sp", g, o.storage, o.fp64_refine != 0, st, o.sweep_tile, o.sweep_quad != 0);
    Problem P{I0, I1, I2, t, tout, false, t1};
    Outcome R = o.fp64_refine ? solve_mixed(*H, P, o, st) : solve_plain(*H, P, o, st);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (per) {  // each slice gets its share of the batch's bytes by cells
      double tot = 0.0;
      for (int64_t c : H->cells) tot += (double)c;
      for (int64_t i = 0; i < n; ++i)
        fill_report(&per[i], R, (int)i, secs, (int)H->lv.size(), (double)H->cells[i] / std::max(tot, 1.0));
    }
    if (rep) {
      fill_report(rep, R, 0, secs, (int)H->lv.size());
      rep->cycles = R.cycles;  // the batch: its last slice
      double worst = 0.0;
      for (double r : R.rel) worst = std::max(worst, r);
      rep->rel_residual = worst;
    }
    if (R.numeric) return fail(GD_ERR_NUMERIC, "gd_screened_poisson_slices: non-finite residual");
    if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, "gd_screened_poisson_slices: tolerance not reached");
    return GD_OK;
  });
}

// ------------------------------------------------------------ hierarchy API

// Levels held in host memory (Sec. 4.1: every V-cycle is two streaming
// passes through the data with a window over the slices).  A streamed
// level's z-axis is cut into slabs of `slab` planes; slab [z0, z1) is
// processed in a window [a, e) = [z0 - halo, z1 + halo) clipped to the grid,
// with halo = 2 max(pre, post) + 2 planes: a red-black sweep moves an error
// of the window's cut faces two planes inwards, the residual one more and
// the pairwise restriction stays within an even-aligned pair, so the planes
// [z0, z1) come out as in a sweep of the whole level.  Windows start on even
// planes (slab and halo are even), which keeps the red-black colouring and
// the pairing of planes by the restriction.  Three window buffer sets
// rotate: while one window is relaxed the next two are uploaded and the
// previous one written back, on streams of their own (with two sets an
// upload would wait for the write-back of the set it reuses, and the two
// directions of the host link would take turns instead of overlapping).
// A level is streamed when it has more than an eighth of the finest level's
// cells (with z-first semi-coarsening the first coarse level has half); the
// finest level's x and b are the caller's, a coarser streamed level's are
// pinned host arrays of the library.  Smaller levels stay in HBM.
struct Streamer {
  static constexpr int NS = 3;  // window buffer sets per level
  struct Win {
    int64_t a, e, z0, z1;
  };
  struct Lvl {
    int64_t slab = 0;
    std::vector<Win> wins;
    // window planes -> window hierarchy (levels 0 and 1, launch tables only);
    // the windows of one set share that set's buffers, sized for the largest
    std::map<int64_t, std::unique_ptr<Hier>> sets[NS];
    void* pool[NS] = {};
    size_t pool_bytes = 0;
    void* hx = nullptr;  // pinned host x and b (levels > 0), dense [nz][ny][nx]
    void* hb = nullptr;
    Hier& win(int k, int64_t planes) { return *sets[k].at(planes); }
  };
  int64_t halo = 0;
  std::vector<Lvl> lv;  // streamed levels 0 .. lv.size() - 1
  hipStream_t up = nullptr, down = nullptr;
  hipEvent_t loaded[NS] = {}, copied[NS] = {}, computed[NS] = {}, unloaded[NS] = {}, start = nullptr,
             done_up = nullptr,
             done_down = nullptr;
  size_t bytes() const {
    size_t b = 0;
    for (const auto& L : lv) {
      b += NS * L.pool_bytes;
      for (const auto& m : L.sets)
        for (const auto& kv : m) b += kv.second->bytes;
    }
    return b;
  }
  ~Streamer() {
    for (auto& L : lv) {
      for (void* p : L.pool)
        if (p) (void)hipFree(p);
      if (L.hx) (void)hipHostFree(L.hx);
      if (L.hb) (void)hipHostFree(L.hb);
    }
    for (int k = 0; k < NS; ++k) {
      if (loaded[k]) (void)hipEventDestroy(loaded[k]);
      if (copied[k]) (void)hipEventDestroy(copied[k]);
      if (computed[k]) (void)hipEventDestroy(computed[k]);
      if (unloaded[k]) (void)hipEventDestroy(unloaded[k]);
    }
    if (start) (void)hipEventDestroy(start);
    if (done_up) (void)hipEventDestroy(done_up);
    if (done_down) (void)hipEventDestroy(done_down);
    if (up) (void)hipStreamDestroy(up);
    if (down) (void)hipStreamDestroy(down);
  }
};

struct gd_hierarchy {
  std::unique_ptr<Hier> H;
  std::unique_ptr<Streamer> sm;  // set: the finest level is streamed from host memory
  gd_solve_opts o;
  void* kv[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // Krylov vectors r, z, p, q, t, u
  ~gd_hierarchy() {
    for (void* p : kv)
      if (p) (void)hipFree(p);
  }
};

namespace gd {
// one V-cycle from a zero guess on A z = r (caller's layout, storage dtype)
// z = one V-cycle on A z = r from z = 0; no_post: without the finest
// level's post-smoothing (the learned smoother takes its place)
static void mg_apply(gd_hierarchy* h, const void* r, void* z, hipStream_t st, bool no_post = false) {
  Hier& H = *h->H;
  Level& L0 = H.lv[0];
  const GridDesc& g0 = L0.h[0];
  const size_t es = dsize(H.s);
  const size_t wb = (size_t)g0.nx * es, pb = (size_t)g0.px * es, rows = (size_t)g0.ny * g0.nz;
  HIP_TRY(hipMemcpy2DAsync(L0.b, pb, r, wb, wb, rows, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * es, st));
  prep(H, h->o);
  Cycler cy(H, st, h->o);
  if (no_post) cy.post0 = 0;
  cy.full(0);
  HIP_TRY(hipMemcpy2DAsync(z, wb, L0.x, pb, wb, rows, hipMemcpyDeviceToDevice, st));
  H.count(0, 4.0 * (double)es);  // r in, x cleared, z out (the cycle counts itself)
}

static double reduce1(Hier& H, hipStream_t st) {
  HIP_TRY(launch_reduce(H.partials, H.lv[0].ew.d_b0, 1, 1, H.dred, st));
  read_dred(H, 1, st);
  return H.hpin[0];
}

static void set_coef(Hier& H, double a, double b, hipStream_t st) {
  HIP_TRY(hipStreamSynchronize(st));
  H.hpin[2] = a;
  H.hpin[3] = b;
  HIP_TRY(hipMemcpyAsync(H.dscal, H.hpin + 2, 2 * sizeof(double), hipMemcpyHostToDevice, st));
}
}  // namespace gd

static gd_status hier_args(const std::string& who, int64_t nx, int64_t ny, int64_t nz, double alpha, double bx,
                           double by, double bz, gd_dtype s, const gd_solve_opts* opts, gd_solve_opts& o) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX)
    return fail(GD_ERR_INVALID, who + ": bad size");
  if (nx * ny > MAX_PLANE) return fail(GD_ERR_UNSUPPORTED, who + ": x-y plane above 2^28 cells");
  if (!valid_dtype(s)) return fail(GD_ERR_INVALID, who + ": bad dtype");
  if (!(alpha >= 0.0) || !(bx >= 0.0) || !(by >= 0.0) || !(bz >= 0.0) || !std::isfinite(alpha) ||
      !std::isfinite(bx) || !std::isfinite(by) || !std::isfinite(bz) || (alpha == 0.0 && bx == 0.0 && by == 0.0 && bz == 0.0))
    return fail(GD_ERR_INVALID, who + ": weights must be >= 0 and not all zero");
  gd_default_opts(&o);
  if (opts) o = *opts;
  o.storage = s;
  o.fp64_refine = 0;
  auto_smooth(o);
  if (!(o.rel_tol > 0.0) || o.pre_smooth < 0 || o.post_smooth < 0 || o.pre_smooth + o.post_smooth < 1 ||
      (o.prolong != 0 && o.prolong != 1) || o.sweep_tile < -1 || o.sweep_tile > 3 || o.discretization < 0 ||
      o.discretization > 2 || o.sweep_quad < 0 || o.sweep_quad > 1)
    return fail(GD_ERR_INVALID, who + ": invalid options");
  return GD_OK;
}

gd_status gd_hierarchy_create(gd_hierarchy** h, int64_t nx, int64_t ny, int64_t nz, double alpha, double bx, double by,
                              double bz, gd_dtype s, const gd_solve_opts* opts, void* stream) {
  if (!h) return fail(GD_ERR_INVALID, "gd_hierarchy_create: null handle pointer");
  *h = nullptr;
  gd_solve_opts o;
  const gd_status a = hier_args("gd_hierarchy_create", nx, ny, nz, alpha, bx, by, bz, s, opts, o);
  if (a != GD_OK) return a;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    auto hh = std::make_unique<gd_hierarchy>();
    hh->o = o;
    hh->H = build_hier({{nx, ny, nz, alpha, bx, by, bz, 0, nx, nx * ny}}, s, false, st, o.sweep_tile);
    *h = hh.release();
    return GD_OK;
  });
}

gd_status gd_hierarchy_destroy(gd_hierarchy* h) {
  if (!h) return GD_OK;
  delete h;
  return GD_OK;
}

gd_status gd_hierarchy_info(const gd_hierarchy* h, int level, int* nlevels, int64_t dims[3], double coef[4]) {
  if (!h) return fail(GD_ERR_INVALID, "gd_hierarchy_info: null handle");
  const Hier& H = *h->H;
  if (nlevels) *nlevels = (int)H.lv.size();
  if (level < 0 || level >= (int)H.lv.size()) {
    if (dims || coef) return fail(GD_ERR_INVALID, "gd_hierarchy_info: level out of range");
    return GD_OK;
  }
  const GridDesc& g = H.lv[level].h[0];
  if (dims) { dims[0] = g.nx; dims[1] = g.ny; dims[2] = g.nz; }
  if (coef) { coef[0] = g.alpha; coef[1] = g.wx; coef[2] = g.wy; coef[3] = g.wz; }
  return GD_OK;
}

gd_status gd_rhs_general(gd_hierarchy* h, const void* V, const void* Gx, const void* Gy, const void* Gz, void* b,
                         void* stream) {
  if (h && h->sm) return fail(GD_ERR_INVALID, "gd_rhs_general: the hierarchy streams its finest level (gd_vcycle_streamed)");
  if (!h || !b) return fail(GD_ERR_INVALID, "gd_rhs_general: null pointer");
  Hier& H = *h->H;
  if (H.lv[0].h[0].alpha != 0.0 && !V) return fail(GD_ERR_INVALID, "gd_rhs_general: V is required when alpha > 0");
  if (b == V || b == Gx || b == Gy || b == Gz) return fail(GD_ERR_INVALID, "gd_rhs_general: output aliases input");
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    HIP_TRY(launch_rhs_general(H.s, H.g_ew(0), V, Gx, Gy, Gz, b, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_vcycle(gd_hierarchy* h, void* x, const void* b, int ncycles, double* relres, void* stream) {
  if (h && h->sm) return fail(GD_ERR_INVALID, "gd_vcycle: the hierarchy streams its finest level (gd_vcycle_streamed)");
  if (!h || !x || !b) return fail(GD_ERR_INVALID, "gd_vcycle: null pointer");
  if (x == b) return fail(GD_ERR_INVALID, "gd_vcycle: x aliases b");
  Hier& H = *h->H;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    Level& L0 = H.lv[0];
    const GridDesc& g0 = L0.h[0];
    const size_t es = dsize(H.s);
    const size_t wb = (size_t)g0.nx * es, pb = (size_t)g0.px * es, rows = (size_t)g0.ny * g0.nz;
    prep(H, h->o);
    Cycler cy(H, st, h->o);
    if (ncycles > 0) {
      HIP_TRY(hipMemcpy2DAsync(L0.x, pb, x, wb, wb, rows, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpy2DAsync(L0.b, pb, b, wb, wb, rows, hipMemcpyDeviceToDevice, st));
      for (int c = 0; c < ncycles; ++c) cy.full(0);
      HIP_TRY(hipMemcpy2DAsync(x, wb, L0.x, pb, wb, rows, hipMemcpyDeviceToDevice, st));
    }
    if (relres) {
      HIP_TRY(launch_general_residual(H.s, H.g_ew(0), x, b, nullptr, H.partials, st));
      HIP_TRY(launch_reduce(H.partials, L0.ew.d_b0, 1, 2, H.dred, st));
      read_dred(H, 2, st);
      const double rr = std::sqrt(H.hpin[0]), bb = std::sqrt(H.hpin[1]);
      *relres = bb > 0.0 ? rr / bb : rr;
      if (!std::isfinite(*relres)) return fail(GD_ERR_NUMERIC, "gd_vcycle: non-finite residual");
    }
    HIP_TRY(hipStreamSynchronize(st));
    cy.harvest();
    return GD_OK;
  });
}

// ------------------------------------------------------- streamed levels

gd_status gd_hierarchy_create_streamed(gd_hierarchy** h, int64_t nx, int64_t ny, int64_t nz, double alpha,
                                       double bx, double by, double bz, gd_dtype s, const gd_solve_opts* opts,
                                       int64_t slab, int stream_levels, void* stream) {
  const char* who = "gd_hierarchy_create_streamed";
  if (!h) return fail(GD_ERR_INVALID, std::string(who) + ": null handle pointer");
  *h = nullptr;
  gd_solve_opts o;
  const gd_status a = hier_args(who, nx, ny, nz, alpha, bx, by, bz, s, opts, o);
  if (a != GD_OK) return a;
  if (slab <= 0) return fail(GD_ERR_INVALID, std::string(who) + ": slab must be > 0");
  if (stream_levels < 0) return fail(GD_ERR_INVALID, std::string(who) + ": stream_levels must be >= 0");
  if (o.discretization != 0)
    return fail(GD_ERR_UNSUPPORTED, std::string(who) + ": only the Constant discretisation is streamed");
  if (ny < 2) return fail(GD_ERR_UNSUPPORTED, std::string(who) + ": ny must be >= 2");
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    // levels to stream: the finest, then each next one with more than an
    // eighth of its cells and ny >= 2, always leaving one level resident;
    // stream_levels > 0 caps the count, 0 streams a coarser level only when
    // its window buffers take less HBM than the level itself
    const int64_t halo = 2 * std::max(o.pre_smooth, o.post_smooth) + 2;
    const size_t es = dsize(s);
    int ns = 1;
    {
      auto probe = build_hier({{nx, ny, nz, alpha, bx, by, bz, 0, nx, nx * ny}}, s, false, st, o.sweep_tile, 99);
      if (probe->lv.size() < 2) throw Unsupported("the grid has no coarser level to stream against");
      const GridDesc& f = probe->lv[0].h[0];
      const double cells0 = (double)f.nx * f.ny * f.nz;
      while (ns + 1 < (int)probe->lv.size() && (stream_levels == 0 || ns < stream_levels)) {
        const GridDesc& g = probe->lv[ns].h[0];
        if (g.ny < 2 || 8.0 * g.nx * g.ny * g.nz <= cells0) break;
        if (stream_levels == 0) {
          const int64_t sl = std::min<int64_t>(g.nz, std::max<int64_t>(slab + (slab & 1), halo));
          const int64_t w = std::min<int64_t>(g.nz, sl + 2 * halo);
          const double fine = (double)g.px * g.ny * w * es;
          const double coarse = (double)g.cpx * g.cny * ((w + g.fz - 1) / g.fz) * es;
          const double resident = 3.0 * g.px * g.ny * g.nz * es;
          if (Streamer::NS * (3.0 * fine + 2.0 * coarse) >= resident) break;
        }
        ++ns;
      }
    }
    auto hh = std::make_unique<gd_hierarchy>();
    hh->o = o;
    hh->o.timing = 0;
    hh->H = build_hier({{nx, ny, nz, alpha, bx, by, bz, 0, nx, nx * ny}}, s, false, st, o.sweep_tile, ns);
    Hier& H = *hh->H;
    auto sm = std::make_unique<Streamer>();
    // slab even and at least the halo, so that only the next window reads
    // planes of a slab (its halo) before they are written back
    sm->halo = halo;
    sm->lv.resize(ns);
    for (int l = 0; l < ns; ++l) {
      Streamer::Lvl& SL = sm->lv[l];
      const GridDesc& g = H.lv[l].h[0];
      SL.slab = std::min<int64_t>(g.nz, std::max<int64_t>(slab + (slab & 1), sm->halo));
      for (int64_t z0 = 0; z0 < g.nz; z0 += SL.slab) {
        const int64_t z1 = std::min<int64_t>(g.nz, z0 + SL.slab);
        SL.wins.push_back({std::max<int64_t>(0, z0 - sm->halo), std::min<int64_t>(g.nz, z1 + sm->halo), z0, z1});
      }
      const int tile = H.lv[l].sw.tile;
      int64_t wmax = 0;
      for (const auto& w : SL.wins) {
        wmax = std::max(wmax, w.e - w.a);
        for (int k = 0; k < Streamer::NS; ++k)
          if (!SL.sets[k].count(w.e - w.a))
            SL.sets[k][w.e - w.a] = build_hier({{g.nx, g.ny, w.e - w.a, g.alpha, g.wx, g.wy, g.wz, 0, g.nx,
                                                 (int64_t)g.nx * g.ny}},
                                               s, false, st, tile, 2, 2);
      }
      // per set: the window's x, x', b (wmax planes) and its coarse b and x
      // (the restriction's output; in the up pass the coarse correction)
      const size_t fine = (size_t)g.px * g.ny * wmax * es;
      const size_t coarse = (size_t)g.cpx * g.cny * ((wmax + g.fz - 1) / g.fz) * es;
      const size_t f256 = (fine + 255) & ~(size_t)255, c256 = (coarse + 255) & ~(size_t)255;
      SL.pool_bytes = 3 * f256 + 2 * c256;
      for (int k = 0; k < Streamer::NS; ++k) {
        HIP_TRY(hipMalloc(&SL.pool[k], SL.pool_bytes));
        char* p = (char*)SL.pool[k];
        for (auto& kv : SL.sets[k]) {
          Hier& W = *kv.second;
          W.lv[0].x = p;
          W.lv[0].xt = p + f256;
          W.lv[0].b = p + 2 * f256;
          W.lv[1].b = p + 3 * f256;
          W.lv[1].x = p + 3 * f256 + c256;
          W.lv[1].xt = nullptr;
        }
      }
      if (l > 0) {
        const size_t hbytes = (size_t)g.nx * g.ny * g.nz * es;
        HIP_TRY(hipHostMalloc(&SL.hx, hbytes, hipHostMallocDefault));
        HIP_TRY(hipHostMalloc(&SL.hb, hbytes, hipHostMallocDefault));
      }
    }
    HIP_TRY(hipStreamCreateWithFlags(&sm->up, hipStreamNonBlocking));
    HIP_TRY(hipStreamCreateWithFlags(&sm->down, hipStreamNonBlocking));
    for (int k = 0; k < Streamer::NS; ++k) {
      HIP_TRY(hipEventCreateWithFlags(&sm->loaded[k], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&sm->copied[k], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&sm->computed[k], hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&sm->unloaded[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&sm->start, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&sm->done_up, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&sm->done_down, hipEventDisableTiming));
    hh->sm = std::move(sm);
    *h = hh.release();
    return GD_OK;
  });
}

// One streaming pass over streamed level l (x and b in host memory).
// down: pre-smoothing, then the residual restricted into level l + 1: into
// HBM when that level is resident (its iterate zeroed), into its host b when
// it is streamed too (its iterate then starts at zero in its own down pass,
// so a coarser level's x is not uploaded there).  up: the correction of
// level l + 1 interpolated and added (read in HBM, or uploaded plane range
// by plane range with the window), then post-smoothing.  x is written back
// slab by slab.
static void stream_pass(gd_hierarchy& h, int l, bool down, void* xh, const void* bh, hipStream_t st) {
  Hier& H = *h.H;
  Streamer& S = *h.sm;
  Streamer::Lvl& SL = S.lv[l];
  const bool cs = l + 1 < (int)S.lv.size();  // level l + 1 is streamed too
  Level& C = H.lv[l + 1];
  const GridDesc& g = H.lv[l].h[0];
  const size_t es = dsize(H.s);
  const size_t wb = (size_t)g.nx * es, pb = (size_t)g.px * es;
  const size_t hplane = (size_t)g.nx * g.ny * es, dplane = (size_t)g.px * g.ny * es;
  const size_t cwb = (size_t)g.cnx * es, cpb = (size_t)g.cpx * es;
  const size_t chplane = (size_t)g.cnx * g.cny * es, cplane = (size_t)g.cpx * g.cny * es;
  const int64_t fz = g.fz;
  const bool zero_x = down && l > 0;
  HIP_TRY(hipEventRecord(S.start, st));
  HIP_TRY(hipStreamWaitEvent(S.up, S.start, 0));
  HIP_TRY(hipStreamWaitEvent(S.down, S.start, 0));
  if (down && !cs) HIP_TRY(hipMemsetAsync(C.x, 0, (size_t)C.total * es, st));
  const size_t n = SL.wins.size();
  constexpr int NS = Streamer::NS;
  auto load = [&](size_t w) {  // set w mod NS, last written back for window w - NS
    const Streamer::Win& W = SL.wins[w];
    const int k = (int)(w % NS);
    Hier& WH = SL.win(k, W.e - W.a);
    Level& L = WH.lv[0];
    if (w >= (size_t)NS) HIP_TRY(hipStreamWaitEvent(S.up, S.unloaded[k], 0));
    // planes [a, ov) are shared with the previous window, whose buffers still
    // hold them as they were at the start of this pass (its kernels wait for
    // this copy): copied on the device, so that every plane crosses the host
    // link once per pass
    int64_t ov = W.a;
    if (w > 0) {
      const Streamer::Win& P = SL.wins[w - 1];
      Level& PL = SL.win((int)((w - 1) % NS), P.e - P.a).lv[0];
      ov = std::max(W.a, std::min(P.e, W.e));
      if (ov > W.a) {
        const size_t bytes = (size_t)(ov - W.a) * dplane, off = (size_t)(W.a - P.a) * dplane;
        if (!zero_x)
          HIP_TRY(hipMemcpyAsync(L.x, (const char*)PL.x + off, bytes, hipMemcpyDeviceToDevice, S.up));
        HIP_TRY(hipMemcpyAsync(L.b, (const char*)PL.b + off, bytes, hipMemcpyDeviceToDevice, S.up));
      }
      HIP_TRY(hipEventRecord(S.copied[(w - 1) % NS], S.up));
    }
    const size_t rows = (size_t)g.ny * (W.e - ov), dof = (size_t)(ov - W.a) * dplane;
    if (zero_x) HIP_TRY(hipMemsetAsync(L.x, 0, dplane * (W.e - W.a), S.up));
    else if (rows)
      HIP_TRY(hipMemcpy2DAsync((char*)L.x + dof, pb, (const char*)xh + ov * hplane, wb, wb, rows,
                               hipMemcpyHostToDevice, S.up));
    if (rows)
      HIP_TRY(hipMemcpy2DAsync((char*)L.b + dof, pb, (const char*)bh + ov * hplane, wb, wb, rows,
                               hipMemcpyHostToDevice, S.up));
    if (!down && cs) {  // the coarse correction under the window: planes [a / fz, a / fz + cnz)
      const int64_t cn = WH.lv[0].h[0].cnz;
      HIP_TRY(hipMemcpy2DAsync(WH.lv[1].x, cpb, (const char*)S.lv[l + 1].hx + (W.a / fz) * chplane, cwb, cwb,
                               (size_t)g.cny * cn, hipMemcpyHostToDevice, S.up));
    }
    HIP_TRY(hipEventRecord(S.loaded[k], S.up));
  };
  for (size_t w = 0; w < std::min<size_t>(n, NS - 1); ++w) load(w);
  for (size_t w = 0; w < n; ++w) {
    if (w + NS - 1 < n) load(w + NS - 1);
    const Streamer::Win& W = SL.wins[w];
    const int k = (int)(w % NS);
    Hier& WH = SL.win(k, W.e - W.a);
    HIP_TRY(hipStreamWaitEvent(st, S.loaded[k], 0));
    // the next window copies its shared planes out of this one first
    if (w + 1 < n) HIP_TRY(hipStreamWaitEvent(st, S.copied[k], 0));
    Cycler cy(WH, st, h.o);
    const int64_t c0 = W.z0 / fz, c1 = (W.z1 + fz - 1) / fz;  // coarse planes of [z0, z1)
    if (down) {
      cy.smooth(0, h.o.pre_smooth);
      HIP_TRY(launch_restrict_z(WH.s, WH.g_rz(0), WH.lv[0].x, WH.lv[0].b, WH.lv[1].b, WH.lv[1].x, nullptr, st));
      if (!cs)
        HIP_TRY(hipMemcpyAsync((char*)C.b + c0 * cplane, (const char*)WH.lv[1].b + (c0 - W.a / fz) * cplane,
                               (size_t)(c1 - c0) * cplane, hipMemcpyDeviceToDevice, st));
    } else {
      const void* ec = cs ? WH.lv[1].x : (const void*)((const char*)C.x + (W.a / fz) * cplane);
      if (h.o.fuse_prolong != 0 && h.o.post_smooth > 0 && WH.lv[0].sw.tile == 0) {
        cy.smooth(0, h.o.post_smooth, ec);
      } else {
        HIP_TRY(launch_prolong_pair(WH.s, WH.g_pp(0), ec, WH.lv[0].x, h.o.prolong, WH.lv[0].keep_x, st));
        cy.smooth(0, h.o.post_smooth);
      }
    }
    HIP_TRY(hipEventRecord(S.computed[k], st));
    HIP_TRY(hipStreamWaitEvent(S.down, S.computed[k], 0));
    // the next window's halo holds this slab's last planes as they were
    // before this pass: write back only after it has been read
    if (w + 1 < n) HIP_TRY(hipStreamWaitEvent(S.down, S.loaded[(w + 1) % NS], 0));
    HIP_TRY(hipMemcpy2DAsync((char*)xh + W.z0 * hplane, wb, (const char*)WH.lv[0].x + (W.z0 - W.a) * dplane, pb, wb,
                             (size_t)g.ny * (W.z1 - W.z0), hipMemcpyDeviceToHost, S.down));
    if (down && cs)
      HIP_TRY(hipMemcpy2DAsync((char*)S.lv[l + 1].hb + c0 * chplane, cwb,
                               (const char*)WH.lv[1].b + (c0 - W.a / fz) * cplane, cpb, cwb,
                               (size_t)g.cny * (c1 - c0), hipMemcpyDeviceToHost, S.down));
    HIP_TRY(hipEventRecord(S.unloaded[k], S.down));
  }
  HIP_TRY(hipEventRecord(S.done_up, S.up));
  HIP_TRY(hipEventRecord(S.done_down, S.down));
  HIP_TRY(hipStreamWaitEvent(st, S.done_up, 0));
  HIP_TRY(hipStreamWaitEvent(st, S.done_down, 0));
}

// sum (b - A x)^2 and sum b^2 over the finest level of a streamed hierarchy
// (x, b in host memory), one streaming pass, every window contributing the
// planes of its own slab
static void streamed_residual(gd_hierarchy& h, const void* x, const void* b, double& rr, double& bb,
                              hipStream_t st) {
  Hier& H = *h.H;
  Streamer& S = *h.sm;
  const GridDesc& g0 = H.lv[0].h[0];
  const size_t es = dsize(H.s), wb = (size_t)g0.nx * es, pb = (size_t)g0.px * es;
  const size_t hplane = (size_t)g0.nx * g0.ny * es;
  rr = bb = 0.0;
  for (const auto& W : S.lv[0].wins) {
    Hier& WH = S.lv[0].win(0, W.e - W.a);
    Level& L = WH.lv[0];
    const size_t rows = (size_t)g0.ny * (W.e - W.a);
    HIP_TRY(hipMemcpy2DAsync(L.x, pb, (const char*)x + W.a * hplane, wb, wb, rows, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpy2DAsync(L.b, pb, (const char*)b + W.a * hplane, wb, wb, rows, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_general_residual(WH.s, WH.g_ew(0), L.x, L.b, nullptr, WH.partials, st, true,
                                    (int)(W.z0 - W.a), (int)(W.z1 - W.a)));
    HIP_TRY(launch_reduce(WH.partials, L.ew.d_b0, 1, 2, WH.dred, st));
    read_dred(WH, 2, st);
    rr += WH.hpin[0];
    bb += WH.hpin[1];
  }
}

gd_status gd_vcycle_streamed(gd_hierarchy* h, void* x, const void* b, int ncycles, double* relres, void* stream) {
  if (!h || !x || !b) return fail(GD_ERR_INVALID, "gd_vcycle_streamed: null pointer");
  if (!h->sm) return fail(GD_ERR_INVALID, "gd_vcycle_streamed: the hierarchy keeps its finest level in HBM (gd_vcycle)");
  if (x == b) return fail(GD_ERR_INVALID, "gd_vcycle_streamed: x aliases b");
  if (ncycles < 0) return fail(GD_ERR_INVALID, "gd_vcycle_streamed: ncycles < 0");
  Hier& H = *h->H;
  Streamer& S = *h->sm;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    const int ns = (int)S.lv.size();
    auto X = [&](int l) { return l == 0 ? x : S.lv[l].hx; };
    auto B = [&](int l) { return l == 0 ? b : (const void*)S.lv[l].hb; };
    Cycler cy(H, st, h->o);
    for (int c = 0; c < ncycles; ++c) {
      for (int l = 0; l < ns; ++l) stream_pass(*h, l, true, X(l), B(l), st);
      cy.below(ns);
      for (int l = ns - 1; l >= 0; --l) stream_pass(*h, l, false, X(l), B(l), st);
    }
    if (relres) {  // ||b - A x|| / ||b||, every window contributing its own slab's planes
      double rr = 0.0, bb = 0.0;
      streamed_residual(*h, x, b, rr, bb, st);
      rr = std::sqrt(rr);
      bb = std::sqrt(bb);
      *relres = bb > 0.0 ? rr / bb : rr;
      if (!std::isfinite(*relres)) return fail(GD_ERR_NUMERIC, "gd_vcycle_streamed: non-finite residual");
    }
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

// Anisotropic diffusion of a stack kept in host memory (Sec. 4.1: every pass
// streams the data through a window).  Passes over z-slabs: the right-hand
// side of the correction E = I1 - I0 (and the canonical norm), the V-cycles
// of the streamed hierarchy with the residual checked by a streaming pass,
// the sum of E for the gauge, and the output I0 + E - mean(E) written back
// slab by slab.  E and its right-hand side live in pinned host arrays of the
// library; only windows of planes are in HBM.
gd_status gd_smooth_z_streamed(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny,
                               int64_t nz, double bx, double by, double bz, const gd_solve_opts* opts, int64_t slab,
                               int stream_levels, int64_t device_budget, gd_solve_report* rep, void* stream) {
  const std::string who = "gd_smooth_z_streamed";
  gd_solve_opts o;
  gd_status s0 = smooth_z_args(who, I0, in_t, I1, out_t, nx, ny, nz, bx, by, bz, opts, o);
  if (s0 != GD_OK) return s0;
  if (o.fp64_refine || (o.storage != GD_F32 && o.storage != GD_F64))
    return fail(GD_ERR_UNSUPPORTED, who + ": plain FP32 or FP64 storage only (no refinement)");
  if (o.discretization != 0) return fail(GD_ERR_UNSUPPORTED, who + ": the Constant discretisation only");
  if (slab <= 0 || stream_levels < 0 || device_budget < 0) return fail(GD_ERR_INVALID, who + ": bad slab, levels or budget");
  hipStream_t st = (hipStream_t)stream;
  gd_hierarchy* hp = nullptr;
  gd_status sc = gd_hierarchy_create_streamed(&hp, nx, ny, nz, 0.0, bx, by, bz, o.storage, &o, slab, stream_levels,
                                              stream);
  if (sc != GD_OK) return sc;
  std::unique_ptr<gd_hierarchy> h(hp);
  void* hx = nullptr;
  void* hb = nullptr;
  std::vector<void*> dbufs;
  struct Cleanup {
    void*& hx;
    void*& hb;
    std::vector<void*>& d;
    ~Cleanup() {
      if (hx) (void)hipHostFree(hx);
      if (hb) (void)hipHostFree(hb);
      for (void* p : d) (void)hipFree(p);
    }
  } cleanup{hx, hb, dbufs};
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    Hier& H = *h->H;
    Streamer& S = *h->sm;
    const size_t es = dsize(o.storage), ei = dsize(in_t), eo = dsize(out_t);
    const int64_t pln = nx * ny, px = pitch_of(nx);
    const int64_t sl = S.lv[0].slab;  // planes per slab of the finest level's passes
    // windows of the setup and output passes: the input with one halo plane
    // on each side, the right-hand side and the output (dense), E (level pitch)
    const size_t bi = (size_t)(sl + 2) * pln * ei, bbz = (size_t)sl * pln * es, be = (size_t)sl * px * ny * es,
                 bo = (size_t)sl * pln * eo;
    const int64_t nrb = stream_rhs_blocks(nx, ny);
    auto dalloc = [&](size_t n) {
      void* p = nullptr;
      HIP_TRY(hipMalloc(&p, std::max<size_t>(n, 16)));
      dbufs.push_back(p);
      return p;
    };
    char* wi = (char*)dalloc(bi);
    char* wbz = (char*)dalloc(bbz);
    char* we = (char*)dalloc(be);
    char* wo = (char*)dalloc(bo);
    double* part = (double*)dalloc((size_t)nrb * sizeof(double));
    int64_t* b0 = (int64_t*)dalloc(2 * sizeof(int64_t));
    {
      const int64_t t[2] = {0, nrb};
      HIP_TRY(hipMemcpy(b0, t, sizeof t, hipMemcpyHostToDevice));
    }
    // slab grids (launch tables only) for the sum and output passes
    std::map<int64_t, std::unique_ptr<Hier>> sg;
    auto slab_grid = [&](int64_t planes) -> Hier& {
      auto it = sg.find(planes);
      if (it == sg.end())
        it = sg.emplace(planes, build_hier({{nx, ny, planes, 0.0, bx, by, bz, 0, nx, pln}}, o.storage, false, st, -1,
                                           1, 1)).first;
      return *it->second;
    };
    int64_t dev = (int64_t)(H.bytes + S.bytes() + bi + bbz + be + bo + nrb * sizeof(double));
    if (device_budget > 0 && dev > device_budget)
      return fail(GD_ERR_NOMEM, who + ": needs " + std::to_string(dev) + " device bytes, budget " +
                                    std::to_string(device_budget));
    const size_t host = (size_t)nz * pln * es;
    HIP_TRY(hipHostMalloc(&hx, host, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc(&hb, host, hipHostMallocDefault));
    std::memset(hx, 0, host);  // E starts at zero
    double acct = 0.0;
    // ---- pass 1: right-hand side of E and the canonical norm
    double bn2 = 0.0;
    for (int64_t z0 = 0; z0 < nz; z0 += sl) {
      const int64_t z1 = std::min(nz, z0 + sl), a = std::max<int64_t>(0, z0 - 1), e = std::min(nz, z1 + 1);
      HIP_TRY(hipMemcpyAsync(wi, (const char*)I0 + a * pln * ei, (size_t)(e - a) * pln * ei, hipMemcpyHostToDevice,
                             st));
      HIP_TRY(launch_stream_rhs(in_t, o.storage, wi, wbz, (int)nx, (int)ny, (int)nz, (int)a, (int)(z0 - a),
                                (int)(z1 - a), bx, by, bz, part, st));
      HIP_TRY(launch_reduce(part, b0, 1, 1, H.dred, st));
      HIP_TRY(hipMemcpyAsync((char*)hb + z0 * pln * es, wbz, (size_t)(z1 - z0) * pln * es, hipMemcpyDeviceToHost, st));
      read_dred(H, 1, st);
      bn2 += H.hpin[0];
      acct += (double)(z1 - z0) * pln * (ei + es);
    }
    const double bnorm = std::sqrt(bn2), den = bnorm > 0.0 ? bnorm : 1.0;
    // ---- V-cycles until the canonical residual (that of E's system) is small enough
    Outcome R;
    R.bnorm = {bnorm};
    double rr = 0.0, bb = 0.0;
    int batch = std::min(4, std::max(1, o.max_cycles));
    double best = INFINITY;
    int stall = 0;
    for (;;) {
      gd_status vs = gd_vcycle_streamed(h.get(), hx, hb, batch, nullptr, stream);
      if (vs != GD_OK) return vs;
      R.cycles += batch;
      streamed_residual(*h, hx, hb, rr, bb, st);
      const double rel = std::sqrt(rr) / den;
      R.rel = {rel};
      if (!std::isfinite(rel)) { R.numeric = true; break; }
      R.converged = rel <= o.rel_tol;
      stall = rel < 0.7 * best ? 0 : stall + 1;
      best = std::min(best, rel);
      if (R.converged || R.cycles >= o.max_cycles || stall >= 3) break;
      batch = 1;
    }
    // ---- pass 3: the gauge, mean(I1) = mean(I0): the sum of E
    double esum = 0.0;
    const size_t hplane = (size_t)pln * es, pb = (size_t)px * es, wb = (size_t)nx * es;
    for (int64_t z0 = 0; z0 < nz; z0 += sl) {
      const int64_t z1 = std::min(nz, z0 + sl);
      Hier& G = slab_grid(z1 - z0);
      HIP_TRY(hipMemcpy2DAsync(we, pb, (const char*)hx + z0 * hplane, wb, wb, (size_t)ny * (z1 - z0),
                               hipMemcpyHostToDevice, st));
      HIP_TRY(launch_sum_shift(in_t, o.storage, 0, G.g_ew(0), nullptr, we, nullptr, G.partials, st));
      HIP_TRY(launch_reduce(G.partials, G.lv[0].ew.d_b0, 1, 1, G.dred, st));
      read_dred(G, 1, st);
      esum += G.hpin[0];
    }
    // ---- pass 4: the output I0 + E - mean(E), slab by slab
    H.hpin[0] = esum / ((double)pln * nz);
    HIP_TRY(hipMemcpyAsync(H.dscal, H.hpin, sizeof(double), hipMemcpyHostToDevice, st));
    for (int64_t z0 = 0; z0 < nz; z0 += sl) {
      const int64_t z1 = std::min(nz, z0 + sl);
      Hier& G = slab_grid(z1 - z0);
      HIP_TRY(hipMemcpyAsync(wi, (const char*)I0 + z0 * pln * ei, (size_t)(z1 - z0) * pln * ei, hipMemcpyHostToDevice,
                             st));
      HIP_TRY(hipMemcpy2DAsync(we, pb, (const char*)hx + z0 * hplane, wb, wb, (size_t)ny * (z1 - z0),
                               hipMemcpyHostToDevice, st));
      HIP_TRY(launch_finalize(in_t, o.storage, out_t, 0, G.g_ew(0), wi, we, nullptr, H.dscal, wo, st));
      HIP_TRY(hipMemcpyAsync((char*)I1 + z0 * pln * eo, wo, (size_t)(z1 - z0) * pln * eo, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      acct += (double)(z1 - z0) * pln * (ei + 2.0 * es + eo);
    }
    HIP_TRY(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) {
      fill_report(rep, R, 0, secs, (int)H.lv.size());
      rep->bytes = acct;  // the setup and output passes' bytes (the V-cycles stream through the host link)
    }
    if (R.numeric) return fail(GD_ERR_NUMERIC, who + ": non-finite residual");
    if (!R.converged) return fail(GD_ERR_NOT_CONVERGED, who + ": tolerance not reached");
    return GD_OK;
  });
}

// Per-slice screened Poisson (Eq. (2)) of a stack held in host memory: the
// slices are independent, so batches of `slab` consecutive slices are
// uploaded, solved as one batch in HBM and written back.
gd_status gd_screened_poisson_streamed(const void* I0, gd_dtype in_t, const void* I1, gd_dtype i1_t, void* I2,
                                       gd_dtype out_t, int64_t nx, int64_t ny, int64_t nz, double alpha, double bx,
                                       double by, const gd_solve_opts* opts, int64_t slab, int64_t device_budget,
                                       gd_solve_report* rep, gd_solve_report* per_slice, void* stream) {
  const std::string who = "gd_screened_poisson_streamed";
  if (!I0 || !I1 || !I2) return fail(GD_ERR_INVALID, who + ": null pointer");
  if (I2 == I0 || I2 == I1) return fail(GD_ERR_INVALID, who + ": output aliases input");
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX || nx * ny > MAX_PLANE)
    return fail(GD_ERR_INVALID, who + ": bad size");
  if (!valid_dtype(in_t) || !valid_dtype(i1_t) || !valid_dtype(out_t) ||
      (i1_t != in_t && i1_t != GD_F32 && i1_t != GD_F64))
    return fail(GD_ERR_INVALID, who + ": bad dtype (I1: I0's, F32 or F64)");
  if (!(alpha > 0.0) || !std::isfinite(alpha) || slab <= 0 || device_budget < 0)
    return fail(GD_ERR_INVALID, who + ": need alpha > 0, slab > 0 and a budget >= 0");
  gd_solve_opts o;
  gd_default_opts(&o);
  if (opts) o = *opts;
  auto_smooth(o);
  gd_status sc = check_opts(o);
  if (sc != GD_OK) return sc;
  hipStream_t st = (hipStream_t)stream;
  void* d[3] = {nullptr, nullptr, nullptr};
  struct Free {
    void** d;
    ~Free() {
      for (int i = 0; i < 3; ++i)
        if (d[i]) (void)hipFree(d[i]);
    }
  } fr{d};
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t sl = std::min(slab, nz), pln = nx * ny;
    const size_t ei = dsize(in_t), e1 = dsize(i1_t), eo = dsize(out_t);
    std::vector<GridSpec> specs;
    for (int64_t i = 0; i < sl; ++i) {
      GridSpec g{nx, 1, ny, alpha, bx, 0.0, by, i * pln, nx, nx};
      g.zin = 1;
      specs.push_back(g);
    }
    const size_t hier = o.discretization != 0 ? 0
                        : build_hier(specs, o.storage, o.fp64_refine != 0, st, -1, 0, 0, nullptr, 0, true)->bytes;
    const size_t need = hier + (size_t)sl * pln * (ei + e1 + eo);
    if (device_budget > 0 && (int64_t)need > device_budget)
      return fail(GD_ERR_NOMEM, who + ": needs " + std::to_string(need) + " device bytes, budget " +
                                    std::to_string(device_budget));
    HIP_TRY(hipMalloc(&d[0], (size_t)sl * pln * ei));
    HIP_TRY(hipMalloc(&d[1], (size_t)sl * pln * e1));
    HIP_TRY(hipMalloc(&d[2], (size_t)sl * pln * eo));
    std::vector<gd_slice_desc> descs(sl);
    for (int64_t i = 0; i < sl; ++i) descs[i] = gd_slice_desc{i * pln, (int32_t)nx, (int32_t)ny, (int32_t)nx, (float)alpha};
    std::vector<gd_solve_report> per(sl);
    gd_solve_report sum{};
    bool numeric = false, converged = true;
    for (int64_t z0 = 0; z0 < nz; z0 += sl) {
      const int64_t n = std::min(sl, nz - z0);
      HIP_TRY(hipMemcpyAsync(d[0], (const char*)I0 + z0 * pln * ei, (size_t)n * pln * ei, hipMemcpyHostToDevice, st));
      HIP_TRY(hipMemcpyAsync(d[1], (const char*)I1 + z0 * pln * e1, (size_t)n * pln * e1, hipMemcpyHostToDevice, st));
      gd_solve_report r{};
      const gd_status s2 = gd_screened_poisson_slices(d[0], in_t, d[1], i1_t, d[2], out_t, descs.data(), n, bx, by,
                                                      &o, &r, per.data(), stream);
      if (s2 == GD_ERR_NUMERIC) numeric = true;
      else if (s2 == GD_ERR_NOT_CONVERGED) converged = false;
      else if (s2 != GD_OK) return s2;
      HIP_TRY(hipMemcpyAsync((char*)I2 + z0 * pln * eo, d[2], (size_t)n * pln * eo, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (per_slice) std::memcpy(per_slice + z0, per.data(), (size_t)n * sizeof(gd_solve_report));
      sum.cycles = std::max(sum.cycles, r.cycles);
      sum.refine_steps = std::max(sum.refine_steps, r.refine_steps);
      sum.rel_residual = std::max(sum.rel_residual, r.rel_residual);
      sum.levels = std::max(sum.levels, r.levels);
      sum.bytes += r.bytes;
    }
    sum.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rep) *rep = sum;
    if (numeric) return fail(GD_ERR_NUMERIC, who + ": non-finite residual");
    if (!converged) return fail(GD_ERR_NOT_CONVERGED, who + ": tolerance not reached");
    return GD_OK;
  });
}

gd_status gd_hierarchy_device_bytes(const gd_hierarchy* h, int64_t* bytes, int64_t* window_planes) {
  if (!h || !bytes) return fail(GD_ERR_INVALID, "gd_hierarchy_device_bytes: null pointer");
  size_t b = h->H->bytes;
  int64_t wp = 0;
  if (h->sm) {
    b += h->sm->bytes();
    for (const auto& W : h->sm->lv[0].wins) wp = std::max(wp, W.e - W.a);
  }
  *bytes = (int64_t)b;
  if (window_planes) *window_planes = wp;
  return GD_OK;
}

gd_status gd_hierarchy_streamed_levels(const gd_hierarchy* h, int* levels) {
  if (!h || !levels) return fail(GD_ERR_INVALID, "gd_hierarchy_streamed_levels: null pointer");
  *levels = h->sm ? (int)h->sm->lv.size() : 0;
  return GD_OK;
}

// ---------------------------------------------------- flexible CG + pairs

gd_status gd_mg_error_pairs(gd_hierarchy* h, const void* b, const void* x_star, int cycles, void* r_out, void* e_out,
                            void* stream) {
  if (h && h->sm) return fail(GD_ERR_INVALID, "gd_mg_error_pairs: the hierarchy streams its finest level (gd_vcycle_streamed)");
  if (!h || !b || !x_star || !r_out || !e_out) return fail(GD_ERR_INVALID, "gd_mg_error_pairs: null pointer");
  if (cycles < 0) return fail(GD_ERR_INVALID, "gd_mg_error_pairs: cycles < 0");
  Hier& H = *h->H;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    Level& L0 = H.lv[0];
    const GridDesc& g0 = L0.h[0];
    const size_t es = dsize(H.s);
    const size_t wb = (size_t)g0.nx * es, pb = (size_t)g0.px * es, rows = (size_t)g0.ny * g0.nz;
    // x_k: k V-cycles from zero, left in e_out for the moment
    HIP_TRY(hipMemcpy2DAsync(L0.b, pb, b, wb, wb, rows, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(L0.x, 0, L0.total * es, st));
    prep(H, h->o);
    Cycler cy(H, st, h->o);
    for (int c = 0; c < cycles; ++c) cy.full(0);
    HIP_TRY(hipMemcpy2DAsync(e_out, wb, L0.x, pb, wb, rows, hipMemcpyDeviceToDevice, st));
    // r_k = b - A x_k; e_k = x* - x_k
    HIP_TRY(launch_general_residual(H.s, H.g_ew(0), e_out, b, r_out, H.partials, st));
    set_coef(H, 1.0, -1.0, st);
    HIP_TRY(launch_axpby(H.s, H.g_ew(0), H.dscal, x_star, e_out, e_out, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_fcg_solve(gd_hierarchy* h, gd_net* net, void* x, const void* b, int precond, double rel_tol,
                       int max_iter, gd_solve_report* rep, void* stream) {
  if (h && h->sm) return fail(GD_ERR_INVALID, "gd_fcg_solve: the hierarchy streams its finest level (gd_vcycle_streamed)");
  if (!h || !x || !b) return fail(GD_ERR_INVALID, "gd_fcg_solve: null pointer");
  if (x == b) return fail(GD_ERR_INVALID, "gd_fcg_solve: x aliases b");
  if (precond < 0 || precond > 3 || (precond > 0 && !net))
    return fail(GD_ERR_INVALID,
                "gd_fcg_solve: precond 0 (V-cycle), 1 (net), 2 (V-cycle then net) or 3 (net as the finest "
                "post-smoother) with a net");
  if (!(rel_tol > 0.0) || max_iter < 0) return fail(GD_ERR_INVALID, "gd_fcg_solve: bad tolerance or max_iter");
  Hier& H = *h->H;
  if (H.s != GD_F32) return fail(GD_ERR_UNSUPPORTED, "gd_fcg_solve: FP32 hierarchies only");
  const GridDesc& g0 = H.lv[0].h[0];
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t n = (size_t)g0.nx * g0.ny * g0.nz, bytes = n * 4;
    for (auto& p : h->kv)
      if (!p) HIP_TRY(hipMalloc(&p, bytes));
    void *r = h->kv[0], *z = h->kv[1], *p = h->kv[2], *q = h->kv[3], *t = h->kv[4], *u = h->kv[5];
    const Geom g = H.g_ew(0);
    int mode = precond, fallback = 0, it = 0;
    double bn = 0.0, rn = 0.0;
    const double a0 = H.acct;  // algorithmic bytes: V-cycles and vector kernels (4 B a value), not the net
    auto residual = [&]() {  // r = b - A x, returns ||r||, sets ||b||
      H.count(0, 12.0);
      HIP_TRY(launch_general_residual(H.s, g, x, b, r, H.partials, st));
      HIP_TRY(launch_reduce(H.partials, H.lv[0].ew.d_b0, 1, 2, H.dred, st));
      read_dred(H, 2, st);
      bn = std::sqrt(H.hpin[1]);
      return std::sqrt(H.hpin[0]);
    };
    auto precondition = [&](int m) -> bool {  // z = M(r); false if the net failed
      if (m == 0 || m == 2) mg_apply(h, r, z, st);
      if (m == 3) mg_apply(h, r, z, st, true);
      if (m == 1) {
        if (gd_net_forward(net, (const float*)r, (float*)z, g0.nx, g0.ny, g0.nz, st) != GD_OK) return false;
      } else if (m == 2 || m == 3) {
        // z += net(r - A z); q still holds A p of this iteration and must survive
        H.count(0, 24.0);  // the residual and the sum
        HIP_TRY(launch_general_residual(H.s, g, z, r, t, H.partials, st));
        if (gd_net_forward(net, (const float*)t, (float*)u, g0.nx, g0.ny, g0.nz, st) != GD_OK) return false;
        set_coef(H, 1.0, 1.0, st);
        HIP_TRY(launch_axpby(H.s, g, H.dscal, u, z, z, st));
      }
      return true;
    };
    rn = residual();
    const double den = bn > 0.0 ? bn : 1.0;
    double best = rn;
    int stall = 0, replaced = 0;
    bool restart = true;
    while (it < max_iter) {
      if (rn <= rel_tol * den) {
        // the recurrence says converged: check against b - A x and, if
        // rounding has let the two drift apart, restart from the true residual
        rn = residual();
        if (rn <= rel_tol * den || ++replaced > 4) break;
        restart = true;
      }
      if (restart) {
        if (!precondition(mode)) { mode = 0; fallback = 1; precondition(0); }
        HIP_TRY(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, st));
        H.count(0, 8.0);
        restart = false;
      }
      H.count(0, 8.0 + 8.0 + 24.0);  // q = A p with p.q, p.r, the x and r update
      HIP_TRY(launch_apply_dot(H.s, g, p, q, H.partials, st));
      const double pq = reduce1(H, st);
      HIP_TRY(launch_dot(H.s, g, p, r, H.partials, st));
      const double pr = reduce1(H, st);
      if (!(pq > 0.0) || !std::isfinite(pr)) {  // preconditioner broke A-conjugacy: restart plainly
        if (mode != 0) { mode = 0; fallback = 1; restart = true; continue; }
        return fail(GD_ERR_NUMERIC, "gd_fcg_solve: breakdown (p.Ap <= 0)");
      }
      const double a = pr / pq;
      set_coef(H, a, 0.0, st);
      HIP_TRY(launch_cg_update(H.s, g, H.dscal, x, r, p, q, H.partials, st));
      rn = std::sqrt(reduce1(H, st));
      ++it;
      if (!std::isfinite(rn)) return fail(GD_ERR_NUMERIC, "gd_fcg_solve: non-finite residual");
      if (rn < 0.9 * best) { best = rn; stall = 0; } else if (++stall >= 5 && mode != 0) {
        mode = 0; fallback = 1; restart = true;  // the learned preconditioner stopped helping
        rn = residual();
        continue;
      }
      if (rn <= rel_tol * den) continue;
      if (!precondition(mode)) { mode = 0; fallback = 1; restart = true; continue; }
      H.count(0, 8.0 + 12.0);  // z.q, p = z + beta p
      HIP_TRY(launch_dot(H.s, g, z, q, H.partials, st));
      const double zq = reduce1(H, st);
      set_coef(H, 1.0, -zq / pq, st);
      HIP_TRY(launch_axpby(H.s, g, H.dscal, z, p, p, st));  // p = z + beta p
    }
    const double rtrue = residual();
    HIP_TRY(hipStreamSynchronize(st));
    if (rep) {
      rep->cycles = it;
      rep->refine_steps = 0;
      rep->fallback_used = fallback;
      rep->bytes = H.acct - a0;
      rep->rel_residual = rtrue / den;
      rep->b_norm = bn;
      rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      rep->levels = (int)H.lv.size();
    }
    if (!(rtrue <= rel_tol * den)) return fail(GD_ERR_NOT_CONVERGED, "gd_fcg_solve: tolerance not reached");
    return GD_OK;
  });
}

// --------------------------------------------------------- single steps

static gd_status one_grid(GridDesc& g, int64_t nx, int64_t ny, int64_t nz, int cx, int cy, int cz, double alpha,
                          double wx, double wy, double wz) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX)
    return fail(GD_ERR_INVALID, "bad size");
  if (nx * ny > MAX_PLANE) return fail(GD_ERR_UNSUPPORTED, "x-y plane above 2^28 cells");
  if ((cx != 1 && cx != 2) || (cy != 1 && cy != 2) || (cz != 1 && cz != 2))
    return fail(GD_ERR_INVALID, "coarsening factors must be 1 or 2");
  if (!(alpha >= 0.0) || !(wx >= 0.0) || !(wy >= 0.0) || !(wz >= 0.0))
    return fail(GD_ERR_INVALID, "weights must be >= 0");
  std::memset(&g, 0, sizeof g);
  g.nx = (int32_t)nx; g.ny = (int32_t)ny; g.nz = (int32_t)nz;
  g.fx = cx; g.fy = cy; g.fz = cz;
  g.cnx = (g.nx + cx - 1) / cx; g.cny = (g.ny + cy - 1) / cy; g.cnz = (g.nz + cz - 1) / cz;
  g.alpha = alpha; g.wx = wx; g.wy = wy; g.wz = wz;
  g.ipy = nx; g.ipz = nx * ny;
  g.px = (int32_t)nx; g.cpx = g.cnx;  // the caller's arrays are unpadded
  return GD_OK;
}

// upload one grid + its table for kernel family (TX, TY, child) and return the geometry
static Geom step_geom(const GridDesc& g, int TX, int TY, bool child, int64_t target, int64_t& nblocks,
                      double** part, hipStream_t st, bool even = false) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_step_mu);
  StepBuf& sb = g_step[dev];
  Tab t;
  build_tab(t, {g}, TX, TY, child, target, even);
  nblocks = t.h_b0.back();
  const size_t bytes = sizeof(GridDesc) + 2 * sizeof(int64_t);
  if (sb.cap < bytes) {
    if (sb.dev) HIP_TRY(hipFree(sb.dev));
    HIP_TRY(hipMalloc((void**)&sb.dev, 256));
    sb.cap = 256;
  }
  if (sb.pcap < (size_t)nblocks * 2 + 2) {
    if (sb.part) HIP_TRY(hipFree(sb.part));
    sb.pcap = (size_t)nblocks * 2 + 2;
    HIP_TRY(hipMalloc((void**)&sb.part, sb.pcap * sizeof(double)));
  }
  char host[256];
  std::memcpy(host, &g, sizeof(GridDesc));
  std::memcpy(host + sizeof(GridDesc), t.h_b0.data(), 2 * sizeof(int64_t));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(sb.dev, host, bytes, hipMemcpyHostToDevice));
  Geom geo;
  geo.grids = (const GridDesc*)sb.dev;
  geo.block0 = (const int64_t*)(sb.dev + sizeof(GridDesc));
  geo.ngrids = 1;
  geo.nblocks = nblocks;
  geo.zlen = t.zlen;
  geo.vec = (g.px % 2) == 0;
  *part = sb.part;
  return geo;
}

gd_status gd_rb_sweep(const void* xin, void* xout, const void* b, gd_dtype s, int64_t nx, int64_t ny, int64_t nz,
                      double alpha, double wx, double wy, double wz, void* stream) {
  if (!xin || !xout || !b) return fail(GD_ERR_INVALID, "gd_rb_sweep: null pointer");
  if (xin == xout || xout == b) return fail(GD_ERR_INVALID, "gd_rb_sweep: output aliases input");
  if (!valid_dtype(s)) return fail(GD_ERR_INVALID, "gd_rb_sweep: bad dtype");
  GridDesc g;
  // a single slice (nz == 1) runs in the one-line form: its rows become z
  const bool slice = nz == 1 && ny > 1;
  gd_status r = slice ? one_grid(g, nx, 1, ny, 1, 1, 1, alpha, wx, 0.0, wy)
                      : one_grid(g, nx, ny, nz, 1, 1, 1, alpha, wx, wy, wz);
  if (r != GD_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    int64_t nb;
    double* part;
    Geom geo = slice ? step_geom(g, SWR_TX, 1, false, sweep_target(true), nb, &part, st)
                     : step_geom(g, SW_TX, SW_TY, false, sweep_target(), nb, &part, st);
    geo.row = slice;
    HIP_TRY(launch_rb_sweep(s, geo, xin, xout, b, nullptr, 0, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_residual_restrict(const void* x, const void* b, void* bc, gd_dtype s, int64_t nx, int64_t ny, int64_t nz,
                               int cx, int cy, int cz, double alpha, double wx, double wy, double wz, double* norm2,
                               void* stream) {
  if (!x || !b || !bc) return fail(GD_ERR_INVALID, "gd_residual_restrict: null pointer");
  if (bc == x || bc == b) return fail(GD_ERR_INVALID, "gd_residual_restrict: output aliases input");
  if (!valid_dtype(s)) return fail(GD_ERR_INVALID, "gd_residual_restrict: bad dtype");
  GridDesc g;
  const bool slice = nz == 1 && ny > 1;  // one-line form, rows as z
  gd_status r = slice ? one_grid(g, nx, 1, ny, cx, 1, cy, alpha, wx, 0.0, wy)
                      : one_grid(g, nx, ny, nz, cx, cy, cz, alpha, wx, wy, wz);
  if (r != GD_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    int64_t nb;
    double* part;
    Geom geo = slice ? step_geom(g, SWR_TX, 1, false, 4096, nb, &part, st, true)
                     : step_geom(g, SW_TX, SW_TY, false, 2048, nb, &part, st, true);
    geo.row = slice;
    HIP_TRY(launch_restrict_z(s, geo, x, b, bc, nullptr, part, st));
    if (norm2) {
      std::vector<double> h(nb);
      HIP_TRY(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      double t = 0.0;
      for (double v : h) t += v;
      *norm2 = t;
    }
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_prolong_add(const void* ec, void* x, gd_dtype s, int64_t nx, int64_t ny, int64_t nz, int cx, int cy,
                         int cz, int prolong, void* stream) {
  if (!ec || !x) return fail(GD_ERR_INVALID, "gd_prolong_add: null pointer");
  if (ec == x) return fail(GD_ERR_INVALID, "gd_prolong_add: output aliases input");
  if (!valid_dtype(s)) return fail(GD_ERR_INVALID, "gd_prolong_add: bad dtype");
  if (prolong != 0 && prolong != 1) return fail(GD_ERR_INVALID, "gd_prolong_add: prolong must be 0 or 1");
  GridDesc g;
  gd_status r = one_grid(g, nx, ny, nz, cx, cy, cz, 0.0, 0.0, 0.0, 0.0);
  if (r != GD_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  return run_guarded([&]() -> gd_status {
    int64_t nb;
    double* part;
    Geom geo = step_geom(g, EW_TX, EW_TY, false, 8192, nb, &part, st);
    HIP_TRY(launch_prolong_add(s, geo, ec, x, prolong, st));
    HIP_TRY(hipStreamSynchronize(st));
    return GD_OK;
  });
}

gd_status gd_get_kernel_time(int variant, double* total_ms, int64_t* launches, double* bytes) {
  if (variant < 0 || variant >= kTimerKinds) return fail(GD_ERR_INVALID, "gd_get_kernel_time: variant must be 0..5");
  std::lock_guard<std::mutex> lk(g_timer.mu);
  if (total_ms) *total_ms = g_timer.total_ms[variant];
  if (launches) *launches = g_timer.launches[variant];
  if (bytes) *bytes = g_timer.launches[variant] ? g_timer.bytes[variant] / (double)g_timer.launches[variant] : 0.0;
  return GD_OK;
}

void gd_reset_kernel_time(void) {
  std::lock_guard<std::mutex> lk(g_timer.mu);
  for (int k = 0; k < kTimerKinds; ++k) {
    g_timer.total_ms[k] = 0.0;
    g_timer.launches[k] = 0;
    g_timer.bytes[k] = 0.0;
  }
}

gd_status gd_sweep_config(int64_t nx, int64_t ny, int64_t nz, gd_dtype s, int* tile_tx, int* tile_ty,
                          int64_t* blocks_target, int* tuned, double* ms) {
  int tile = sweep_tile();
  int64_t target = sweep_target(false);
  int t = 0;
  double m = 0.0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(nx, ny, nz, (int)s));
    if (it != g_tune.end()) {
      tile = it->second.tile;
      target = it->second.target;
      t = 1;
      m = it->second.ms;
    }
  }
  if (tile_tx) *tile_tx = SWEEP_TILE_TX[tile];
  if (tile_ty) *tile_ty = SWEEP_TILE_TY[tile];
  if (blocks_target) *blocks_target = target;
  if (tuned) *tuned = t;
  if (ms) *ms = m;
  return GD_OK;
}

gd_status gd_release_workspace(void) {
  return run_guarded([&]() -> gd_status {
    dct_release();
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      evict_idle(0);  // hierarchies in use by a running solve stay
    }
    std::lock_guard<std::mutex> lk(g_step_mu);
    for (auto& kv : g_step) {
      if (kv.second.dev) HIP_TRY(hipFree(kv.second.dev));
      if (kv.second.part) HIP_TRY(hipFree(kv.second.part));
    }
    g_step.clear();
    return GD_OK;
  });
}

}  // extern "C"

