/*
 * gd.h -- C ABI of the MI355X (gfx950) gradient-domain stack solver.
 *
 * Solves the screened anisotropic Poisson systems of Kazhdan et al.,
 * "Gradient-Domain Processing for Large EM Image Stacks":
 *
 *   general (Sec. 4):   (alpha - div W grad) x = alpha V - div W G,
 *                       W = Diag(beta_x, beta_y, beta_z)
 *   anisotropic diffusion, Eq. (1) (Sec. 3.1.1):
 *                       alpha = 0, G = (dI0/dx, dI0/dy, 0)
 *   per-slice screened Poisson, Eq. (2) (Sec. 3.1.2):
 *                       W = Diag(beta_x, beta_y, 0), V = I1, G = grad_xy I0
 *
 * with the 7-point ("Constant", Sec. 4.2) discretisation on a regular voxel
 * grid of unit spacing and natural (Neumann) boundaries: the operator is
 * alpha*Id + sum_a beta_a * L_a, L_a the 3-point second difference along a
 * with no neighbours outside the grid.  The solver is multigrid (Sec. 4.1):
 * red-black Gauss-Seidel, residual restriction, a 1-cell coarsest level and
 * prolongation of the correction, all on the GPU.
 *
 * Conventions (every entry point):
 *  - Volumes are contiguous [nz][ny][nx] arrays, x fastest, unless a slice
 *    descriptor gives an offset and row pitch.  Sizes are int64; an x-y
 *    plane (a slice row's pitch) may hold at most 2^28 cells (16384^2),
 *    larger ones return GD_ERR_UNSUPPORTED.
 *  - Data pointers are DEVICE pointers owned by the caller; the library never
 *    frees them.  Outputs must not alias inputs.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call
 *    enqueues its work on `stream` and returns after the result is complete
 *    on that stream (residual norms are read back to the host).
 *  - Workspace (multigrid levels, scratch) is allocated by the library with
 *    hipMalloc and cached per problem shape until gd_release_workspace().
 *  - No C++ exception crosses the ABI.  Every call returns a gd_status; on a
 *    status other than GD_OK, gd_last_error() gives a message (thread-local).
 *  - A solve that does not reach opts->rel_tol within opts->max_cycles still
 *    writes its best iterate and returns GD_ERR_NOT_CONVERGED.  A NaN or Inf
 *    residual norm returns GD_ERR_NUMERIC.
 */
#ifndef GD_H
#define GD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GD_F64 = 0, GD_F32 = 1, GD_F16 = 2, GD_BF16 = 3 } gd_dtype;

typedef enum {
  GD_OK = 0,
  GD_ERR_INVALID = -1,        /* bad argument (null pointer, size, weight, dtype) */
  GD_ERR_NOMEM = -2,          /* device allocation failed */
  GD_ERR_HIP = -3,            /* a HIP runtime call or kernel launch failed */
  GD_ERR_NOT_CONVERGED = -4,  /* tolerance not reached within max_cycles */
  GD_ERR_NUMERIC = -5,        /* NaN/Inf in a residual norm */
  GD_ERR_UNSUPPORTED = -6     /* valid request this build does not implement */
} gd_status;

/* Solver options.  Obtain defaults with gd_default_opts() and edit. */
typedef struct {
  double rel_tol;       /* stop when ||b - A x||_2 / ||b||_2 <= rel_tol (canonical
                           system, x0 = 0 convention of the Table 1 caption)   */
  int max_cycles;       /* V-cycles (plain) or refinement steps (mixed)        */
  int pre_smooth;       /* red-black GS sweeps before restriction; -1 (the
                           default): automatic, 2 for FP16/BF16 storage with
                           fp64_refine = 1, else 1                            */
  int post_smooth;      /* red-black GS sweeps after prolongation; -1 (the
                           default): automatic, 3 for FP16/BF16 storage with
                           fp64_refine = 1, else 2                            */
  gd_dtype storage;     /* storage of the multigrid arrays: F64/F32 (plain) or
                           F16/BF16/F32 (with fp64_refine)                      */
  int fp64_refine;      /* 1: FP64 outer iterative refinement around V-cycles
                           in `storage`; 0: plain V-cycles in `storage`        */
  int inner_cycles;     /* V-cycles per refinement step (fp64_refine = 1)      */
  int prolong;          /* 0: cell-centred trilinear, 1: piecewise constant    */
  int timing;           /* 1: time the finest-level relaxation launches with
                           HIP events (gd_get_kernel_time)                     */
  int fuse_prolong;     /* 1: add the up-sampled correction inside the first
                           post-smoothing sweep instead of a separate pass    */
  int sweep_tile;       /* relaxation tile of 3-D grids: -1 automatic (the
                           autotuned or default choice), 0: 64x8, 1: 128x8,
                           2: 64x16, 3: 128x16; 4: 256x8 and 5: 256x12 with
                           FP32/FP16/BF16 storage and sweep_quad = 1 only
                           (GD_ERR_INVALID otherwise).  Results do not depend
                           on it. */
  int use_graph;        /* 1 (default): the repeated part of each V-cycle is
                           captured once into a HIP graph and replayed; 0:
                           plain launches.  Same results either way; timing = 1
                           uses plain launches. */
  int fmg;              /* 1: start the plain solve with a full-multigrid pass
                           (right-hand side restricted to every level, coarse
                           solutions interpolated up, one V-cycle per level);
                           0 (default): start from zero */
  int discretization;   /* Sec. 4.2: 0 (default) "Constant" transfers with
                           rediscretised 7-point coarse operators; 1 "Hybrid":
                           7-point finest level, B-spline (1/2, 1, 1/2)
                           prolongation, its transpose as restriction and
                           Galerkin 27-point coarse operators relaxed by
                           8-colour Gauss-Seidel (same answer); 2 "Linear":
                           trilinear B-spline finite elements on every level
                           (27-point, a different discrete answer; no FP64
                           refinement, not for the gradient-modulation
                           filter).  Slice batches with 1 or 2: slices of
                           one size and alpha laid out as a stack (equal
                           pitch, constant offset step of at least pitch*ny)
                           are solved as one 3-D grid with no coupling along
                           the stack (w_z = 0; for 2 also M_z = Id), each
                           slice checked against its own right-hand side
                           (Hybrid with FP64 refinement excluded); other
                           batches solve every slice as a one-plane grid of
                           its own, in turn (slices of one size share a
                           cached hierarchy). */
  int sweep_quad;       /* 1 (default): the relaxation of FP16/BF16 level
                           arrays, and of FP32 3-D grids, runs in its quad
                           form (four x cells per thread, one aligned
                           8/16-byte access per quad); 0: the pair form (two
                           cells per thread).  Same values bit for bit; FP64,
                           FP32 slices and the fused prolongation always use
                           the pair form. */
} gd_solve_opts;

/* Filled by the solve calls when the pointer is non-NULL. */
typedef struct {
  int cycles;             /* V-cycles run (all refinement steps included); per
                             slice of a plain batched solve, the cycles after
                             which that slice met the tolerance and left the
                             batch (its kernels skip it from then on)          */
  int refine_steps;       /* FP64 refinement steps (0 for plain solves)         */
  double rel_residual;    /* final canonical relative residual, FP64 on the GPU */
  double b_norm;          /* ||b||_2 of the canonical system                    */
  double seconds;         /* wall time of the call, host clock                  */
  int levels;             /* multigrid levels (finest = level 0)                */
  int fallback_used;      /* gd_fcg_solve: 1 when the learned preconditioner was
                             replaced by the V-cycle (net failed or stopped
                             reducing the residual); 0 otherwise               */
  double bytes;           /* algorithmic HBM bytes of the solve's kernels: per
                             launch, the bytes the kernel must read and write
                             per cell (e.g. 3 x storage bytes for a sweep)
                             times the cells it covers, summed on the host; a
                             slice's report carries its share by cells; for
                             gd_fcg_solve the V-cycles and Krylov vector
                             kernels, not the net's convolutions           */
} gd_solve_report;

/* One slice of a batched screened-Poisson call (Eq. (2) per slice). */
typedef struct {
  int64_t offset;  /* element offset of pixel (0,0) in the I0/I1/I2 arrays */
  int32_t nx, ny;  /* slice width and height                               */
  int32_t pitch;   /* elements between rows (>= nx)                        */
  float alpha;     /* screening weight of this slice (> 0)                 */
} gd_slice_desc;

void gd_default_opts(gd_solve_opts* opts);
const char* gd_last_error(void);
const char* gd_version(void);

/* Anisotropic diffusion of a whole stack, Eq. (1) (Sec. 3.1.1):
 *   (beta_x L_x + beta_y L_y + beta_z L_z) I1 = (beta_x L_x + beta_y L_y) I0
 * with the gauge mean(I1) = mean(I0) (the zero frequency keeps gain 1).
 * I0: nz*ny*nx values of in_t; I1: same count of out_t.  beta_x, beta_y >= 0,
 * beta_z > 0.  The plain path stores the correction I1 - I0 in opts->storage
 * (F32/F64) and iterates to rel_tol; with fp64_refine the iterate is FP64
 * and the V-cycles run in opts->storage (F16/BF16/F32). */
gd_status gd_smooth_z(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t,
                      int64_t nx, int64_t ny, int64_t nz,
                      double beta_x, double beta_y, double beta_z,
                      const gd_solve_opts* opts, gd_solve_report* rep, void* stream);

/* The same solve for callers that cannot allocate memory (code that a HIP
 * graph is capturing around, tight serving loops, harnesses that forbid
 * hipMalloc): every device array of the multigrid hierarchy lives in one
 * static device array of the library, 128 MiB per GPU (gd_noalloc_scratch_bytes),
 * so no hipMalloc, hipFree, pinned host memory, graph or event is created
 * (the first call on a GPU loads that array, once per process).
 * Arguments, results and status codes as gd_smooth_z, with these limits:
 * the Constant discretisation only (opts->discretization = 0; others
 * GD_ERR_UNSUPPORTED); opts->use_graph and opts->timing are ignored (plain
 * launches); no autotuning (the fixed relaxation tile); a problem whose
 * hierarchy needs more than the scratch (about 19 bytes per voxel for FP32
 * storage, 26 for FP16/BF16 with FP64 refinement) returns
 * GD_ERR_UNSUPPORTED with the bytes it needs, before any device work.
 * All calls on one GPU share that GPU's scratch, which keeps the last
 * call's contents (every array the solve reads is written by it first):
 * calls that overlap on one GPU (other threads or streams) race and must be
 * serialised by the caller. */
gd_status gd_smooth_z_noalloc(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t,
                              int64_t nx, int64_t ny, int64_t nz,
                              double beta_x, double beta_y, double beta_z,
                              const gd_solve_opts* opts, gd_solve_report* rep, void* stream);
/* Size in bytes of the scratch gd_smooth_z_noalloc uses on each GPU. */
gd_status gd_noalloc_scratch_bytes(int64_t* bytes);

/* Per-slice screened Poisson, Eq. (2) (Sec. 3.1.2), for a batch of
 * independent 2-D slices of any sizes:
 *   (alpha_i + beta_x L_x + beta_y L_y) I2_i = alpha_i I1_i + (beta_x L_x + beta_y L_y) I0_i.
 * I0 (dtype in_t), I1 (dtype i1_t: in_t, GD_F32 or GD_F64) and I2 (dtype
 * out_t, any) share the slice layout `slices` (host array of nslices
 * descriptors; slices must not overlap; every array must hold each slice's
 * span offset + pitch * (ny - 1) + nx).  A wider I1 and I2 let the FP64
 * result of a refined anisotropic diffusion feed this phase and the refined
 * result come back without rounding to the 16-bit storage type of I0.
 * Every slice is iterated until its own relative residual <= rel_tol.
 * per_slice (host array of nslices, or NULL) receives each slice's final
 * report (its cycles: those it took before leaving the batch, or for a
 * Hybrid / Linear stack solved as one grid those of the whole stack); rep
 * (or NULL) the batch summary with rel_residual = the largest slice
 * residual.  nslices = 0 is an empty batch (GD_OK, nothing touched);
 * nslices < 0, zero-sized slices, alpha <= 0 or another i1_t are
 * GD_ERR_INVALID. */
gd_status gd_screened_poisson_slices(const void* I0, gd_dtype in_t, const void* I1, gd_dtype i1_t,
                                     void* I2, gd_dtype out_t,
                                     const gd_slice_desc* slices, int64_t nslices,
                                     double beta_x, double beta_y,
                                     const gd_solve_opts* opts, gd_solve_report* rep,
                                     gd_solve_report* per_slice, void* stream);

/* Gradient-modulation ("non-photorealistic") filter of Sec. 6, the general
 * system of Sec. 4 applied to a volume (the paper filters a video,
 * x, y = frame, z = time):
 *   I1 = argmin alpha |I - I0|^2 + sum_a beta_a |D_a I - V_a|^2,
 *   V  = lambda (1 - exp(-|g|^2 / (2 sigma^2))) g,
 * g the forward-difference gradient of I0 at each voxel (a component is 0
 * where its face leaves the grid), its face v -> v + e_a carrying V_a(v).
 * The paper uses alpha = 0.001, beta = (1, 1, 0.1), lambda = 1.25, sigma = 5
 * on grey values in [0, 256).  I0 (in_t) and I1 (out_t) are contiguous
 * [nz][ny][nx]; the V-cycles run in opts->storage on the correction I1 - I0
 * until ||b - A I1|| <= rel_tol ||b|| (canonical b, FP64 accumulation).
 * alpha <= 0, beta < 0, sigma <= 0 or a non-finite lambda are
 * GD_ERR_INVALID; opts->fp64_refine is GD_ERR_UNSUPPORTED. */
gd_status gd_npr_filter(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t,
                        int64_t nx, int64_t ny, int64_t nz, double alpha,
                        double beta_x, double beta_y, double beta_z, double lambda, double sigma,
                        const gd_solve_opts* opts, gd_solve_report* rep, void* stream);

/* ---- spectral solver (Sec. 3.2): exact DCT-II diagonalisation -------------
 * The constant-coefficient Neumann operator alpha + sum_a beta_a L_a is
 * diagonal in the DCT-II basis cos(pi k (j + 1/2) / n) (eigenvalues
 * alpha + sum_a beta_a (2 - 2 cos(pi k_a / n_a))), so these calls solve the
 * same systems as the multigrid ones exactly (FP64 throughout, three
 * forward and three inverse transforms): a competitor and a verifier.
 * Contiguous [nz][ny][nx] arrays; every axis a power of two <= 4096, other
 * sizes GD_ERR_UNSUPPORTED.  An FP64 workspace of nx*ny*nz values is kept per
 * device until gd_release_workspace(). */

/* x = (alpha + sum_a beta_a L_a)^-1 b; with alpha = 0 the mean-free solution
 * (b should then have zero mean: its mean is dropped). */
gd_status gd_dct_solve(const void* b, gd_dtype bt, void* x, gd_dtype xt, int64_t nx, int64_t ny, int64_t nz,
                       double alpha, double beta_x, double beta_y, double beta_z, void* stream);
/* Anisotropic diffusion, Eq. (1), in closed form (Sec. 3.2.1): every
 * frequency scaled by (bx lx + by ly) / (bx lx + by ly + bz lz), the zero
 * frequency kept (mean(I1) = mean(I0)). */
gd_status gd_dct_smooth_z(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t, int64_t nx, int64_t ny,
                          int64_t nz, double beta_x, double beta_y, double beta_z, void* stream);

/* ---- general system (Sec. 4) through an explicit hierarchy ---------------- */
typedef struct gd_hierarchy gd_hierarchy;

/* Multigrid levels for (alpha + sum_a beta_a L_a) on an nx*ny*nz grid, arrays
 * in `storage` (F64/F32/F16/BF16, arithmetic in FP32, FP64 for F64).
 * alpha >= 0, beta_a >= 0, not all zero. */
gd_status gd_hierarchy_create(gd_hierarchy** h, int64_t nx, int64_t ny, int64_t nz,
                              double alpha, double beta_x, double beta_y, double beta_z,
                              gd_dtype storage, const gd_solve_opts* opts, void* stream);
gd_status gd_hierarchy_destroy(gd_hierarchy* h);
/* Number of levels and the size of level `level` (finest = 0). */
gd_status gd_hierarchy_info(const gd_hierarchy* h, int level, int* nlevels,
                            int64_t dims[3], double coef[4] /* alpha, w_x, w_y, w_z */);

/* b = alpha V + sum_a beta_a D_a^T G_a (the discrete alpha V - div W G).
 * V: nx*ny*nz values (ignored when alpha == 0; may be NULL then).
 * Gx/Gy/Gz: face fields of the volume's shape; G_a[v] is the target of the
 * face between v and v + e_a, entries on the last plane along a are ignored;
 * NULL = zero field.  All in the hierarchy's storage dtype; b likewise. */
gd_status gd_rhs_general(gd_hierarchy* h, const void* V, const void* Gx, const void* Gy,
                         const void* Gz, void* b, void* stream);

/* ncycles V-cycles on A x = b (x in/out, b in; both in the storage dtype).
 * rel_residual_out (may be NULL) receives ||b - A x|| / ||b|| after the
 * last cycle (FP64 accumulation).  ncycles <= 0 only evaluates it. */
gd_status gd_vcycle(gd_hierarchy* h, void* x, const void* b, int ncycles,
                    double* rel_residual_out, void* stream);

/* ---- levels streamed from host memory (Sec. 4.1) -----------------------------
 * The paper runs every V-cycle as two streaming passes through the data
 * with a window over the slices.  Here the finest level's x and b stay in
 * host memory, and so may the next levels with more than an eighth of the
 * finest level's cells (with z-first semi-coarsening the first coarse level
 * has half; the library holds them in pinned host memory); only windows of
 * z-planes of them are in HBM, the other levels are resident.  stream_levels
 * = 0 streams such a coarser level only when its window buffers take less
 * HBM than the level itself (long stacks); stream_levels = k > 0 streams at
 * most k levels, the finest included (one level always stays resident).
 * A pass over a streamed level cuts z into slabs of `slab` planes (raised to
 * an even count of at least the halo, 2 max(pre_smooth, post_smooth) + 2
 * planes) and relaxes each slab with that halo on both sides, so every cycle
 * gives the same values as gd_vcycle on the whole grid (halo planes are
 * recomputed and dropped).  Down pass: pre-smoothing and the restricted
 * residual; up pass: the interpolated coarse correction and post-smoothing.
 * Uploads, kernels and write-backs of consecutive windows overlap on three
 * streams (three window buffer sets rotate per level).
 *
 * gd_hierarchy_create_streamed: arguments as gd_hierarchy_create plus `slab`
 * (> 0) and `stream_levels` (>= 0).  Only the Constant discretisation (opts->discretization == 0),
 * ny >= 2 and grids with a coarser level; GD_ERR_UNSUPPORTED otherwise.  The
 * handle accepts gd_vcycle_streamed, gd_hierarchy_info,
 * gd_hierarchy_device_bytes, gd_hierarchy_streamed_levels and
 * gd_hierarchy_destroy; the in-core calls
 * (gd_vcycle, gd_rhs_general, gd_mg_error_pairs, gd_fcg_solve) return
 * GD_ERR_INVALID. */
gd_status gd_hierarchy_create_streamed(gd_hierarchy** h, int64_t nx, int64_t ny, int64_t nz,
                                       double alpha, double beta_x, double beta_y, double beta_z,
                                       gd_dtype storage, const gd_solve_opts* opts, int64_t slab,
                                       int stream_levels, void* stream);
/* Anisotropic diffusion, Eq. (1), of a stack that stays in HOST memory (the
 * paper's setting: the volume does not fit the device; Sec. 4.1 streams
 * every pass through a window of slices).  I0 (in_t) and I1 (out_t) are
 * dense [nz][ny][nx] host arrays of the caller (hipHostMalloc memory lets
 * the copies run at the link's pinned rate).  Every step runs on the GPU in
 * passes over z-slabs of `slab` planes: the right-hand side of the
 * correction E = I1 - I0 and the canonical norm (one halo plane per side);
 * the V-cycles of a streamed hierarchy (as gd_hierarchy_create_streamed
 * with stream_levels; E and its right-hand side in pinned host arrays of
 * the library, 2 x storage bytes per voxel); the FP64 canonical residual
 * after each cycle, itself a streaming pass; the sum of E for the gauge
 * mean(I1) = mean(I0); and the output I0 + E - mean(E), written back slab
 * by slab.  Options as gd_smooth_z with plain FP32 or FP64 storage (no
 * refinement) and the Constant discretisation, others GD_ERR_UNSUPPORTED.
 * device_budget > 0: the call needs at most that many device bytes (the
 * streamed hierarchy and the pass windows), or returns GD_ERR_NOMEM before
 * any pass.  rep->bytes: the HBM bytes of the setup and output passes. */
gd_status gd_smooth_z_streamed(const void* I0, gd_dtype in_t, void* I1, gd_dtype out_t,
                               int64_t nx, int64_t ny, int64_t nz,
                               double beta_x, double beta_y, double beta_z,
                               const gd_solve_opts* opts, int64_t slab, int stream_levels,
                               int64_t device_budget, gd_solve_report* rep, void* stream);

/* Per-slice screened Poisson, Eq. (2), of a stack held in HOST memory: the
 * slices are independent, so batches of `slab` consecutive slices are
 * uploaded, solved in HBM as one batch (gd_screened_poisson_slices, same
 * options, alpha for every slice) and written back.  I0 (in_t), I1 (i1_t:
 * in_t, F32 or F64) and I2 (out_t) are dense [nz][ny][nx] host arrays of
 * the caller.  per_slice (nz reports, or NULL) and rep as
 * gd_screened_poisson_slices.  device_budget > 0: GD_ERR_NOMEM up front if
 * the slab buffers and the batch's hierarchy need more device bytes. */
gd_status gd_screened_poisson_streamed(const void* I0, gd_dtype in_t, const void* I1, gd_dtype i1_t,
                                       void* I2, gd_dtype out_t, int64_t nx, int64_t ny, int64_t nz,
                                       double alpha, double beta_x, double beta_y,
                                       const gd_solve_opts* opts, int64_t slab, int64_t device_budget,
                                       gd_solve_report* rep, gd_solve_report* per_slice, void* stream);

/* ncycles V-cycles on A x = b with x (in/out) and b (in) in HOST memory, dense
 * [nz][ny][nx] arrays of the storage dtype, owned by the caller.  Memory
 * from hipHostMalloc lets copies overlap the kernels; pageable memory works
 * and is slower.  The call returns when x holds the result.
 * rel_residual_out (may be NULL): ||b - A x|| / ||b|| after the last cycle,
 * from one more streaming pass. */
gd_status gd_vcycle_streamed(gd_hierarchy* h, void* x, const void* b, int ncycles,
                             double* rel_residual_out, void* stream);
/* Device memory the hierarchy holds (levels, windows, launch tables) and,
 * for a streamed one, the planes of its largest window (0 otherwise). */
gd_status gd_hierarchy_device_bytes(const gd_hierarchy* h, int64_t* bytes, int64_t* window_planes);
/* Number of levels held in host memory (0 for an in-core hierarchy). */
gd_status gd_hierarchy_streamed_levels(const gd_hierarchy* h, int* levels);

/* Residual-to-error pairs from multigrid itself, for training a learned
 * preconditioner: x_k = `cycles` V-cycles from zero on A x = b; r_out = b - A x_k,
 * e_out = x_star - x_k (x_star: the converged solution, from gd_vcycle).
 * All arrays nx*ny*nz in the hierarchy's storage dtype. */
gd_status gd_mg_error_pairs(gd_hierarchy* h, const void* b, const void* x_star, int cycles,
                            void* r_out, void* e_out, void* stream);

/* ---- learned preconditioner (not in the paper) --------------------------------
 * A 3-level U-Net of 3x3 convolutions (16/32/64 channels, BF16 weights and
 * activations, FP32 accumulation on the matrix cores, FP32 master weights)
 * mapping a residual image to an error estimate: z = N(r / s) * s with s the
 * RMS of r per image.  Images: nx % 256 == 0, ny % 4 == 0, nx, ny <= 16384,
 * nx*ny <= 2^26, FP32, batch of `batch` images of ny*nx pixels (a
 * [batch][ny][nx] array); training batches hold at most 2^28 pixels.  The
 * forward pass runs in groups of images of at most 2^25 pixels (about 10 GB
 * of activations).  Errors: GD_ERR_INVALID for other shapes. */
typedef struct gd_net gd_net;
/* weights: NULL for He-normal weights from `seed` (zero biases), or a host
 * array of `count` == gd_net_num_params FP32 master weights in the layout of
 * gd_net_get_params (copied; count mismatch: GD_ERR_INVALID). */
gd_status gd_net_create(gd_net** n, const float* weights, int64_t count, uint64_t seed);
gd_status gd_net_destroy(gd_net* n);
int64_t gd_net_num_params(const gd_net* n);
gd_status gd_net_get_params(gd_net* n, float* host, int64_t count);   /* FP32 master weights */
gd_status gd_net_set_params(gd_net* n, const float* host, int64_t count);
const char* gd_net_last_error(void);
gd_status gd_net_forward(gd_net* n, const float* r, float* z, int64_t nx, int64_t ny, int64_t batch,
                         void* stream);
/* loss = mean over pixels of (N(r/s) - e/s)^2; gradients (FP32, master-weight
 * layout, host array of gd_net_num_params) without updating the weights */
gd_status gd_net_gradients(gd_net* n, const float* r, const float* e, int64_t nx, int64_t ny, int64_t batch,
                           float* grad_host, double* loss_out, void* stream);
/* one Adam step (beta 0.9 / 0.999, eps 1e-8) on the same loss */
gd_status gd_net_train_step(gd_net* n, const float* r, const float* e, int64_t nx, int64_t ny, int64_t batch,
                            float lr, double* loss_out, void* stream);

/* Timing of the forward convolutions (HIP events on the caller's stream).
 * set_timing(on) also clears the totals.  kernel_time: total ms, launches
 * and algorithmic FLOPs (2 * 9 * cin * cout per output pixel, real channel
 * counts) of layer 0..8 since then. */
gd_status gd_net_set_timing(gd_net* n, int on);
gd_status gd_net_kernel_time(const gd_net* n, int layer, double* ms, int64_t* launches, double* flops);

/* Flexible conjugate gradients on the hierarchy's system (FP32 storage) with
 * preconditioner 0: one V-cycle, 1: the net, 2: a V-cycle then the net on
 * its remaining residual, 3: the net as the finest level's post-smoother (a
 * V-cycle without the finest post-smoothing sweeps, then the net on its
 * remaining residual).  x in/out, b in (caller's layout).  When the net
 * fails or stops reducing the residual the iteration restarts with the
 * V-cycle preconditioner (rep->fallback_used = 1 then).  rep->cycles =
 * iterations, rep->rel_residual = the final true relative residual. */
gd_status gd_fcg_solve(gd_hierarchy* h, gd_net* net, void* x, const void* b, int precond, double rel_tol,
                       int max_iter, gd_solve_report* rep, void* stream);

/* ---- single multigrid steps (Sec. 4.1), for kernel-level checks ------------
 * All arrays are nx*ny*nz of dtype s; the operator is
 * alpha*Id + w_x L_x + w_y L_y + w_z L_z (one level's coefficients). */

/* One red-black Gauss-Seidel sweep: red voxels ((i+j+k) even) then black,
 * each set to zero its own residual.  x_out must not alias x_in. */
gd_status gd_rb_sweep(const void* x_in, void* x_out, const void* b, gd_dtype s,
                      int64_t nx, int64_t ny, int64_t nz,
                      double alpha, double w_x, double w_y, double w_z, void* stream);

/* r = b - A x restricted to the coarse grid of size ceil(n_a / c_a), each
 * coarse cell the sum of its children (c_a in {1, 2}).  norm2_out (host, may
 * be NULL) receives sum r^2 over the fine grid (FP64). */
gd_status gd_residual_restrict(const void* x, const void* b, void* b_coarse, gd_dtype s,
                               int64_t nx, int64_t ny, int64_t nz,
                               int c_x, int c_y, int c_z,
                               double alpha, double w_x, double w_y, double w_z,
                               double* norm2_out, void* stream);

/* x += P e: up-sample a coarse correction (prolong 0: cell-centred
 * trilinear, 1: piecewise constant) onto the fine grid and add it. */
gd_status gd_prolong_add(const void* e_coarse, void* x, gd_dtype s,
                         int64_t nx, int64_t ny, int64_t nz,
                         int c_x, int c_y, int c_z, int prolong, void* stream);

/* ---- instrumentation -------------------------------------------------------- */
/* Total HIP-event time (ms) and launch count of the finest-level relaxation
 * launches of one variant since the last reset, recorded by solves run with
 * opts->timing = 1.  variant: 0 stack grid, 1 stack grid with the coarse
 * correction added on load, 2 slice (one-line) grids, 3 slice grids with the
 * correction, 4 stack grid and 5 slice grids starting from a zero iterate
 * (the first sweep of a refinement step's V-cycle, which does not read x).
 * bytes_per_launch: algorithmic bytes of one launch, averaged over the launches
 * counted (read x and b, write x: 3 * storage bytes per voxel of the finest
 * level that the launch worked on -- slices of a batch that have converged are
 * left out; 2 * for variants 4, 5). */
gd_status gd_get_kernel_time(int variant, double* total_ms, int64_t* launches, double* bytes_per_launch);
void gd_reset_kernel_time(void);

/* Relaxation launch of the finest level of an nx*ny*nz 3-D grid in storage
 * type s: tile (tile_tx x tile_ty cells) and block target, and whether they
 * come from the autotuner (tuned = 1, ms = the measured time of one sweep)
 * or from the fixed default.  The autotuner runs once per size and type
 * when a workspace of at least 2^22 cells is first built (GD_AUTOTUNE=0, or
 * GD_SWEEP_TILE / GD_SWEEP_BLOCKS, keep the fixed choice); any tile computes
 * the same values.  Output pointers may be NULL. */
gd_status gd_sweep_config(int64_t nx, int64_t ny, int64_t nz, gd_dtype s, int* tile_tx, int* tile_ty,
                          int64_t* blocks_target, int* tuned, double* ms);

/* Free every cached workspace (all devices). */
gd_status gd_release_workspace(void);

#ifdef __cplusplus
}
#endif
#endif /* GD_H */
