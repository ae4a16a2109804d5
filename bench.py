"""Benchmark: voxels/s of the full gradient-domain pass (anisotropic diffusion
of the stack, Eq. (1), then the per-slice screened Poisson, Eq. (2)), each
solved to 1e-6 canonical relative residual on one MI355X.

One step = AD + SP of the whole stack, inputs already resident in HBM.
Prints one JSON line (rank 0).  The dominant kernel is the finest-level
red-black relaxation; its HIP-event time inside the timed steps gives the
achieved algorithmic HBM bandwidth (read x and b, write x per voxel).
The CPU baseline is the FP64 oracle (conjugate gradients on the same
systems) timed on the host on a crop of the same stack.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

WORKLOADS = {
    # name: (spec key, storage, fp64_refine, description)
    "stack4k": ("stack4k", "f16", 1, "4096x4096x256 stack, FP16 storage of the input and the V-cycles, FP32 "
                "relaxation, FP64 refinement (headline); legs: BF16 + FP64 refinement, FP32 plain V-cycles"),
    "stack1k": ("stack1k", "f32", 0, "1024x1024x128 stack, FP32 storage + arithmetic, plain V-cycles"),
    "stack4k-f16": ("stack4k", "f16", 1, "4096x4096x256 stack, FP16 storage, FP32 relaxation, FP64 refinement"),
    "stack4k-bf16": ("stack4k", "bf16", 1, "4096x4096x256 stack, BF16 storage, FP32 relaxation, FP64 refinement"),
    "stack4k-f32": ("stack4k", "f32", 0, "4096x4096x256 stack, FP32 storage + arithmetic, plain V-cycles"),
    "learned2k": ("learned", "f32", 0, "2048x2048x64 stack, per-slice screened Poisson (alpha 0.01), flexible CG "
                  "preconditioned by a V-cycle then the BF16 U-Net, net trained on multigrid error pairs of "
                  "1024x1024 slices"),
    "ad1k-dct": ("dct", "f32", 0, "1024x1024x128 stack (the stack1k input), anisotropic diffusion only, spectral "
                 "solver (FP64 DCT-II diagonalisation, exact) beside the FP32 multigrid AD to 1e-6"),
    "npr-video": ("npr", "f32", 0, "1920x1080x742 grey-level video volume, gradient-modulation filter of Sec. 6 "
                  "(alpha 0.001, W = diag(1, 1, 0.1), lambda 1.25, sigma 5), FP32 storage, plain V-cycles"),
    "stack1k-streamed": ("streamed:stack1k", "f32", 0, "1024x1024x128 stack, anisotropic-diffusion V-cycles (FP32) "
                         "with the finest level's x and b in pinned host memory, streamed through HBM in halo-padded "
                         "z-slabs (Sec. 4.1), coarse levels resident; the in-core V-cycles of the same system beside it"),
    "stack4k-streamed": ("streamed:stack4k", "f32", 0, "4096x4096x256 stack, as stack1k-streamed"),
    "slices2048": ("slices", "f32", 0, "2048 independent slices, sides log-uniform in [256, 2048], alpha U(0.001, 0.1), "
                   "per-slice screened Poisson, FP32, plain V-cycles, one batched launch per level step"),
}
BETA = (1.0, 1.0, 4.0)
ALPHA = 0.01
TOL = 1e-6
HBM_PEAK_GBS = 8000.0


def smooth_split(a, storage="f32", refine=0):
    """(pre, post) sweeps per V-cycle: --smooth, or with "auto" what the
    library picks for the storage path (V(2,3) for 16-bit storage with FP64
    refinement, V(1,2) otherwise)."""
    if a.smooth != "auto":
        pre, post = (int(v) for v in a.smooth.split(","))
        return pre, post
    return (2, 3) if refine and storage in ("f16", "bf16") else (1, 2)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="stack4k", choices=sorted(WORKLOADS))
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-crop", default="32,512,512", help="nz,ny,nx of the oracle's crop")
    p.add_argument("--smooth", default="auto",
                   help="pre,post red-black sweeps per V-cycle; auto: the library's choice per storage path "
                        "(V(2,3) for 16-bit storage with FP64 refinement, V(1,2) otherwise)")
    p.add_argument("--fmg", type=int, default=None, help="1: full-multigrid start of the plain solves")
    p.add_argument("--discretization", default="constant", choices=["constant", "hybrid", "linear"],
                   help="discretisation of both solves (Sec. 4.2); Hybrid and Linear solve the SP slices one "
                        "by one")
    p.add_argument("--prolong", default="trilinear", choices=["trilinear", "constant"],
                   help="up-sampling of the Constant scheme: cell-centred trilinear or replication")
    p.add_argument("--inner-cycles", type=int, default=None,
                   help="V-cycles per FP64 refinement step (mixed storage; library default if omitted)")
    p.add_argument("--slab", type=int, default=32, help="z-planes per slab of the streamed workloads")
    p.add_argument("--stream-levels", type=int, default=0,
                   help="levels held in host memory by the streamed workloads (0: the library's choice by HBM use)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only copy a 1 GiB buffer 3 times (reference for HBM byte counters)")
    p.add_argument("--traffic-json", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                          "profiles", "traffic.json"))
    return p.parse_args()


def cpu_baseline(I0_host, crop, min_s=10.0):
    """The FP64 oracle on a crop of the same stack, solved as its own problem:
    AD then SP by the oracle's exact DCT-II solves (scipy.fft with one worker
    per host core), repeated for at least `min_s` seconds."""
    import scipy.fft as sfft

    from oracle import solvers

    nz, ny, nx = crop
    sub = np.ascontiguousarray(I0_host[:nz, :ny, :nx], dtype=np.float64)
    ncpu = os.cpu_count() or 1
    reps = 0
    t0 = time.perf_counter()
    with sfft.set_workers(ncpu):
        while reps == 0 or time.perf_counter() - t0 < min_s:
            I1 = solvers.ad_dct(sub, BETA)
            solvers.sp_dct(sub, I1, ALPHA)
            reps += 1
    dt = (time.perf_counter() - t0) / reps
    return {
        "value": sub.size / dt,
        "unit": "voxels/s",
        "cores": ncpu,
        "kind": "oracle",
        "sample": f"crop [0:{nz},0:{ny},0:{nx}] of the same (quantised) stack ({sub.size} voxels), AD then SP "
                  f"by the oracle's exact DCT-II solves in FP64 (numpy/scipy.fft, workers={ncpu} = os.cpu_count()), "
                  f"{reps} repetitions in {dt * reps:.1f} s",
    }


def bench_slices(a, gd, synth, torch, desc):
    """Batched per-slice screened Poisson of 2048 uneven slices."""
    t0 = time.perf_counter()
    meta = synth.make_slice_batch(device="cuda", dtype=torch.float32)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    I0, I1 = meta["I0"], meta["I1"]
    npx = I0.numel()
    pre, post = smooth_split(a)
    opts = dict(rel_tol=TOL, pre_smooth=pre, post_smooth=post)
    out = torch.empty_like(I0)
    for _ in range(a.warmup):
        gd.screened_poisson_slices(I0, I1, descs, out=out, **opts)
    torch.cuda.synchronize()
    gd.reset_kernel_time()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, rep, per = gd.screened_poisson_slices(I0, I1, descs, out=out, timing=1, **opts)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ms, launches, bytes_per = gd.kernel_time(gd.SWEEP_SLICE)
    avg_ms = ms / max(launches, 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    line = {
        "metric": "pixels/s to 1e-6 rel. residual per slice (batched SP)",
        "value": npx / dt, "unit": "pixels/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}; beta=(1,1), tol {TOL:g} per slice", "slices": len(descs),
                   "pixels": npx, "smooth": [pre, post]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_rb_sweep<f32,256,1,false,true> finest level",
                     "launches": launches, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per},
        "sp": {"cycles": rep["cycles"], "max_slice_rel_residual": rep["rel_residual"], "levels": rep["levels"]},
        "generate_s": gen_s,
    }
    print(json.dumps(line), flush=True)


def bench_learned(a, gd, synth, torch, desc):
    """Learned preconditioner: train on multigrid (residual, error) pairs of
    1024^2 slices (untimed), then solve the per-slice screened Poisson system
    of a 2048^2 x 64 stack by flexible CG with the V-cycle + net
    preconditioner; plain V-cycles and V-cycle-preconditioned FCG on the
    same system are timed beside it."""
    dev = torch.device("cuda:0")

    def sp_rhs(I0, I1):
        # alpha I1 + (D_x^T D_x + D_y^T D_y) I0 per slice (Eq. (2)); input preparation
        b = ALPHA * I1.double()
        for ax in (2, 1):
            d = torch.diff(I0.double(), dim=ax)
            n = I0.shape[ax]
            b.narrow(ax, 0, n - 1).sub_(d)
            b.narrow(ax, 1, n - 1).add_(d)
        return b.float().contiguous()

    def stack(n, nz, seed):
        spec = synth.StackSpec(n, n, nz, (4.0, 40.0), True, seed)
        I0 = synth.make_stack(spec, device=dev, dtype=torch.float32)
        I1, _ = gd.smooth_z(I0, BETA, out_dtype=torch.float32, rel_tol=TOL)
        return sp_rhs(I0, I1)

    t0 = time.perf_counter()
    btr = stack(1024, 16, 13100430)
    h = gd.Hierarchy(tuple(btr.shape), ALPHA, (1.0, 1.0, 0.0), torch.float32)
    xs = torch.zeros_like(btr)
    h.vcycle(xs, btr, 30)
    pairs = [h.error_pairs(btr, xs, k) for k in (1, 2, 3)]
    h.close()
    r = torch.cat([p[0] for p in pairs])
    e = torch.cat([p[1] for p in pairs])
    del pairs, xs, btr
    net = gd.Net(seed=1)
    g = torch.Generator().manual_seed(0)
    nsteps, bs, lr = 300, 4, 2e-3
    perm = torch.randperm(r.shape[0], generator=g)
    losses = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(nsteps):
        i = (s * bs) % r.shape[0]
        idx = perm[i:i + bs] if i + bs <= r.shape[0] else perm[:bs]
        losses.append(net.train_step(r[idx].contiguous(), e[idx].contiguous(), lr=lr if s < 0.7 * nsteps else 0.2 * lr))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    sc = torch.sqrt((r.double() ** 2).mean(dim=(1, 2)))
    zero_loss = ((e.double() / sc[:, None, None]) ** 2).mean().item()
    del r, e
    b = stack(2048, 64, 13100431)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nvox = b.numel()
    h = gd.Hierarchy(tuple(b.shape), ALPHA, (1.0, 1.0, 0.0), torch.float32)

    def solve(mode):
        x = torch.zeros_like(b)
        if mode == "mg":
            for c in range(1, 100):
                rr = h.vcycle(x, b, 1)
                if rr <= TOL:
                    return {"iterations": c, "rel_residual": rr}
            raise RuntimeError("plain V-cycles did not converge")
        rep = h.fcg(x, b, net=net, precond=mode, rel_tol=TOL, max_iter=100)
        return rep

    results = {}
    for mode, name in (("mg", "plain_vcycles"), (0, "fcg_vcycle"), (3, "fcg_net_smoother"), (2, "fcg_vcycle_net")):
        for _ in range(a.warmup):
            solve(mode)
        torch.cuda.synchronize()
        if mode == 2:
            net.set_timing(True)
        t2 = time.perf_counter()
        for _ in range(a.steps):
            rep = solve(mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t2) / a.steps
        results[name] = {"ms_per_solve": dt * 1e3, "iterations": rep["iterations"],
                         "rel_residual": rep["rel_residual"], "voxels_per_s": nvox / dt}
        if mode in (2, 3):
            results[name]["fallback_used"] = rep["fallback_used"]
    layers = []
    for l in range(9):
        ms, n, fl = net.kernel_time(l)
        layers.append({"layer": l, "launches": n, "avg_launch_ms": ms / max(n, 1),
                       "TFLOP/s": fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0})
    net.set_timing(False)
    dom = max(range(9), key=lambda l: layers[l]["avg_launch_ms"] * layers[l]["launches"])
    peak = 2500.0  # dense BF16 MFMA, TFLOP/s
    learned = results["fcg_vcycle_net"]
    line = {
        "metric": "voxels/s to 1e-6 rel. residual (per-slice SP, learned-preconditioned FCG)",
        "value": learned["voxels_per_s"], "unit": "voxels/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": learned["ms_per_solve"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}; tol {TOL:g}", "nx": 2048, "ny": 2048, "nz": 64,
                   "voxels": nvox},
        "roofline": {"bound": "mfma", "achieved": layers[dom]["TFLOP/s"], "peak": peak, "unit": "TFLOP/s",
                     "frac": layers[dom]["TFLOP/s"] / peak, "traffic": None,
                     "kernel": f"k_conv3x3 forward, layer {dom}", "layers": layers},
        "solvers": results,
        "training": {"pairs": "48 (r_k, e_k), k = 1, 2, 3 V-cycles on 16 slices of 1024^2", "steps": nsteps,
                     "batch": bs, "seconds": train_s, "loss_first": losses[0], "loss_last": losses[-1],
                     "loss_zero_net": zero_loss},
        "setup_s": setup_s,
    }
    h.close()
    net.close()
    print(json.dumps(line), flush=True)


NPR = dict(alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.25, sigma=5.0)

# algorithmic HBM bytes per voxel of the spectral path for FP32 input and
# output: the x forward pass reads the input and writes FP64 (4 + 8), the y
# and z forward passes (the z pass also scales) and the z and y inverse
# passes read and write FP64 (8 + 8 each), the x inverse pass writes the
# output (8 + 4)
DCT_BYTES_PER_VOXEL = 12 + 4 * 16 + 12


def bench_dct(a, gd, synth, torch, desc):
    """Anisotropic diffusion of the stack1k input by the spectral solver;
    the multigrid AD of the same input is timed beside it."""
    spec = synth.CONFIGS["stack1k"]
    I0 = synth.make_stack(spec, device=torch.device("cuda:0"), dtype=torch.float32)
    torch.cuda.synchronize()
    nvox = I0.numel()
    out = torch.empty_like(I0)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / a.steps

    dt = timed(lambda: gd.dct_smooth_z(I0, BETA, out_dtype=torch.float32))
    rep = {}

    def mg():
        rep.update(gd.smooth_z(I0, BETA, out_dtype=torch.float32, rel_tol=TOL)[1])

    dt_mg = timed(mg)
    ref, _ = gd.dct_smooth_z(I0, BETA, out_dtype=torch.float64)
    mg_out, _ = gd.smooth_z(I0, BETA, out_dtype=torch.float64, rel_tol=TOL)
    diff = (torch.linalg.norm(mg_out - ref) / torch.linalg.norm(ref)).item()
    achieved = DCT_BYTES_PER_VOXEL * nvox / dt / 1e9
    line = {
        "metric": "voxels/s (anisotropic diffusion, exact spectral solve)",
        "value": nvox / dt, "unit": "voxels/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}", "nx": spec.nx, "ny": spec.ny, "nz": spec.nz,
                   "voxels": nvox},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole spectral path (six DCT passes, scaling and conversions fused), "
                               f"{DCT_BYTES_PER_VOXEL} algorithmic B/voxel"},
        "multigrid_ad": {"ms": dt_mg * 1e3, "voxels_per_s": nvox / dt_mg, "cycles": rep.get("cycles"),
                         "rel_residual": rep.get("rel_residual"),
                         "rel_difference_to_spectral": diff},
    }
    print(json.dumps(line), flush=True)


def bench_streamed(a, gd, synth, torch, desc):
    """V-cycles of the AD system of a stack with its large levels in pinned
    host memory (gd_vcycle_streamed), as many as the in-core cycles need to
    reach 1e-6 from zero; the in-core cycles are timed beside them and must
    give the same iterate."""
    spec = synth.CONFIGS[a.workload.split("-")[0]]
    I0 = synth.make_stack(spec, device=torch.device("cuda:0"), dtype=torch.float32)
    shape = tuple(I0.shape)
    nvox = I0.numel()
    pre, post = smooth_split(a)
    kw = dict(pre_smooth=pre, post_smooth=post)
    # right-hand side of Eq. (1): G = (d I0 / dx, d I0 / dy, 0) on the faces
    gx = torch.zeros_like(I0)
    gx[:, :, :-1] = I0[:, :, 1:] - I0[:, :, :-1]
    gy = torch.zeros_like(I0)
    gy[:, :-1, :] = I0[:, 1:, :] - I0[:, :-1, :]
    hc = gd.Hierarchy(shape, 0.0, BETA, torch.float32, **kw)
    b = hc.rhs(None, gx, gy, None)
    del gx, gy, I0
    xd = torch.zeros_like(b)
    cycles, rr = 0, 1.0
    while rr > TOL and cycles < 30:
        rr = hc.vcycle(xd, b, 1)
        cycles += 1
    bh = torch.empty(shape, dtype=torch.float32, pin_memory=True)
    bh.copy_(b)
    xh = torch.empty(shape, dtype=torch.float32, pin_memory=True)
    hs = gd.StreamedHierarchy(shape, 0.0, BETA, torch.float32, a.slab, a.stream_levels, **kw)

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / a.steps

    def streamed():
        xh.zero_()
        hs.vcycle(xh, bh, cycles, relres=False)

    def in_core():
        xd.zero_()
        hc.vcycle(xd, b, cycles)

    dt = timed(streamed)
    dt_c = timed(in_core)
    same = bool(torch.equal(xh, xd.cpu()))
    rr_s = hs.vcycle(xh, bh, 0)
    dev_s, planes = hs.device_bytes()
    dev_c, _ = hc.device_bytes()
    # host-link bytes of one cycle, level by level over the streamed levels
    # (planes shared by consecutive windows are copied on the device, so
    # every plane crosses the link once per pass): down pass: b (and x on
    # the finest level; a coarser level's x starts at zero on the device), x
    # written back, the restricted residual written back when the next level
    # is streamed; up pass: x and b (and the coarse correction under every
    # window when the next level is streamed), x written back
    halo = 2 * max(pre, post) + 2
    ns = hs.streamed_levels()
    dims = [hs.info(l)[0] for l in range(ns + 1)]
    link = 0
    for l in range(ns):
        nz_l, ny_l, nx_l = dims[l]
        nzc, nyc, nxc = dims[l + 1]
        fz = 2 if nzc < nz_l else 1
        plane, cplane = nx_l * ny_l * 4, nxc * nyc * 4
        slab_l = min(nz_l, max(a.slab + a.slab % 2, halo))
        coarse_win = 0
        for z0 in range(0, nz_l, slab_l):
            z1 = min(nz_l, z0 + slab_l)
            wa, we = max(0, z0 - halo), min(nz_l, z1 + halo)
            coarse_win += (we - wa + fz - 1) // fz
        down = (nz_l * (2 if l == 0 else 1) + nz_l) * plane
        upp = 3 * nz_l * plane
        if l + 1 < ns:
            down += nzc * cplane
            upp += coarse_win * cplane
        link += down + upp
    link *= cycles
    slab = min(spec.nz, max(a.slab + a.slab % 2, halo))
    # a plain pinned upload of 1 GiB, the link's practical rate
    src = torch.empty(1 << 28, dtype=torch.float32, pin_memory=True)
    dst = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    copy_gbs = 3 * src.numel() * 4 / (time.perf_counter() - t0) / 1e9
    line = {
        "metric": "voxels/s (anisotropic-diffusion V-cycles, large levels streamed from host memory)",
        "value": nvox / dt, "unit": "voxels/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}", "nx": spec.nx, "ny": spec.ny, "nz": spec.nz,
                   "voxels": nvox, "cycles": cycles, "slab": slab, "halo": halo, "window_planes": planes,
                   "streamed_levels": ns},
        "link": {"bytes_per_step": link, "achieved_gbs": link / dt / 1e9, "pinned_upload_gbs": copy_gbs,
                 "note": "host<->device bytes of the streamed passes (uploads and write-backs; planes shared by consecutive windows are copied on the device)"},
        "device_bytes": {"streamed": dev_s, "in_core": dev_c},
        "in_core": {"ms": dt_c * 1e3, "voxels_per_s": nvox / dt_c, "same_iterate": same,
                    "rel_residual": rr},
        "rel_residual": rr_s,
    }
    print(json.dumps(line), flush=True)


def bench_npr(a, gd, synth, torch, desc):
    """Gradient-modulation filter (Sec. 6) of a synthetic 1920x1080x742 video
    volume: one step = the modulated right-hand side, V-cycles to 1e-6 and
    the output, inputs resident in HBM."""
    spec = synth.VIDEO_CONFIGS["video1080"]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    I0 = synth.make_video(spec, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nvox = I0.numel()
    pre, post = smooth_split(a)
    opts = dict(rel_tol=TOL, pre_smooth=pre, post_smooth=post)

    def step(timing):
        return gd.npr_filter(I0, NPR["alpha"], NPR["beta"], NPR["lam"], NPR["sigma"], timing=timing, **opts)[1]

    for _ in range(a.warmup):
        step(0)
    torch.cuda.synchronize()
    gd.reset_kernel_time()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        rep = step(1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    ms, launches, bytes_per = gd.kernel_time(gd.SWEEP_STACK)
    avg_ms = ms / max(launches, 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    cfg = gd.sweep_config((spec.nt, spec.ny, spec.nx), torch.float32)
    line = {
        "metric": "voxels/s to 1e-6 rel. residual (gradient-modulation filter)",
        "value": nvox / dt, "unit": "voxels/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.workload}: {desc}; Neumann, tol {TOL:g}", "nx": spec.nx, "ny": spec.ny,
                   "nz": spec.nt, "voxels": nvox, "smooth": [pre, post]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_rb_sweep<f32,%d,%d,false,true> finest level" % tuple(cfg["tile"]),
                     "sweep_config": cfg, "launches": launches, "avg_launch_ms": avg_ms,
                     "algorithmic_bytes_per_launch": bytes_per},
        "solve": {"cycles": rep["cycles"], "rel_residual": rep["rel_residual"], "levels": rep["levels"]},
        "generate_s": gen_s,
    }
    if not a.no_cpu_baseline:
        from oracle import npr

        nz, ny, nx = (int(v) for v in a.cpu_crop.split(","))
        sub = I0[:nz, :ny, :nx].double().cpu().numpy()
        t1 = time.perf_counter()
        npr.npr_filter(sub, NPR["alpha"], NPR["beta"], NPR["lam"], NPR["sigma"], method="cg", rtol=TOL)
        cdt = time.perf_counter() - t1
        line["cpu_baseline"] = {
            "value": sub.size / cdt, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"crop [0:{nz},0:{ny},0:{nx}] of the same video ({sub.size} voxels), modulated field and "
                      f"right-hand side, then conjugate gradients to {TOL:g}, numpy FP64, {cdt:.1f} s"}
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {a.gpus}); "
              "sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1310_0041_amd as gd
    import synth

    if a.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 4, "copies": 3}))
        return
    gd.load()
    spec_key, storage, refine, desc = WORKLOADS[a.workload]
    spec = synth.CONFIGS.get(spec_key)

    if spec_key == "slices":
        return bench_slices(a, gd, synth, torch, desc)
    if spec_key == "learned":
        return bench_learned(a, gd, synth, torch, desc)
    if spec_key == "npr":
        return bench_npr(a, gd, synth, torch, desc)
    if spec_key == "dct":
        return bench_dct(a, gd, synth, torch, desc)
    if spec_key.startswith("streamed"):
        return bench_streamed(a, gd, synth, torch, desc)
    legs = [(storage, refine)]
    if a.workload == "stack4k":  # the headline line carries the other storage types as legs
        legs += [("bf16", 1), ("f32", 0)]
    results = []
    for i, (stg, ref) in enumerate(legs):
        steps, warmup = (a.steps, a.warmup) if i == 0 else (min(a.steps, 5), min(a.warmup, 1))
        results.append(run_stack_leg(a, gd, synth, torch, spec, stg, ref, steps, warmup))
        gd.release_workspace()
        torch.cuda.empty_cache()
    head = results[0]
    line = {
        "metric": "voxels/s to 1e-6 rel. residual (AD + per-slice SP)",
        "value": head["voxels_per_s"],
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16": "f16+f64", "bf16": "bf16+f64"}[storage],
        "data": "synthetic",
        "config": {
            "workload": f"{a.workload}: {desc}; beta=(1,1,4), alpha={ALPHA}, Neumann, tol {TOL:g}"
                        + ("" if a.discretization == "constant" and a.prolong == "trilinear"
                           else f"; AD {a.discretization} discretisation, {a.prolong} up-sampling"),
            "nx": spec.nx, "ny": spec.ny, "nz": spec.nz, "voxels": spec.nx * spec.ny * spec.nz,
            "smooth": list(smooth_split(a, storage, refine)),
        },
        "roofline": head["roofline"],
        "ad": head["ad"],
        "sp": head["sp"],
        "generate_s": head["generate_s"],
    }
    if len(results) > 1:
        line["legs"] = {r["leg"]: {k: r[k] for k in ("ms_per_step", "voxels_per_s", "steps", "warmup", "smooth", "ad",
                                                     "sp", "finest_sweep")}
                        for r in results}
        plain = next(r for r in results if r["leg"] == "f32")
        line["legs"]["speedup_vs_f32_plain"] = {r["leg"]: plain["ms_per_step"] / r["ms_per_step"] for r in results}
    if not a.no_cpu_baseline:
        crop = tuple(int(v) for v in a.cpu_crop.split(","))
        sub = synth.make_stack(spec, device="cuda", z_range=(0, crop[0]))[:, :crop[1], :crop[2]]
        sub = sub.to({"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]).double().cpu()
        line["cpu_baseline"] = cpu_baseline(sub.numpy(), crop)
    print(json.dumps(line), flush=True)


def source_sha(path):
    import hashlib

    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


SWEEP_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1310_0041_amd", "csrc", "k_sweep.hip")


def measured_traffic(a, leg, tile):
    """HBM bytes per launch of this leg's finest relaxation from the committed
    rocprofv3 counters (FETCH_SIZE, WRITE_SIZE, each scaled by what it reads
    for a plain copy), used only when they were taken on the same workload,
    storage type and tile from the same relaxation source (sha)."""
    if not os.path.exists(a.traffic_json):
        return None, None
    try:
        t = json.load(open(a.traffic_json))
    except Exception:
        return None, None
    entries = t if isinstance(t, list) else [t]
    sha = source_sha(SWEEP_SRC)
    spec_key = WORKLOADS[a.workload][0]  # the input (stack4k-f16 is the stack4k input's FP16 leg)
    for e in entries:
        if (e.get("workload") == spec_key and e.get("storage", "f32") == leg and list(e.get("tile", [])) == list(tile)
                and e.get("source_sha") == sha):
            return e["bytes_per_launch"], (f"{os.path.relpath(a.traffic_json)}: rocprofv3 FETCH_SIZE x "
                                           f"{e['fetch_factor']:.3g} + WRITE_SIZE x {e['write_factor']:.3g} of this "
                                           f"launch, k_sweep.hip sha {sha}")
    return None, None


def run_stack_leg(a, gd, synth, torch, spec, storage, refine, steps, warmup):
    """One storage type of the stack workload: AD then per-slice SP of the
    whole stack, each to 1e-6, inputs resident in HBM; `steps` timed steps."""
    tdt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]
    sdt = {"f32": gd.F32, "f16": gd.F16, "bf16": gd.BF16}[storage]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    I0 = synth.make_stack(spec, device=dev, dtype=tdt)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nvox = I0.numel()
    out_dtype = torch.float32  # I1 and I2 in FP32 (16-bit storage covers the input and the V-cycles)
    pre, post = smooth_split(a, storage, refine)
    opts = dict(storage=sdt, fp64_refine=refine, rel_tol=TOL, pre_smooth=pre, post_smooth=post)
    if a.inner_cycles is not None:
        opts["inner_cycles"] = a.inner_cycles
    if a.fmg is not None:
        opts["fmg"] = a.fmg
    opts["prolong"] = 0 if a.prolong == "trilinear" else 1
    ad_opts = dict(opts, discretization={"constant": 0, "hybrid": 1, "linear": 2}[a.discretization])
    I1 = torch.empty_like(I0, dtype=out_dtype)
    I2 = torch.empty_like(I0, dtype=out_dtype)

    def step(timing):
        r1 = gd.smooth_z_into(I0, I1, BETA, timing=timing, **ad_opts)
        _, r2, _ = gd.screened_poisson_stack(I0, I1, ALPHA, timing=timing, out=I2, **ad_opts)
        return r1, r2

    for _ in range(warmup):
        step(0)
    torch.cuda.synchronize()
    gd.reset_kernel_time()
    t0 = time.perf_counter()
    reps = []
    for _ in range(steps):
        reps.append(step(1))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # dominant kernel: the finest-level relaxation of the stack (AD phase)
    ms, launches, bytes_per = gd.kernel_time(gd.SWEEP_STACK)
    avg_ms = ms / max(launches, 1)
    others = {}
    for name, v in (("stack_fused_prolong", gd.SWEEP_STACK_PROLONG), ("slice", gd.SWEEP_SLICE),
                    ("slice_fused_prolong", gd.SWEEP_SLICE_PROLONG), ("stack_from_zero", gd.SWEEP_STACK_ZERO),
                    ("slice_from_zero", gd.SWEEP_SLICE_ZERO)):
        m2, n2, b2 = gd.kernel_time(v)
        if n2:
            others[name] = {"launches": n2, "avg_launch_ms": m2 / n2, "GB/s": b2 / (m2 / n2 * 1e-3) / 1e9}
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    cfg = gd.sweep_config((spec.nz, spec.ny, spec.nx), tdt)
    traffic, traffic_src = measured_traffic(a, storage, cfg["tile"])
    r1, r2 = reps[-1]
    tname = {"f32": "float", "f16": "__half", "bf16": "__hip_bfloat16"}[storage]
    roof = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "traffic_source": traffic_src,
        "kernel": "k_rb_sweep4<%s, %d, %d, false> finest level (HIP events on the solve's stream)"
                  % ((tname,) + tuple(cfg["tile"])),
        "sweep_config": cfg,
        "launches": launches,
        "avg_launch_ms": avg_ms,
        "algorithmic_bytes_per_launch": bytes_per,
        "other_finest_sweeps": others,
    }
    leg = {
        "leg": storage, "steps": steps, "warmup": warmup, "ms_per_step": dt * 1e3, "voxels_per_s": nvox / dt,
        "smooth": [pre, post],
        "generate_s": gen_s, "roofline": roof,
        "finest_sweep": {"avg_launch_ms": avg_ms, "GB/s": achieved, "frac": achieved / HBM_PEAK_GBS,
                         "tile": cfg["tile"]},
        "ad": {"cycles": r1["cycles"], "refine_steps": r1["refine_steps"], "rel_residual": r1["rel_residual"],
               "levels": r1["levels"], "bytes": r1["bytes"], "discretization": a.discretization,
               "prolong": a.prolong, "factor_per_cycle": r1["rel_residual"] ** (1.0 / max(r1["cycles"], 1))},
        "sp": {"cycles": r2["cycles"], "refine_steps": r2["refine_steps"], "rel_residual": r2["rel_residual"],
               "bytes": r2["bytes"], "factor_per_cycle": r2["rel_residual"] ** (1.0 / max(r2["cycles"], 1))},
    }
    del I0, I1, I2
    return leg


if __name__ == "__main__":
    main()
