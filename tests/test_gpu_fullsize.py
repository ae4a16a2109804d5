"""Parity at the full workload sizes, in the configuration bench.py times.

* 1024x1024x128 FP32 stack: the whole answer against the FP64 DCT oracle.
* 4096x4096x256 FP16/BF16 stack with FP64 refinement: the 512x512x32 crop
  solved as its own problem against the oracle; the full stack through
  properties that hold at any size (slice means of the answer equal the
  global input mean; the oracle's own residual on sampled slabs).
"""

import os

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og
from oracle import linear as olin
from oracle import solvers as osv

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
BETA = (1.0, 1.0, 4.0)


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_stack1k_full_against_dct(gd):
    say("stack1k full AD+SP vs DCT")
    spec = synth.CONFIGS["stack1k"]
    I0 = synth.make_stack(spec, device="cuda", dtype=torch.float32)
    # error <= 1e-5 needs the residual a little below 1e-6 here (the smoothest
    # modes amplify it ~13x); 4e-7 is above this stack's FP32 floor (~2.6e-7)
    opts = dict(pre_smooth=1, post_smooth=2, rel_tol=4e-7, check=False)
    I1, r1 = gd.smooth_z(I0, BETA, out_dtype=torch.float64, **opts)
    print("AD", r1, flush=True)
    assert r1["rel_residual"] <= 1e-6
    I2, r2, per = gd.screened_poisson_stack(I0, I1.float(), 0.01, **opts)
    print("SP", r2, flush=True)
    assert r2["rel_residual"] <= 1e-6
    a0 = I0.double().cpu().numpy()
    ref1 = osv.ad_dct(a0, BETA)
    assert rel(I1.cpu().numpy(), ref1) <= 1e-5
    # the SP phase as run: value target = the FP32 AD output the GPU used
    ref2 = osv.sp_dct(a0, I1.float().double().cpu().numpy(), 0.01)
    assert rel(I2.double().cpu().numpy(), ref2) <= 1e-5


def test_stack1k_hybrid_full_against_dct(gd):
    """The stack1k workload with the Hybrid discretisation as bench.py runs it
    (AD, then the SP slices as one stack grid; its large 27-point levels take
    the plane-parity relaxation): both phases against the FP64 DCT oracle of
    the 7-point system, which Hybrid keeps on the finest level: SP to 1e-5,
    AD to its FP32 floor's 1.2e-5 (below)."""
    say("stack1k Hybrid full AD+SP vs DCT")
    spec = synth.CONFIGS["stack1k"]
    I0 = synth.make_stack(spec, device="cuda", dtype=torch.float32)
    # In FP32 storage Hybrid's AD stops at its floor, a relative residual of
    # 3.1e-7 (Constant reaches 2.6e-7), where its error against the oracle is
    # 1.13e-5 whatever tolerance below that is asked: the error bar of this
    # phase is that floor's, 1.2e-5 (FP64 and refined FP16 storage are held
    # to 1e-8 and 1e-6 by the small-size Hybrid tests).
    opts = dict(rel_tol=4e-7, check=False, discretization=1)
    I1, r1 = gd.smooth_z(I0, BETA, out_dtype=torch.float64, **opts)
    print("AD", r1, flush=True)
    assert r1["rel_residual"] <= 4e-7
    I2, r2, per = gd.screened_poisson_stack(I0, I1.float(), 0.01, out_dtype=torch.float64, **opts)
    print("SP", r2, flush=True)
    assert max(p["rel_residual"] for p in per) <= 4e-7
    a0 = I0.double().cpu().numpy()
    assert rel(I1.cpu().numpy(), osv.ad_dct(a0, BETA)) <= 1.2e-5
    assert rel(I2.cpu().numpy(), osv.sp_dct(a0, I1.float().double().cpu().numpy(), 0.01)) <= 1e-5
    gd.release_workspace()


def test_stack1k_linear_sp_sampled(gd):
    """The Linear SP phase of the stack1k workload as bench.py runs it (the
    128 slices as one stack grid, FP32 storage, to 1e-6 per slice): sampled
    slices by the oracle's own residual of the Linear system (the answer's
    parity at this size would need the oracle's per-slice CG on 1024^2
    slices; the stack route's answer is checked against it at small sizes)."""
    say("stack1k Linear SP, sampled slices by the oracle's residual")
    spec = synth.CONFIGS["stack1k"]
    I0 = synth.make_stack(spec, device="cuda", dtype=torch.float32)
    I1, r1 = gd.smooth_z(I0, BETA, discretization=2, check=False)
    assert r1["rel_residual"] <= 1e-6
    I2, r2, per = gd.screened_poisson_stack(I0, I1, 0.01, discretization=2, out_dtype=torch.float64)
    print("SP", r2, flush=True)
    assert r2["status"] == 0 and max(p["rel_residual"] for p in per) <= 1e-6
    for z in (0, 77, 127):
        res = olin.sp_relative_residuals(I2[z:z + 1].cpu().numpy(), I0[z:z + 1].double().cpu().numpy(),
                                         I1[z:z + 1].double().cpu().numpy(), 0.01)
        say(f"slice {z}: oracle residual {res[0]:.2e}")
        assert res[0] <= 2e-6
    gd.release_workspace()


@pytest.mark.parametrize("dt", [torch.float16, torch.bfloat16])
def test_stack4k_crop_mixed(gd, dt):
    """The 512x512x32 crop of the 4096x4096x256 stack, solved as its own
    problem with 16-bit storage of the input and the V-cycles and FP64
    refinement, end to end: the FP64 result of the anisotropic diffusion
    feeds the screened-Poisson phase, whose refined result comes back in
    FP64.  Both phases and the pipeline match the FP64 oracle to 1e-6."""
    say("stack4k crop mixed", dt)
    spec = synth.CONFIGS["stack4k"]
    full = synth.make_stack(spec, device="cuda", z_range=(0, 32))
    crop = full[:, :512, :512].to(dt).contiguous()
    del full
    st = gd.F16 if dt == torch.float16 else gd.BF16
    I1, r1 = gd.smooth_z(crop, BETA, out_dtype=torch.float64, storage=st, fp64_refine=1, rel_tol=5e-8)
    a0 = crop.double().cpu().numpy()
    ref1 = osv.ad_dct(a0, BETA)
    assert r1["rel_residual"] <= 5e-8
    assert rel(I1.cpu().numpy(), ref1) <= 1e-6
    I2, r2, per = gd.screened_poisson_stack(crop, I1, 0.01, storage=st, fp64_refine=1, rel_tol=5e-8,
                                            out_dtype=torch.float64)
    assert I2.dtype == torch.float64 and r2["rel_residual"] <= 5e-8
    assert max(p["rel_residual"] for p in per) <= 5e-8
    got = I2.cpu().numpy()
    # the phase as run (value target: the GPU's own FP64 AD result) ...
    e_phase = rel(got, osv.sp_dct(a0, I1.cpu().numpy(), 0.01))
    # ... and the whole pipeline against the oracle's AD then SP
    e_pipe = rel(got, osv.sp_dct(a0, ref1, 0.01))
    say(f"AD err {rel(I1.cpu().numpy(), ref1):.2e}; SP err {e_phase:.2e}; pipeline err {e_pipe:.2e}")
    assert e_phase <= 1e-6 and e_pipe <= 1e-6
    gd.release_workspace()


@pytest.mark.parametrize("dt", [torch.float16])
def test_stack4k_full_properties(gd, dt):
    say("stack4k full mixed", dt)
    spec = synth.CONFIGS["stack4k"]
    I0 = synth.make_stack(spec, device="cuda", dtype=dt)
    I1, r1 = gd.smooth_z(I0, BETA, out_dtype=torch.float32, storage=gd.F16, fp64_refine=1)
    assert r1["rel_residual"] <= 1e-6
    # slice means of the answer equal the global mean of the input
    gm = I0.double().mean().item()
    sm = I1.double().mean(dim=(1, 2)).cpu().numpy()
    assert np.abs(sm - gm).max() <= 1e-5 * max(1.0, abs(gm)) + 1e-3
    # the oracle's residual on sampled slabs (interior planes k0 .. k0+7,
    # with their z-neighbours for the stencil)
    rng = np.random.default_rng(0)
    for k0 in rng.choice(np.arange(1, 256 - 9), 2, replace=False):
        sl = slice(int(k0) - 1, int(k0) + 9)
        x = I1[sl].double().cpu().numpy()
        i0 = I0[sl].double().cpu().numpy()
        r = og.rhs_ad(i0, BETA) - og.apply_A(x, 0.0, BETA)
        b = og.rhs_ad(i0, BETA)
        inner = slice(1, -1)
        # FP32 output rounding floor: ~3e-6 of ||b|| per slab; the solve itself is at 1e-6
        assert np.linalg.norm(r[inner]) <= 2e-5 * np.linalg.norm(b[inner])
    del I0, I1
    gd.release_workspace()
    torch.cuda.empty_cache()


def _sp_slice_errors(gd, meta, I2, idx):
    """Relative error of each slice in `idx` against the FP64 DCT oracle of
    its own system (slices copied to the host one at a time; the oracle runs
    in a thread pool, scipy's transforms release the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    w, h, a, off = meta["w"], meta["h"], meta["alpha"], meta["offset"]

    def one(i):
        n = int(w[i]) * int(h[i])
        sh = (1, int(h[i]), int(w[i]))
        s0 = meta["I0h"][off[i]:off[i] + n].astype(np.float64).reshape(sh)
        s1 = meta["I1h"][off[i]:off[i] + n].astype(np.float64).reshape(sh)
        got = meta["I2h"][off[i]:off[i] + n].astype(np.float64).reshape(sh)
        return rel(got, osv.sp_dct(s0, s1, float(np.float32(a[i]))))

    meta["I0h"], meta["I1h"], meta["I2h"] = (t.cpu().numpy() for t in (meta["I0"], meta["I1"], I2))
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return np.array(list(ex.map(one, idx)))


def test_slices2048_full_all_slices(gd):
    """The 2048 uneven slices of the batched workload, solved as bench.py
    solves them (one batched solve, FP32, V(1,2)) to 5e-8 per slice (each
    slice leaves the batch at its own tolerance, and the smoothest modes of
    the small-alpha slices amplify the residual about 100 times), so that the
    error bar of 1e-5 holds; every slice against the FP64 DCT oracle of its
    own system."""
    say("slices2048 full batch, every slice vs DCT")
    meta = synth.make_slice_batch(device="cuda", dtype=torch.float32)
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    I2, rep, per = gd.screened_poisson_slices(meta["I0"], meta["I1"], descs, rel_tol=5e-8, pre_smooth=1,
                                              post_smooth=2, check=False)
    print("batch", {k: rep[k] for k in ("cycles", "rel_residual", "status")}, flush=True)
    res = np.array([p["rel_residual"] for p in per])
    assert res.max() <= 1e-6
    err = _sp_slice_errors(gd, meta, I2, range(len(descs)))
    worst = int(np.argmax(err))
    say(f"{len(err)} slices: max rel err {err.max():.2e} (slice {worst}, {meta['w'][worst]}x{meta['h'][worst]}, "
        f"alpha {meta['alpha'][worst]:.4f}), median {np.median(err):.2e}")
    assert err.max() <= 1e-5


def test_learned2k_full_sampled(gd):
    """The learned workload's solve (2048x2048x64 per-slice SP, alpha 0.01)
    by flexible CG with the V-cycle + net preconditioner, as bench.py runs it
    after training: the net stays in use (no fallback to the V-cycle), the
    true residual reaches 1e-6 in fewer iterations than with the V-cycle
    alone, and sampled slices agree with the FP64 DCT oracle to 1e-5."""
    say("learned2k full solve, sampled slices vs DCT")
    n, nz, alpha = 2048, 64, 0.01
    spec = synth.StackSpec(n, n, nz, (4.0, 40.0), True, 13100431)
    I0 = synth.make_stack(spec, device="cuda", dtype=torch.float32)
    I1 = torch.roll(I0, 1, 0).contiguous()
    b = torch.zeros_like(I0, dtype=torch.float64)
    b += alpha * I1.double()
    for ax in (2, 1):
        d = torch.diff(I0.double(), dim=ax)
        m = I0.shape[ax]
        b.narrow(ax, 0, m - 1).sub_(d)
        b.narrow(ax, 1, m - 1).add_(d)
    b = b.float().contiguous()
    # a briefly trained net (the pairs of a 1024^2 stack, as bench.py)
    tb = b[:16, :1024, :1024].contiguous()
    ht = gd.Hierarchy(tuple(tb.shape), alpha, (1.0, 1.0, 0.0), torch.float32)
    xs = torch.zeros_like(tb)
    ht.vcycle(xs, tb, 30)
    r, e = ht.error_pairs(tb, xs, 1)
    ht.close()
    net = gd.Net(seed=1)
    for s in range(100):
        i = (4 * s) % 16
        net.train_step(r[i:i + 4].contiguous(), e[i:i + 4].contiguous(), lr=2e-3)
    h = gd.Hierarchy(tuple(b.shape), alpha, (1.0, 1.0, 0.0), torch.float32)
    x = torch.zeros_like(b)
    rep = h.fcg(x, b, net=net, precond=2, rel_tol=1e-6, max_iter=100)
    # the same FCG with the V-cycle alone: the net saves an iteration at this
    # size (measured 4 against 5; in time it still loses, ~3.5x per solve)
    x0 = torch.zeros_like(b)
    rep0 = h.fcg(x0, b, precond=0, rel_tol=1e-6, max_iter=100)
    h.close()
    net.close()
    print("fcg", rep, "v-cycle only", rep0, flush=True)
    assert rep["rel_residual"] <= 1e-6
    assert rep["fallback_used"] == 0
    assert rep["cycles"] < rep0["cycles"], (rep["cycles"], rep0["cycles"])
    for z in (0, 31, 63):
        ref = osv.dct_solve(b[z:z + 1].double().cpu().numpy(), alpha, (1.0, 1.0, 0.0))
        err = rel(x[z:z + 1].double().cpu().numpy(), ref)
        say(f"slice {z}: rel err {err:.2e}")
        assert err <= 1e-5
