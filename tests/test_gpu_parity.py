"""HIP path vs the FP64 oracle, element by element, on the same seeded inputs.

Kernel-level steps (one red-black sweep, residual + restriction,
prolongation) are compared to the oracle's definitions of the same step;
whole solves are compared to the oracle's solution of the paper's systems.
Tolerances: FP64 steps 1e-12 relative, FP32 steps 2e-6 relative (a handful
of roundings of values of similar magnitude); solves to 1e-6 (FP64 iterate)
or 1e-5 (plain FP32) relative L2, the bars stated for this path.
"""

import os

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og
from oracle import mgsteps as om
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

BETA = (1.0, 1.0, 4.0)
TD = {np.float64: torch.float64, np.float32: torch.float32}


def say(*a):
    print("[case]", *a, flush=True)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    return t.double().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


STEP_SHAPES = [(9, 17, 130), (1, 33, 200), (40, 3, 5), (3, 8, 64), (1, 1, 1), (5, 1, 7), (2, 70, 1), (1, 300, 517),
               (1, 7, 1), (6, 21, 67)]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", STEP_SHAPES)
@pytest.mark.parametrize("alpha,w", [(0.0, BETA), (0.01, (1.0, 1.0, 0.0)), (0.7, (2.0, 0.5, 3.0))])
def test_rb_sweep_step(gd, dt, shape, alpha, w):
    say("rb_sweep", shape, dt, alpha, w)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(shape) * 10
    b = rng.standard_normal(shape)
    xq, bq = host(dev(x, dt)), host(dev(b, dt))
    ref = om.rb_sweep(xq, bq, alpha, w)
    out = host(gd.rb_sweep(dev(x, dt), dev(b, dt), alpha, w))
    tol = 1e-12 if dt == torch.float64 else 2e-6
    assert np.abs(out - ref).max() <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", STEP_SHAPES)
@pytest.mark.parametrize("c", [(2, 2, 2), (1, 1, 2), (2, 2, 1)])
def test_residual_restrict_step(gd, dt, shape, c):
    say("residual_restrict", shape, dt, c)
    rng = np.random.default_rng(2)
    alpha, w = 0.3, (1.0, 2.0, 4.0)
    x = rng.standard_normal(shape) * 10
    b = rng.standard_normal(shape)
    xq, bq = host(dev(x, dt)), host(dev(b, dt))
    r = om.residual(xq, bq, alpha, w)
    ref = om.restrict_sum(r, c)
    bc, n2 = gd.residual_restrict(dev(x, dt), dev(b, dt), alpha, w, c)
    tol = 1e-12 if dt == torch.float64 else 2e-6
    scale = max(1.0, np.abs(xq).max() * 24)
    assert np.abs(host(bc) - ref).max() <= tol * scale * 8
    assert abs(n2 - float((r * r).sum())) <= 1e-5 * float((r * r).sum()) + 1e-12


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", STEP_SHAPES)
@pytest.mark.parametrize("c", [(2, 2, 2), (1, 1, 2), (2, 2, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_prolong_step(gd, dt, shape, c, mode):
    say("prolong", shape, dt, c, mode)
    rng = np.random.default_rng(3)
    cs = om.coarse_shape(shape, c)
    e = rng.standard_normal(cs)
    x = rng.standard_normal(shape)
    eq, xq = host(dev(e, dt)), host(dev(x, dt))
    P = om.prolong_trilinear if mode == 0 else om.prolong_constant
    ref = xq + P(eq, shape, c)
    out = host(gd.prolong_add(dev(e, dt), dev(x, dt), c, mode))
    tol = 1e-13 if dt == torch.float64 else 1e-6
    assert np.abs(out - ref).max() <= tol * max(1.0, np.abs(ref).max())


# ----------------------------------------------------------------- solves


def stack(spec, dt):
    I0 = synth.make_stack(spec).numpy()
    return host(dev(I0, dt))  # the quantised input both sides see


def test_ad_then_sp_fp64_stack64(gd):
    """64x64x16, FP64, V-cycles to 1e-8 (the FP64 plain configuration)."""
    say("AD+SP f64 64x64x16")
    I0 = stack(synth.CONFIGS["stack64"], torch.float64)
    I1, rep = gd.smooth_z(dev(I0, torch.float64), BETA, storage=gd.F64, rel_tol=1e-8)
    assert rep["rel_residual"] <= 1e-8
    ref1 = osv.ad_dct(I0, BETA)
    assert rel(host(I1), ref1) <= 1e-6
    # residual recomputed by the oracle on the returned FP64 output
    b = og.rhs_ad(I0, BETA)
    assert om.relative_residual(host(I1), b, 0.0, BETA) <= 1.01e-8
    I2, rep2, per = gd.screened_poisson_stack(dev(I0, torch.float64), I1, 0.01, storage=gd.F64, rel_tol=1e-8)
    assert rep2["rel_residual"] <= 1e-8
    ref2 = osv.sp_dct(I0, host(I1), 0.01)
    assert rel(host(I2), ref2) <= 1e-6
    assert rel(host(I2), osv.sp_dct(I0, ref1, 0.01)) <= 1e-6


def fp32_floor(I0, ref, b):
    """Relative residual of the exact answer when its correction I1 - I0 is
    stored in FP32: no plain FP32 iterate can do much better."""
    E = (ref - I0).astype(np.float32).astype(np.float64)
    return om.relative_residual(I0 + E, b, 0.0, BETA)


@pytest.mark.parametrize("shape", [(32, 256, 256), (7, 45, 99), (1, 40, 33), (16, 1, 64), (3, 2, 1), (16, 64, 64)])
def test_ad_plain_fp32(gd, shape):
    say("AD f32 plain", shape)
    nz, ny, nx = shape
    spec = synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100412)
    I0 = stack(spec, torch.float32)
    ref = osv.ad_dct(I0, BETA)
    b = og.rhs_ad(I0, BETA)
    tol = 1e-6
    if np.linalg.norm(b) > 0:
        tol = max(1e-6, 3.0 * fp32_floor(I0, ref, b))
    I1, rep = gd.smooth_z(dev(I0), BETA, out_dtype=torch.float64, rel_tol=tol)
    assert rep["status"] == 0 and rep["rel_residual"] <= tol
    assert rel(host(I1), ref) <= 1e-5
    if np.linalg.norm(b) > 0:
        assert om.relative_residual(host(I1), b, 0.0, BETA) <= 1.01 * tol
    # gauge: mean preserved
    assert abs(host(I1).mean() - I0.mean()) <= 1e-9 * max(1.0, abs(I0.mean()))


@pytest.mark.parametrize("fuse", [0, 1])
def test_prolongation_fused_or_separate(gd, fuse):
    """The coarse correction added in its own pass or inside the first
    post-smoothing sweep's loads gives the same answer."""
    say("AD fuse_prolong", fuse)
    spec = synth.StackSpec(70, 50, 12, (4.0, 40.0), True, 13100412)
    I0 = stack(spec, torch.float64)
    I1, rep = gd.smooth_z(dev(I0, torch.float64), BETA, storage=gd.F64, rel_tol=1e-10, fuse_prolong=fuse)
    assert rep["rel_residual"] <= 1e-10
    assert rel(host(I1), osv.ad_dct(I0, BETA)) <= 1e-8
    for p in (0, 1):  # trilinear and piecewise-constant up-sampling
        I1, rep = gd.smooth_z(dev(I0, torch.float64), BETA, storage=gd.F64, rel_tol=1e-10, fuse_prolong=fuse,
                              prolong=p)
        assert rep["rel_residual"] <= 1e-10


def test_plain_fp32_stops_at_its_floor(gd):
    """Smooth slices with strong slice-to-slice jumps: the FP32 correction
    cannot represent an answer at 1e-9; the solve stops on stagnation and
    says so, with a finite best iterate close to the oracle."""
    say("AD f32 floor")
    spec = synth.StackSpec(64, 64, 16, (4.0, 40.0), False, 13100411)
    I0 = stack(spec, torch.float32)
    I1, rep = gd.smooth_z(dev(I0), BETA, out_dtype=torch.float64, rel_tol=1e-9, check=False)
    assert rep["status"] == gd.ERR_NOT_CONVERGED
    assert rep["cycles"] < 40
    assert rel(host(I1), osv.ad_dct(I0, BETA)) <= 1e-5


@pytest.mark.parametrize("storage", ["f16", "bf16", "f32"])
def test_ad_mixed_refinement(gd, storage):
    say("AD mixed", storage)
    st = {"f16": gd.F16, "bf16": gd.BF16, "f32": gd.F32}[storage]
    tin = {"f16": torch.float16, "bf16": torch.bfloat16, "f32": torch.float32}[storage]
    spec = synth.StackSpec(96, 80, 24, (4.0, 40.0), True, 13100413)
    I0f = synth.make_stack(spec)
    I0 = I0f.to(tin).double().numpy()
    ref = osv.ad_dct(I0, BETA)
    I1, rep = gd.smooth_z(I0f.to(tin).cuda(), BETA, out_dtype=torch.float64, storage=st, fp64_refine=1)
    assert rep["rel_residual"] <= 1e-6 and rep["refine_steps"] >= 1
    assert rel(host(I1), ref) <= 1e-5
    # the error bar of 1e-6 vs the oracle needs a residual below it (the
    # smoothest modes have eigenvalues ~1e-3): the FP64 iterate gets there
    I1, rep = gd.smooth_z(I0f.to(tin).cuda(), BETA, out_dtype=torch.float64, storage=st, fp64_refine=1,
                          rel_tol=2e-7)
    assert rep["rel_residual"] <= 2e-7
    assert rel(host(I1), ref) <= 1e-6


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("factor", [2.0 ** 10, 2.0 ** -10])
def test_mixed_refinement_power_of_two_invariant(gd, storage, factor):
    """16-bit storage with FP64 refinement covers the range of the input:
    the right-hand side and every refinement residual are scaled by powers
    of two, so scaling I0 by 2^k scales the AD and SP results by exactly 2^k
    (bit for bit), for inputs up to 2.6e5 (far beyond FP16's 65504) and
    down to 2.5e-1."""
    say("mixed 2^k invariance", storage, factor)
    st = {"f16": gd.F16, "bf16": gd.BF16}[storage]
    spec = synth.StackSpec(128, 40, 12, (4.0, 40.0), True, 13100427)
    I0 = synth.make_stack(spec).to(torch.float32).cuda()
    kw = dict(storage=st, fp64_refine=1, out_dtype=torch.float32)
    a1, ra = gd.smooth_z(I0, BETA, **kw)
    b1, rb = gd.smooth_z(I0 * factor, BETA, **kw)
    assert ra["refine_steps"] == rb["refine_steps"]
    assert torch.equal(b1, a1 * factor)
    a2, ra2, _ = gd.screened_poisson_stack(I0, a1, 0.01, storage=st, fp64_refine=1)
    b2, rb2, _ = gd.screened_poisson_stack(I0 * factor, b1, 0.01, storage=st, fp64_refine=1)
    assert ra2["refine_steps"] == rb2["refine_steps"]
    assert torch.equal(b2, a2 * factor)


@pytest.mark.parametrize("shape", [(8, 256, 256), (3, 37, 130), (2, 1, 1)])
def test_sp_stack_plain_fp32(gd, shape):
    say("SP stack f32", shape)
    nz, ny, nx = shape
    rng = np.random.default_rng(4)
    I0 = host(dev(rng.uniform(0, 255, shape)))
    I1 = host(dev(I0 + rng.uniform(-20, 20, (nz, 1, 1)) + rng.standard_normal(shape)))
    # each slice stops once it meets the tolerance; the error bar of 1e-5
    # needs its residual well below 1e-6 on this white-noise input (its
    # smoothest modes amplify the residual about 150 times)
    I2, rep, per = gd.screened_poisson_stack(dev(I0), dev(I1), 0.01, rel_tol=5e-8)
    assert rep["rel_residual"] <= 5e-8
    assert all(p["rel_residual"] <= 5e-8 for p in per)
    assert rel(host(I2), osv.sp_dct(I0, I1, 0.01)) <= 1e-5


def test_sp_batched_uneven_slices(gd):
    """Independent slices of uneven sizes and per-slice alpha in one call."""
    say("SP batch uneven")
    meta = synth.make_slice_batch(nslices=24, lo=16, hi=300, seed=77, dtype=torch.float32)
    I0 = meta["I0"].cuda()
    I1 = meta["I1"].cuda()
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    I2, rep, per = gd.screened_poisson_slices(I0, I1, descs)
    assert rep["rel_residual"] <= 1e-6
    out = host(I2)
    a0 = meta["I0"].double().numpy()
    a1 = meta["I1"].double().numpy()
    for i in range(24):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        s0 = a0[o:o + w * h].reshape(1, h, w)
        s1 = a1[o:o + w * h].reshape(1, h, w)
        alpha = float(np.float32(meta["alpha"][i]))
        ref = osv.sp_dct(s0, s1, alpha)
        # each slice stops once it meets the tolerance; the operator's smallest
        # eigenvalue is alpha, so ||x - x*|| <= ||r|| / alpha bounds the error
        bnorm = np.linalg.norm(og.rhs_sp(s0, s1, alpha))
        bar = max(1e-5, 1.01 * per[i]["rel_residual"] * bnorm / (alpha * np.linalg.norm(ref)))
        assert rel(out[o:o + w * h].reshape(1, h, w), ref) <= bar, i
        assert per[i]["rel_residual"] <= 1e-6


@pytest.mark.parametrize("use_graph", [1, 0])
def test_sp_batch_retires_converged_slices(gd, use_graph):
    """A batch whose slices converge at very different rates (alpha 0.5 next
    to 0.001): each slice leaves the cycle once its FP64 residual meets the
    tolerance, its result stays where it was (whichever of the level's two
    buffers held it) and matches the DCT; the per-slice reports give the
    cycle at which each slice left (fewer for the fast ones); a second call on
    the cached hierarchy returns the same bits (the flags are cleared)."""
    say("SP batch retire", use_graph)
    meta = synth.make_slice_batch(nslices=12, lo=40, hi=260, seed=91, dtype=torch.float32)
    alpha = np.where(np.arange(12) % 3 == 0, 0.5, np.where(np.arange(12) % 3 == 1, 0.02, 0.001))
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], alpha)
    I0, I1 = meta["I0"].cuda(), meta["I1"].cuda()
    I2, rep, per = gd.screened_poisson_slices(I0, I1, descs, use_graph=use_graph)
    assert rep["rel_residual"] <= 1e-6
    res = np.array([p["rel_residual"] for p in per])
    assert (res <= 1e-6).all()
    a0 = meta["I0"].double().numpy()
    a1 = meta["I1"].double().numpy()
    out = host(I2)
    for i in range(12):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        s0, s1 = a0[o:o + w * h].reshape(1, h, w), a1[o:o + w * h].reshape(1, h, w)
        al = float(np.float32(alpha[i]))
        ref = osv.sp_dct(s0, s1, al)
        # error bound from the slice's own residual: ||x - x*|| <= ||r|| / alpha
        bar = max(1e-5, 1.01 * res[i] * np.linalg.norm(og.rhs_sp(s0, s1, al)) / (al * np.linalg.norm(ref)))
        assert rel(out[o:o + w * h].reshape(1, h, w), ref) <= bar, i
    # the fast slices (alpha 0.5) left the batch while the slow ones went on
    cyc = np.array([p["cycles"] for p in per])
    assert cyc.max() == rep["cycles"] and cyc[0::3].max() < cyc.max() and cyc[0::3].mean() < cyc[2::3].mean(), cyc
    J2, rep2, per2 = gd.screened_poisson_slices(I0, I1, descs, use_graph=use_graph)
    assert torch.equal(I2, J2) and rep2["cycles"] == rep["cycles"]
    # a slice's result does not depend on the rest of the batch: the slow
    # slices alone give the same bits
    k = np.arange(2, 12, 3)
    sub = gd.make_slice_descs(meta["offset"][k], meta["w"][k], meta["h"][k], alpha[k])
    K2, _, perk = gd.screened_poisson_slices(I0, I1, sub, use_graph=use_graph, out=torch.zeros_like(I0))
    for j, i in enumerate(k):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        assert torch.equal(K2[o:o + w * h], I2[o:o + w * h]) and perk[j]["cycles"] == per[i]["cycles"]


def test_sp_batched_mixed_bf16(gd):
    say("SP batch mixed bf16")
    meta = synth.make_slice_batch(nslices=8, lo=30, hi=200, seed=78, dtype=torch.bfloat16)
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    I2, rep, per = gd.screened_poisson_slices(meta["I0"].cuda(), meta["I1"].cuda(), descs, storage=gd.BF16,
                                              fp64_refine=1)
    assert rep["rel_residual"] <= 1e-6
    a0 = meta["I0"].double().numpy()
    a1 = meta["I1"].double().numpy()
    out = host(I2)
    for i in range(8):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        ref = osv.sp_dct(a0[o:o + w * h].reshape(1, h, w), a1[o:o + w * h].reshape(1, h, w),
                         float(np.float32(meta["alpha"][i])))
        # output rounded to bf16 (8-bit mantissa)
        assert rel(out[o:o + w * h].reshape(1, h, w), ref) <= 4e-3


@pytest.mark.parametrize("tin,t1,tout,storage,refine", [
    (torch.bfloat16, torch.float64, torch.float64, "bf16", 1),
    (torch.float16, torch.float32, torch.float32, "f16", 1),
    (torch.float32, torch.float64, torch.float64, "f32", 1),
    (torch.float64, torch.float32, torch.float64, "f64", 0),
])
def test_sp_batched_wider_target_and_output(gd, tin, t1, tout, storage, refine):
    """Eq. (2) with I1 wider than I0 (the refined FP64 or FP32 result of the
    first phase) and the result returned in its own type: element-wise
    against the oracle on the same values, at the 1e-6 bar (FP64 iterate:
    refinement, or FP64 storage)."""
    say("SP batch wider I1/out", tin, t1, tout, storage, refine)
    meta = synth.make_slice_batch(nslices=9, lo=20, hi=180, seed=79, dtype=torch.float64)
    I0 = meta["I0"].to(tin).cuda()
    I1 = (meta["I1"] + 0.123456789).to(t1).cuda()  # digits beyond I0's precision
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    st = {"bf16": gd.BF16, "f16": gd.F16, "f32": gd.F32, "f64": gd.F64}[storage]
    # (plain FP64 storage: each slice stops at its tolerance, so the 1e-6 error bar needs a tight one)
    tol = 2e-7 if refine else 1e-9
    I2, rep, per = gd.screened_poisson_slices(I0, I1, descs, storage=st, fp64_refine=refine, rel_tol=tol,
                                              out_dtype=tout)
    assert I2.dtype == tout and rep["rel_residual"] <= tol
    a0, a1, out = host(I0), host(I1), host(I2)
    bar = 1e-6
    for i in range(9):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        ref = osv.sp_dct(a0[o:o + w * h].reshape(1, h, w), a1[o:o + w * h].reshape(1, h, w),
                         float(np.float32(meta["alpha"][i])))
        assert rel(out[o:o + w * h].reshape(1, h, w), ref) <= bar, i
        assert per[i]["rel_residual"] <= tol
        assert per[i]["bytes"] > 0
    assert abs(sum(p["bytes"] for p in per) - rep["bytes"]) <= 1e-6 * rep["bytes"]


def test_sp_new_alphas_reuse_the_hierarchy(gd):
    """A second batch of the same slice sizes with other alphas reuses the
    cached hierarchy (no new device memory) and gives what a fresh hierarchy
    gives, bit for bit."""
    say("SP new alphas, cached hierarchy")
    meta = synth.make_slice_batch(nslices=12, lo=40, hi=260, seed=80, dtype=torch.float32)
    I0, I1 = meta["I0"].cuda(), meta["I1"].cuda()
    w, h, off = meta["w"], meta["h"], meta["offset"]
    d1 = gd.make_slice_descs(off, w, h, meta["alpha"])
    d2 = gd.make_slice_descs(off, w, h, np.random.default_rng(3).uniform(0.001, 0.1, len(w)))
    gd.release_workspace()
    gd.screened_poisson_slices(I0, I1, d1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    cached, _, _ = gd.screened_poisson_slices(I0, I1, d2)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 >= free0 - (1 << 20), (free0, free1)
    gd.release_workspace()
    fresh, _, _ = gd.screened_poisson_slices(I0, I1, d2)
    assert torch.equal(cached, fresh)
    again, _, _ = gd.screened_poisson_slices(I0, I1, d1)  # and back: the first alphas again
    first, _, _ = gd.screened_poisson_slices(I0, I1, d1)
    assert torch.equal(again, first)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_general_system_hierarchy(gd, dt):
    say("general hierarchy", dt)
    shape = (12, 50, 70)
    alpha, beta = 0.05, (1.0, 0.5, 2.0)
    rng = np.random.default_rng(5)
    V = rng.standard_normal(shape)
    G = [rng.standard_normal(shape) for _ in range(3)]
    Vq = host(dev(V, dt))
    Gq = [host(dev(g, dt)) for g in G]
    faces = (Gq[0][:, :, :-1], Gq[1][:, :-1, :], Gq[2][:-1, :, :])
    ref = osv.general_solve(Vq, faces, alpha, beta, method="dct")
    h = gd.Hierarchy(shape, alpha, beta, dt)
    b = h.rhs(dev(V, dt), *[dev(g, dt) for g in G])
    bref = og.rhs_general(Vq, faces, alpha, beta)
    assert np.abs(host(b) - bref).max() <= (1e-13 if dt == torch.float64 else 1e-6) * np.abs(bref).max()
    x = torch.zeros(shape, dtype=dt, device="cuda")
    rr = 1.0
    for _ in range(30):
        rr = h.vcycle(x, b, 1)
        if rr < (1e-10 if dt == torch.float64 else 1e-6):
            break
    assert rr < (1e-10 if dt == torch.float64 else 1e-6)
    # the oracle's own FP64 residual of the returned x
    ores = om.relative_residual(host(x), host(b), alpha, beta)
    assert ores <= (1.01e-10 if dt == torch.float64 else 2e-6)
    # error bar: residual times the condition number (white-noise targets
    # excite every mode; kappa = lambda_max / alpha here)
    kappa = (alpha + 4 * sum(beta)) / alpha
    assert rel(host(x), osv.dct_solve(host(b), alpha, beta)) <= kappa * ores * 1.01
    tol_ref = 1e-8 if dt == torch.float64 else 1e-5
    assert rel(host(b), bref) <= tol_ref
    assert rel(osv.dct_solve(bref, alpha, beta), ref) <= 1e-12
    h.close()


def test_not_converged_status(gd):
    say("not converged")
    I0 = dev(np.random.default_rng(6).uniform(0, 255, (8, 64, 64)))
    I1, rep = gd.smooth_z(I0, BETA, check=False, max_cycles=1, rel_tol=1e-12)
    assert rep["status"] == gd.ERR_NOT_CONVERGED
    assert torch.isfinite(I1).all()


def test_deterministic(gd):
    say("determinism")
    I0 = dev(np.random.default_rng(7).uniform(0, 255, (16, 100, 90)))
    a, _ = gd.smooth_z(I0, BETA)
    b, _ = gd.smooth_z(I0, BETA)
    assert torch.equal(a, b)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_sweep_tiles_identical(gd, storage):
    """Every relaxation tile computes the same values: the AD and SP results
    agree bit for bit across the six tile variants (the two wide ones in the
    quad form only; odd sizes, several z-chunks and ragged tile edges)."""
    import synth

    spec = synth.StackSpec(203, 77, 37, (4.0, 40.0), True, 13100422)
    I0 = synth.make_stack(spec).to(torch.float32).cuda()
    # a fixed number of cycles (the FP32 rounding floor of this stack is near 1e-6)
    kw = dict(rel_tol=1e-9, max_cycles=5, check=False)
    if storage == "f16":
        kw.update(storage=gd.F16, fp64_refine=1)
    outs = []
    for tile in range(6):
        I1, r1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, sweep_tile=tile, **kw)
        I2, r2, _ = gd.screened_poisson_stack(I0, I1, 0.01, sweep_tile=tile, **kw)
        outs.append((I1, I2, r1["cycles"], r2["cycles"]))
    for I1, I2, c1, c2 in outs[1:]:
        assert (c1, c2) == outs[0][2:]
        assert torch.equal(I1, outs[0][0]) and torch.equal(I2, outs[0][1])


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("shape", [(37, 77, 203), (9, 130, 64), (5, 3, 9), (1, 1, 1), (24, 64, 256), (7, 13, 132),
                                   (9, 41, 801)])
def test_sweep_quad_equals_pair(gd, storage, shape):
    """The quad forms of the relaxation and of the finest-level stencil
    passes (four x cells per thread; the stencil passes where the input's
    width is a multiple of four) give the pair forms' values bit for bit:
    AD and SP results after a fixed number of cycles, every tile variant of
    the stack and the slices' row form, on odd sizes, ragged tile edges and
    several z-chunks; 801 x 41 has interior tiles for every tile variant, so
    its stack runs the split launch (interior tiles with uniform weights,
    then the edge tiles).  The residual norms are the same sums taken in
    another order (equal to 1e-12)."""
    import synth

    nz, ny, nx = shape
    say("quad vs pair", storage, shape)
    spec = synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100424)
    I0 = synth.make_stack(spec).to(torch.float32).cuda()
    kw = dict(rel_tol=1e-9, max_cycles=4, check=False, use_graph=0)
    if storage != "f32":
        kw.update(storage=gd.F16 if storage == "f16" else gd.BF16, fp64_refine=1)
    for tile in range(4):
        outs = []
        for quad in (0, 1):
            I1, r1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, sweep_tile=tile, sweep_quad=quad,
                                 **kw)
            I2, r2, _ = gd.screened_poisson_stack(I0, I1, 0.01, sweep_tile=tile, sweep_quad=quad, **kw)
            outs.append((I1, I2, r1["cycles"], r2["cycles"], r1["rel_residual"], r2["rel_residual"]))
        assert outs[0][2:4] == outs[1][2:4], (tile, outs[0][2:], outs[1][2:])
        for a, b in zip(outs[0][4:], outs[1][4:]):
            assert abs(a - b) <= 1e-12 * max(abs(a), 1e-300), (tile, a, b)
        assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1]), tile


def test_wide_tiles_need_the_quad_form(gd):
    """The 256-wide tiles exist in the quad form only: asking for them with
    FP64 storage or with the pair form is refused before any launch."""
    I0 = dev(np.random.default_rng(3).uniform(0, 255, (6, 20, 30)))
    for tile in (4, 5):
        with pytest.raises(RuntimeError, match="sweep_tile 4 and 5"):
            gd.smooth_z(I0, BETA, sweep_tile=tile, storage=gd.F64)
        with pytest.raises(RuntimeError, match="sweep_tile 4 and 5"):
            gd.smooth_z(I0.float(), BETA, sweep_tile=tile, sweep_quad=0)
    J, rep = gd.smooth_z(I0.float(), BETA, sweep_tile=4)
    K, _ = gd.smooth_z(I0.float(), BETA, sweep_tile=0)
    assert torch.equal(J, K)


def test_autotune_choice(gd):
    """A workspace of 2^22 cells is autotuned once; the choice is reported
    and changes nothing in the result."""
    import synth

    spec = synth.StackSpec(256, 256, 64, (4.0, 40.0), True, 13100423)
    I0 = synth.make_stack(spec).to(torch.float32).cuda()
    I1, r1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, rel_tol=1e-6)
    cfg = gd.sweep_config(tuple(I0.shape), torch.float32)
    if os.environ.get("GD_AUTOTUNE", "1") != "0" and "GD_SWEEP_TILE" not in os.environ \
            and "GD_SWEEP_BLOCKS" not in os.environ:
        assert cfg["tuned"] and cfg["ms"] > 0.0
    assert cfg["tile"] in [(64, 8), (128, 8), (64, 16), (128, 16)]
    J1, s1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, rel_tol=1e-6, sweep_tile=0)
    assert r1["cycles"] == s1["cycles"] and torch.equal(I1, J1)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_graph_replays_match_eager(gd, storage):
    """The graph-captured V-cycle pieces give the eager launches' results bit
    for bit, on every replay: several solves in a row (graphs replayed many
    times, eager work and synchronisations in between), a stack and a batch
    of uneven slices."""
    import synth

    spec = synth.StackSpec(96, 80, 24, (4.0, 40.0), True, 13100424)
    I0 = synth.make_stack(spec).to(torch.float32).cuda()
    kw = dict(rel_tol=1e-9, max_cycles=6, check=False)
    if storage == "f16":
        kw.update(storage=gd.F16, fp64_refine=1)
    ref1, rep1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, use_graph=0, **kw)
    ref2, rep2, _ = gd.screened_poisson_stack(I0, ref1, 0.01, use_graph=0, **kw)
    for _ in range(3):
        a1, r1 = gd.smooth_z(I0, (1.0, 1.0, 4.0), out_dtype=torch.float32, use_graph=1, **kw)
        a2, r2, _ = gd.screened_poisson_stack(I0, ref1, 0.01, use_graph=1, **kw)
        torch.cuda.synchronize()
        assert r1["cycles"] == rep1["cycles"] and r2["cycles"] == rep2["cycles"]
        assert torch.equal(a1, ref1) and torch.equal(a2, ref2)


def test_fmg_start(gd):
    """The full-multigrid start reaches the same answer (DCT oracle)."""
    import synth

    spec = synth.StackSpec(96, 64, 16, (4.0, 40.0), True, 13100425)
    I0 = synth.make_stack(spec).to(torch.float64)
    I1, r1 = gd.smooth_z(I0.cuda(), (1.0, 1.0, 4.0), out_dtype=torch.float64, storage=gd.F64, rel_tol=1e-10,
                         fmg=1)
    assert r1["rel_residual"] <= 1e-10
    ref = osv.ad_dct(I0.numpy(), (1.0, 1.0, 4.0))
    assert np.linalg.norm(I1.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-8
