"""Finest level streamed from host memory (Sec. 4.1: each V-cycle is two
streaming passes through the data with a window over the slices).

The streamed cycle relaxes every slab inside a halo wide enough that its own
planes come out as in a cycle over the whole grid, so it must agree with the
in-core V-cycle bit for bit (same kernels, same per-voxel arithmetic).  It is
also checked against the oracle: the FP64 residual of the iterate and the
exact DCT solution of the same system.
"""

import numpy as np
import pytest
import torch

from oracle import grid as og
from oracle import mgsteps as om
from oracle import solvers as osv

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (shape [nz][ny][nx], slab, dtype, alpha, beta, pre/post): several windows
# with a ragged last slab, odd nz, a slab below the halo (raised to it), one
# window holding the whole grid, z kept at level 0 (beta_z small), FP16 and
# FP64 storage, unequal pre- and post-smoothing
CASES = [
    ((40, 33, 47), 8, torch.float32, 0.0, (1.0, 1.0, 4.0), (2, 2)),
    ((37, 16, 64), 10, torch.float32, 0.0, (1.0, 1.0, 4.0), (2, 2)),
    ((45, 20, 24), 4, torch.float32, 0.02, (1.0, 1.0, 1.0), (2, 2)),
    ((18, 20, 20), 64, torch.float32, 0.0, (1.0, 1.0, 4.0), (2, 2)),
    ((48, 24, 30), 12, torch.float32, 0.01, (1.0, 1.0, 0.2), (2, 2)),
    ((64, 24, 40), 16, torch.float16, 0.0, (1.0, 1.0, 4.0), (2, 2)),
    ((33, 18, 22), 8, torch.float64, 0.05, (1.0, 0.5, 2.0), (2, 2)),
    ((52, 16, 20), 10, torch.float32, 0.0, (1.0, 1.0, 4.0), (1, 3)),
    ((72, 12, 18), 8, torch.float32, 0.0, (1.0, 1.0, 16.0), (2, 2)),
    ((66, 10, 14), 6, torch.float32, 0.001, (1.0, 1.0, 16.0), (1, 2)),
]


def expected_streamed_levels(h):
    """The finest level, then every next level with more than an eighth of
    its cells and ny >= 2, leaving at least one level in HBM."""
    n = h.info()
    dims = [h.info(l)[0] for l in range(n)]
    cells = [d[0] * d[1] * d[2] for d in dims]
    k = 1
    while k + 1 < n and dims[k][1] >= 2 and 8 * cells[k] > cells[0]:
        k += 1
    return k


def case_id(c):
    return f"{c[0]}-slab{c[1]}-{str(c[2]).split('.')[-1]}-a{c[3]}-p{c[5]}"


@pytest.mark.parametrize("levels", [1, 8])
@pytest.mark.parametrize("case", CASES, ids=case_id)
def test_streamed_cycles_equal_in_core(gd, case, levels):
    shape, slab, dt, alpha, beta, (pre, post) = case
    say("streamed vs in-core", case_id(case), "levels", levels)
    rng = np.random.default_rng(11)
    b = torch.from_numpy(rng.standard_normal(shape)).to(dt)
    x0 = torch.from_numpy(rng.standard_normal(shape) * 0.5).to(dt)
    hc = gd.Hierarchy(shape, alpha, beta, dt, pre_smooth=pre, post_smooth=post)
    xd, bd = x0.cuda(), b.cuda()
    rr_c = hc.vcycle(xd, bd, 2)
    hs = gd.StreamedHierarchy(shape, alpha, beta, dt, slab, levels, pre_smooth=pre, post_smooth=post)
    assert hs.info() == hc.info()
    xh = torch.empty(shape, dtype=dt, pin_memory=True)
    xh.copy_(x0)
    bh = torch.empty(shape, dtype=dt, pin_memory=True)
    bh.copy_(b)
    rr_s = hs.vcycle(xh, bh, 2)
    assert torch.equal(xh, xd.cpu())
    assert abs(rr_s - rr_c) <= 1e-9 * rr_c
    assert hs.streamed_levels() == min(levels, expected_streamed_levels(hc))
    if beta[2] == 16.0 and levels > 1:
        assert hs.streamed_levels() == 3
    _, planes = hs.device_bytes()
    halo = 2 * max(pre, post) + 2
    want = min(shape[0], max(slab + slab % 2, halo) + 2 * halo)
    assert planes == want
    hs.close()
    hc.close()


def test_pageable_host_memory(gd):
    say("streamed pageable")
    shape = (30, 16, 24)
    rng = np.random.default_rng(12)
    b = torch.from_numpy(rng.standard_normal(shape)).float()
    hc = gd.Hierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32)
    xd = torch.zeros(shape, device="cuda")
    hc.vcycle(xd, b.cuda(), 3)
    hs = gd.StreamedHierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32, 8)
    xh = torch.zeros(shape)
    hs.vcycle(xh, b.clone(), 3)
    assert torch.equal(xh, xd.cpu())


def test_streamed_solve_matches_oracle(gd):
    """FP64 storage, cycles until the residual is at the FP64 level; the
    oracle's own residual of the iterate and the exact DCT solution."""
    say("streamed vs oracle")
    shape = (41, 20, 26)
    alpha, beta = 0.05, (1.0, 0.5, 2.0)
    b = np.random.default_rng(13).standard_normal(shape)
    hs = gd.StreamedHierarchy(shape, alpha, beta, torch.float64, 8, 8)
    assert hs.streamed_levels() == 2
    xh = torch.zeros(shape, dtype=torch.float64, pin_memory=True)
    bh = torch.from_numpy(b).pin_memory()
    rr = 1.0
    for _ in range(30):
        rr = hs.vcycle(xh, bh, 1)
        if rr < 1e-11:
            break
    assert rr < 1e-11
    x = xh.numpy()
    ores = om.relative_residual(x, b, alpha, beta)
    assert ores <= 1.01e-11
    kappa = (alpha + 4 * sum(beta)) / alpha
    assert rel(x, osv.dct_solve(b, alpha, beta)) <= kappa * ores * 1.01


def test_streamed_holds_less_device_memory(gd):
    say("streamed device bytes")
    shape = (1024, 64, 64)
    hc = gd.Hierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32)
    hs = gd.StreamedHierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32, 16)  # levels chosen by HBM use
    bc, _ = hc.device_bytes()
    bs, planes = hs.device_bytes()
    assert planes == 16 + 2 * 6
    # in core: x, x', b of every level (about 3 x 1.57 finest arrays); streamed:
    # levels 2 and below (about 3 x 0.07) and three window buffer sets of
    # levels 0 and 1 (28 planes each), which do not grow with nz
    assert hs.streamed_levels() == 2
    assert bs < 0.25 * bc


def test_in_core_calls_refuse_a_streamed_hierarchy(gd):
    say("streamed refusals")
    shape = (16, 8, 8)
    hs = gd.StreamedHierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32, 8)
    x = torch.zeros(shape, device="cuda")
    with pytest.raises(RuntimeError):
        gd.Hierarchy.vcycle(hs, x, x.clone(), 1)
    with pytest.raises(RuntimeError):
        hs.fcg(x, x.clone())
    with pytest.raises(ValueError):
        hs.vcycle(torch.zeros(4, 8, 8), torch.zeros(4, 8, 8))


def test_automatic_choice_keeps_short_coarse_levels_resident(gd):
    """With stream_levels = 0 a coarser level is streamed only when its
    window buffers take less HBM than the level: not on a short stack."""
    say("streamed automatic levels")
    hs = gd.StreamedHierarchy((40, 33, 47), 0.0, (1.0, 1.0, 4.0), torch.float32, 8)
    assert hs.streamed_levels() == 1
    hs2 = gd.StreamedHierarchy((40, 33, 47), 0.0, (1.0, 1.0, 4.0), torch.float32, 8, 8)
    assert hs2.streamed_levels() == 2
    assert hs.device_bytes()[0] < hs2.device_bytes()[0]


@pytest.mark.parametrize("shape,slab,dt,storage", [
    ((70, 80, 96), 16, torch.float32, "f32"),
    ((41, 33, 57), 8, torch.float16, "f32"),
    ((30, 24, 40), 64, torch.float64, "f64"),
])
def test_smooth_z_streamed_end_to_end(gd, shape, slab, dt, storage):
    """The anisotropic diffusion of a stack held in host memory, every pass
    streamed through HBM (right-hand side, V-cycles, residual, gauge,
    output): the same answer as the in-core gd_smooth_z and the oracle's."""
    import synth

    say("streamed AD end to end", shape, slab, dt, storage)
    nz, ny, nx = shape
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100428)).to(dt)
    beta = (1.0, 1.0, 4.0)
    kw = dict(storage=gd.F64, rel_tol=1e-10) if storage == "f64" else dict(rel_tol=1e-6, check=False)
    out, rep = gd.smooth_z_streamed(I0.pin_memory(), beta, out_dtype=torch.float64, slab=slab, **kw)
    incore, rin = gd.smooth_z(I0.cuda(), beta, out_dtype=torch.float64, **kw)
    say(f"streamed: status {rep['status']} cycles {rep['cycles']} res {rep['rel_residual']:.3g}; "
        f"in core: status {rin['status']} cycles {rin['cycles']} res {rin['rel_residual']:.3g}")
    a0 = I0.double().numpy()
    ref = osv.ad_dct(a0, beta)
    x = out.numpy()
    res = om.relative_residual(x, og_rhs(a0, beta), 0.0, beta)
    assert abs(x.mean() - a0.mean()) <= 1e-9 * max(1.0, abs(a0.mean()))
    if storage == "f64":
        assert rep["status"] == 0 and res <= 1.01e-10
        assert rel(x, ref) <= 1e-7 and rel(x, incore.cpu().numpy()) <= 1e-8
    else:
        # the plain FP32 correction reaches 1e-6 or stops at its rounding floor, as in core
        assert rep["status"] in (0, gd.ERR_NOT_CONVERGED) and res <= max(1.01e-6, 1.01 * rep["rel_residual"])
        assert rel(x, ref) <= 1e-5 and rel(x, incore.cpu().numpy()) <= 2e-6
    assert rep["bytes"] > 0


def og_rhs(I0, beta):
    from oracle import grid as og

    return og.rhs_ad(I0, beta)


def test_smooth_z_streamed_within_a_device_budget(gd):
    """A long stack whose in-core hierarchy needs more device memory than the
    budget given: the streamed solve stays within it and matches the oracle;
    a budget below what the streamed solve needs is refused up front."""
    import synth

    say("streamed AD under a device budget")
    shape = (1024, 64, 64)
    nz, ny, nx = shape
    hc = gd.Hierarchy(shape, 0.0, (1.0, 1.0, 4.0), torch.float32)
    incore_bytes, _ = hc.device_bytes()
    hc.close()
    budget = incore_bytes // 2
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100429)).float().pin_memory()
    out, rep = gd.smooth_z_streamed(I0, (1.0, 1.0, 4.0), out_dtype=torch.float64, slab=16, device_budget=budget,
                                    check=False)
    say(f"in-core hierarchy {incore_bytes} B, budget {budget} B; status {rep['status']}, cycles {rep['cycles']}")
    assert rep["status"] in (0, gd.ERR_NOT_CONVERGED)
    a0 = I0.double().numpy()
    assert rel(out.numpy(), osv.ad_dct(a0, (1.0, 1.0, 4.0))) <= 1e-5
    with pytest.raises(gd.GDError) as ei:
        gd.smooth_z_streamed(I0, (1.0, 1.0, 4.0), slab=16, device_budget=1 << 20)
    assert ei.value.status == gd.ERR_NOMEM


@pytest.mark.parametrize("slab,refine", [(5, 0), (64, 0), (7, 1)])
def test_screened_poisson_streamed(gd, slab, refine):
    """Eq. (2) of a stack held in host memory, in batches of slices through
    HBM: every slice against the DCT oracle and the in-core solve."""
    import synth

    say("streamed SP", slab, refine)
    shape = (23, 48, 72)
    nz, ny, nx = shape
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100430))
    I1 = osv.ad_dct(I0.numpy(), (1.0, 1.0, 4.0))
    kw = dict(storage=gd.F16, fp64_refine=1, rel_tol=1e-7) if refine else dict()
    I0t = (I0.half() if refine else I0.float()).pin_memory()
    I1t = torch.from_numpy(I1).float().pin_memory()
    out, rep, per = gd.screened_poisson_streamed(I0t, I1t, 0.01, out_dtype=torch.float64, slab=slab, **kw)
    assert rep["status"] == 0 and max(p["rel_residual"] for p in per) <= kw.get("rel_tol", 1e-6)
    ref = osv.sp_dct(I0t.double().numpy(), I1t.double().numpy(), 0.01)
    # each slice stops at its own tolerance: ||x - x*|| <= max_i rel_i ||b|| / alpha bounds the error
    worst = max(p["rel_residual"] for p in per)
    b = np.linalg.norm(og.rhs_sp(I0t.double().numpy(), I1t.double().numpy(), 0.01))
    bar = max(1e-6 if refine else 1e-5, 1.01 * worst * b / (0.01 * np.linalg.norm(ref)))
    assert rel(out.numpy(), ref) <= bar
    incore, _, _ = gd.screened_poisson_stack(I0t.cuda(), I1t.cuda(), 0.01, out_dtype=torch.float64, **kw)
    assert rel(out.numpy(), incore.cpu().numpy()) <= (1e-6 if refine else 2e-6)
