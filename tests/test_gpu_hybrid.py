"""The Hybrid and Linear discretisations (Sec. 4.2) on the GPU.

One V-cycle of the library (7-point red-black relaxation on the finest
level, 8-colour Gauss-Seidel on the Galerkin levels, B-spline transfers) is
compared element by element with the same cycle composed from the oracle's
step functions on the library's own level sizes: 1e-11 relative in FP64,
1e-5 in FP32.  Whole solves must reach the same answer as the "Constant"
solver: the DCT oracle's solution of the finest-level system.  The Linear
scheme (B-spline finite elements on every level, 8-colour Gauss-Seidel
everywhere) is checked the same way against its own oracle.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og
from oracle import hybrid, linear, mgsteps, solvers

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def oracle_vcycle(x, b, sizes, alpha, w, pre, post, fem=False):
    """One V-cycle composed from oracle steps on the level sizes `sizes`
    ([nz][ny][nx] per level, finest first).  fem: the Linear scheme (level 0
    is the B-spline operator, relaxed by 8-colour GS like the others)."""
    last = len(sizes) - 1
    halv = [[sizes[l + 1][::-1][a] != sizes[l][::-1][a] for l in range(last)] for a in range(3)]  # per axis x, y, z
    n0 = sizes[0][::-1]
    mats = [linear.tables(sizes[0]) if fem else [(np.eye(n), hybrid.laplace_1d(n)) for n in n0]]
    for l in range(last):
        nxt = []
        for a in range(3):
            Pa = hybrid.prolong_1d(mats[l][a][0].shape[0], halv[a][l])
            nxt.append((Pa.T @ mats[l][a][0] @ Pa, Pa.T @ mats[l][a][1] @ Pa))
        mats.append(nxt)
    P = [hybrid.transfer_mats(sizes[l], [halv[a][l] for a in range(3)]) for l in range(last)]
    table = (lambda l: True) if fem else (lambda l: l > 0)

    def smooth(l, x, b, n):
        for _ in range(n):
            x = hybrid.gs8_sweep(x, b, mats[l], alpha, w) if table(l) else mgsteps.rb_sweep(x, b, alpha, w)
        return x

    def full(l, x, b):
        if l == last:
            return smooth(l, x, b, 1)
        x = smooth(l, x, b, pre)
        r = b - hybrid.apply(x, mats[l], alpha, w) if table(l) else mgsteps.residual(x, b, alpha, w)
        bc = hybrid.restrict(r, P[l])
        xc = full(l + 1, np.zeros(bc.shape), bc)
        return smooth(l, x + hybrid.prolong(xc, P[l]), b, post)

    return full(0, og.as3d(x), og.as3d(b))


SHAPES = [(9, 17, 30), (8, 8, 8), (5, 33, 20), (1, 12, 40), (16, 3, 5), (2, 2, 2), (1, 1, 1), (12, 1, 7)]
SYSTEMS = [(0.0, (1.0, 1.0, 4.0)), (0.01, (1.0, 1.0, 0.0)), (0.001, (1.0, 1.0, 0.1))]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("alpha,w", SYSTEMS)
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_one_vcycle_matches_oracle_steps(gd, shape, alpha, w, dt):
    say("hybrid vcycle", shape, alpha, w, dt)
    rng = np.random.default_rng(7)
    x0, b = rng.standard_normal(shape), rng.standard_normal(shape)
    if alpha == 0.0:
        b -= b.mean()
    xq = torch.from_numpy(x0).to(dt).double().numpy()
    bq = torch.from_numpy(b).to(dt).double().numpy()
    h = gd.Hierarchy(shape, alpha, w, dt, discretization=1, pre_smooth=1, post_smooth=2)
    sizes = [h.info(l)[0] for l in range(h.info())]
    x = torch.from_numpy(xq).to(dt).cuda()
    h.vcycle(x, torch.from_numpy(bq).to(dt).cuda(), 1)
    h.close()
    ref = oracle_vcycle(xq, bq, sizes, alpha, w, 1, 2)
    tol = 1e-11 if dt == torch.float64 else 1e-5
    assert np.abs(x.double().cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(16, 64, 64), (7, 45, 99), (32, 128, 96)])
def test_ad_solve_hybrid_same_answer(gd, shape):
    say("hybrid AD", shape)
    nz, ny, nx = shape
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100422)).numpy()
    ref = solvers.ad_dct(I0, (1.0, 1.0, 4.0))
    out, rep = gd.smooth_z(torch.from_numpy(I0).cuda(), (1.0, 1.0, 4.0), storage=gd.F64, rel_tol=1e-10,
                           discretization=1)
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-10
    assert np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    # the same system with the Constant transfers, for the cycle counts
    _, rep0 = gd.smooth_z(torch.from_numpy(I0).cuda(), (1.0, 1.0, 4.0), storage=gd.F64, rel_tol=1e-10)
    say("cycles hybrid", rep["cycles"], "constant", rep0["cycles"])


def test_ad_mixed_fp16_hybrid(gd):
    say("hybrid AD f16 + FP64 refinement")
    I0t = synth.make_stack(synth.StackSpec(96, 80, 24, (4.0, 40.0), True, 13100423)).to(torch.float16)
    I0 = I0t.double().numpy()
    out, rep = gd.smooth_z(I0t.cuda(), (1.0, 1.0, 4.0), out_dtype=torch.float64, storage=gd.F16, fp64_refine=1,
                           discretization=1)
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-6
    ref = solvers.ad_dct(I0, (1.0, 1.0, 4.0))
    assert np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-5


def test_npr_hybrid(gd):
    say("hybrid NPR")
    from oracle import npr
    I0 = synth.make_video(synth.VideoSpec(80, 48, 10)).numpy()
    ref = npr.npr_filter(I0)
    out, rep = gd.npr_filter(torch.from_numpy(I0).cuda(), storage=gd.F64, rel_tol=1e-11, discretization=1)
    assert rep["status"] == 0
    assert np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8


def _sp_inputs(shape, seed):
    nz, ny, nx = shape
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, seed)).numpy()
    rng = np.random.default_rng(seed)
    I1 = I0 * rng.uniform(0.8, 1.2, (nz, 1, 1)) + rng.uniform(-20, 20, (nz, 1, 1))
    return I0, I1


@pytest.mark.parametrize("shape", [(5, 33, 47), (1, 64, 96), (3, 1, 40)])
def test_sp_hybrid_stack(gd, shape):
    """Eq. (2) with the Hybrid scheme (7-point finest level, B-spline
    transfers, Galerkin coarse levels): the 7-point answer, so the DCT
    oracle's, slice by slice."""
    say("hybrid SP stack", shape)
    I0, I1 = _sp_inputs(shape, 13100426)
    out, rep, per = gd.screened_poisson_stack(torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), 0.01,
                                              storage=gd.F64, rel_tol=1e-10, discretization=1)
    assert rep["status"] == 0 and max(p["rel_residual"] for p in per) <= 1e-10
    ref = solvers.sp_dct(I0, I1, 0.01)
    assert np.linalg.norm(out.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8


def test_sp_hybrid_stack_as_one_grid(gd):
    """Hybrid SP of equal slices laid out as a stack runs as one 3-D grid
    with no coupling across slices (w_z = 0, z never coarsened) and per-slice
    FP64 norms: every slice meets the tolerance against its own right-hand
    side and matches the DCT within the bound its residual gives (the
    operator's smallest eigenvalue is alpha); the same slices passed out of
    stack order take the slice-by-slice route and agree with it to that
    bound."""
    say("hybrid SP stack as one grid")
    nz, ny, nx = 6, 40, 72
    # I1 a few percent and a few grey levels off I0: the exact answer rounded
    # to FP32 leaves relative residuals of 1.3e-7 .. 3.4e-7 per slice, so
    # FP32 storage can meet 1e-6 (offsets of +-20 put that floor at 1.2e-6)
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100431)).numpy()
    rng = np.random.default_rng(13100431)
    I1 = I0 * rng.uniform(0.95, 1.05, (nz, 1, 1)) + rng.uniform(-2, 2, (nz, 1, 1))
    x0, x1 = torch.from_numpy(I0).float().cuda(), torch.from_numpy(I1).float().cuda()
    out, rep, per = gd.screened_poisson_stack(x0, x1, 0.01, discretization=1, out_dtype=torch.float64)
    q0, q1 = x0.double().cpu().numpy(), x1.double().cpu().numpy()
    ref = solvers.sp_dct(q0, q1, 0.01)
    got = out.cpu().numpy()
    for z in range(nz):
        assert per[z]["rel_residual"] <= 1e-6
        b = np.linalg.norm(og.rhs_sp(q0[z:z + 1], q1[z:z + 1], 0.01))
        bar = max(1e-5, 1.01 * per[z]["rel_residual"] * b / (0.01 * np.linalg.norm(ref[z])))
        assert np.linalg.norm(got[z] - ref[z]) / np.linalg.norm(ref[z]) <= bar, z
    # out of stack order: the slice-by-slice route
    order = np.arange(nz)[::-1]
    descs = gd.make_slice_descs(order * nx * ny, nx, ny, 0.01)
    out2, rep2, per2 = gd.screened_poisson_slices(x0.reshape(-1), x1.reshape(-1), descs, discretization=1,
                                                  out_dtype=torch.float64)
    got2 = out2.cpu().numpy().reshape(nz, ny, nx)
    for z in range(nz):
        assert per2[z]["rel_residual"] <= 1e-6
        assert np.linalg.norm(got2[z] - ref[z]) / np.linalg.norm(ref[z]) <= 1e-4, z


def test_sp_hybrid_uneven_batch_fp32_and_mixed(gd):
    """A batch of uneven slices with per-slice alpha, Hybrid: plain FP32 to
    1e-6 (error bar 1e-5) and FP16 storage with FP64 refinement (1e-6)."""
    say("hybrid SP batch")
    meta = synth.make_slice_batch(nslices=7, lo=20, hi=150, seed=81, dtype=torch.float64)
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    a0, a1 = meta["I0"].numpy(), meta["I1"].numpy()
    for kw, dt, bar in ((dict(), torch.float32, 1e-5),
                        (dict(storage=gd.F16, fp64_refine=1, rel_tol=5e-8), torch.float16, 1e-6)):
        I0 = meta["I0"].to(dt)
        I1 = meta["I1"].to(torch.float32)
        out, rep, per = gd.screened_poisson_slices(I0.cuda(), I1.cuda(), descs, discretization=1,
                                                   out_dtype=torch.float64, **kw)
        assert rep["status"] == 0, rep
        q0, q1, got = I0.double().numpy(), I1.double().numpy(), out.cpu().numpy()
        for i in range(7):
            o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
            ref = solvers.sp_dct(q0[o:o + w * h].reshape(1, h, w), q1[o:o + w * h].reshape(1, h, w),
                                 float(np.float32(meta["alpha"][i])))
            err = np.linalg.norm(got[o:o + w * h].reshape(1, h, w) - ref) / np.linalg.norm(ref)
            assert err <= bar, (i, err, kw)
            assert per[i]["rel_residual"] <= kw.get("rel_tol", 1e-6)


@pytest.mark.parametrize("disc", [1, 2])
@pytest.mark.parametrize("storage,dt", [("F32", torch.float32), ("F64", torch.float64), ("F16", torch.float16)])
@pytest.mark.parametrize("use_graph", [1, 0])
def test_table_relaxation_by_plane_parity_equals_colour_launches(gd, monkeypatch, disc, storage, dt, use_graph):
    """The table levels' 8-colour Gauss-Seidel sweep as two launches (even
    planes, then odd planes; each block's four in-plane colours on a tile
    widened by 3, 2, 1, 0 samples in LDS) gives the eight in-place colour
    launches' values bit for bit: whole solves, several 64 x 16 tiles with
    ragged edges, odd and single-plane grids, with and without graph replay
    (GD_HYB_COLOURS forces one form; by default the size of a level picks it)."""
    if disc == 2 and storage == "F16":
        pytest.skip("the Linear discretisation has no FP64 refinement")
    for shape in [(9, 40, 150), (2, 37, 70), (6, 1, 45), (13, 17, 66), (1, 37, 70)]:
        say("table relaxation by plane parity", disc, storage, use_graph, shape)
        rng = np.random.default_rng(1310)
        I0 = torch.from_numpy(rng.uniform(0, 60, shape)).to(dt).cuda()
        kw = dict(storage=getattr(gd, storage), discretization=disc, use_graph=use_graph, rel_tol=1e-6, check=False,
                  out_dtype=torch.float64)
        if storage == "F16":
            kw["fp64_refine"] = 1
        if shape[0] > 1:  # (one plane: the AD right-hand side is zero, no cycle runs)
            monkeypatch.setenv("GD_HYB_COLOURS", "1")
            ref, rep_ref = gd.smooth_z(I0, (1.0, 1.0, 4.0), **kw)
            monkeypatch.setenv("GD_HYB_COLOURS", "2")
            got, rep = gd.smooth_z(I0, (1.0, 1.0, 4.0), **kw)
            assert rep["cycles"] == rep_ref["cycles"] and rep["cycles"] > 0
            assert torch.equal(got.view(torch.int64), ref.view(torch.int64)), shape
        # two V-cycles of the hierarchy call on a random system
        if disc == 1 or storage != "F16":
            x0 = torch.from_numpy(rng.standard_normal(shape)).to(dt)
            b = torch.from_numpy(rng.standard_normal(shape)).to(dt)
            outs = []
            for env in ("1", "2"):
                monkeypatch.setenv("GD_HYB_COLOURS", env)
                h = gd.Hierarchy(shape, 0.01, (1.0, 1.0, 0.5), dt, discretization=disc, pre_smooth=2, post_smooth=3)
                x = x0.clone().cuda()
                h.vcycle(x, b.cuda(), 2)
                h.close()
                outs.append(x.cpu())
            assert torch.equal(outs[0].view(torch.int16 if dt == torch.float16 else torch.int32 if dt == torch.float32
                                            else torch.int64),
                               outs[1].view(torch.int16 if dt == torch.float16 else torch.int32 if dt == torch.float32
                                            else torch.int64)), shape


@pytest.mark.parametrize("disc,shape", [(2, (16, 256, 256)), (1, (32, 256, 300))])
def test_table_relaxation_default_choice(gd, monkeypatch, disc, shape):
    """Levels of at least 8 rows and 2^20 samples take the plane-parity form
    by default (Linear: level 0 here; Hybrid: the z-halved level 1), the rest
    the colour launches: the mix gives the colour launches' answer bit for
    bit."""
    say("table relaxation default choice", disc, shape)
    rng = np.random.default_rng(1311)
    I0 = torch.from_numpy(rng.uniform(0, 60, shape)).float().cuda()
    kw = dict(discretization=disc, rel_tol=1e-6, check=False, out_dtype=torch.float64)
    monkeypatch.setenv("GD_HYB_COLOURS", "1")
    ref, rep_ref = gd.smooth_z(I0, (1.0, 1.0, 4.0), **kw)
    monkeypatch.setenv("GD_HYB_COLOURS", "0")
    got, rep = gd.smooth_z(I0, (1.0, 1.0, 4.0), **kw)
    assert rep["cycles"] == rep_ref["cycles"] and rep["cycles"] > 0
    assert torch.equal(got.view(torch.int64), ref.view(torch.int64))


@pytest.mark.parametrize("shape", [(9, 17, 30), (5, 8, 8), (1, 12, 40), (16, 3, 5), (2, 2, 2), (1, 1, 1)])
@pytest.mark.parametrize("alpha,w", SYSTEMS)
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_linear_one_vcycle_matches_oracle_steps(gd, shape, alpha, w, dt):
    say("linear vcycle", shape, alpha, w, dt)
    rng = np.random.default_rng(8)
    x0, b = rng.standard_normal(shape), rng.standard_normal(shape)
    if alpha == 0.0:
        b -= b.mean()
    xq = torch.from_numpy(x0).to(dt).double().numpy()
    bq = torch.from_numpy(b).to(dt).double().numpy()
    h = gd.Hierarchy(shape, alpha, w, dt, discretization=2, pre_smooth=1, post_smooth=2)
    sizes = [h.info(l)[0] for l in range(h.info())]
    x = torch.from_numpy(xq).to(dt).cuda()
    h.vcycle(x, torch.from_numpy(bq).to(dt).cuda(), 1)
    h.close()
    ref = oracle_vcycle(xq, bq, sizes, alpha, w, 1, 2, fem=True)
    tol = 1e-11 if dt == torch.float64 else 1e-5
    assert np.abs(x.double().cpu().numpy() - ref).max() <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(8, 32, 40), (5, 17, 23)])
def test_linear_ad_solve_fp64(gd, shape):
    say("linear AD f64", shape)
    nz, ny, nx = shape
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100424)).numpy()
    ref = linear.ad_solve(I0, (1.0, 1.0, 4.0), method="cg")
    out, rep = gd.smooth_z(torch.from_numpy(I0).cuda(), (1.0, 1.0, 4.0), storage=gd.F64, rel_tol=1e-10,
                           discretization=2)
    x = out.cpu().numpy()
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-10, rep
    assert linear.relative_residual(x, I0, (1.0, 1.0, 4.0)) <= 1.01e-10
    assert abs(x.mean() - I0.mean()) <= 1e-9 * abs(I0.mean())
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-8


def test_linear_ad_solve_fp32(gd):
    say("linear AD f32")
    I0 = synth.make_stack(synth.StackSpec(96, 64, 12, (4.0, 40.0), True, 13100425)).float().double().numpy()
    beta = (1.0, 1.0, 4.0)
    ref = linear.ad_solve(I0, beta, method="cg")
    E = (ref - I0).astype(np.float32).astype(np.float64)
    tol = max(1e-6, 3.0 * linear.relative_residual(I0 + E, I0, beta))
    out, rep = gd.smooth_z(torch.from_numpy(I0).float().cuda(), beta, out_dtype=torch.float64, rel_tol=tol,
                           discretization=2)
    x = out.cpu().numpy()
    assert rep["status"] == 0 and linear.relative_residual(x, I0, beta) <= 1.01 * tol
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-5
    # and it is a different answer from the 7-point one
    assert np.linalg.norm(ref - solvers.ad_dct(I0, beta)) > 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape", [(4, 24, 37), (1, 50, 64), (2, 1, 30)])
def test_linear_sp_fp64(gd, shape):
    """Eq. (2) with the Linear scheme against its own oracle (per-slice CG),
    FP64: every slice's residual of the Linear system and the answer."""
    say("linear SP f64", shape)
    I0, I1 = _sp_inputs(shape, 13100427)
    out, rep, per = gd.screened_poisson_stack(torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), 0.01,
                                              storage=gd.F64, rel_tol=1e-10, discretization=2)
    x = out.cpu().numpy()
    assert rep["status"] == 0
    res = linear.sp_relative_residuals(x, I0, I1, 0.01)
    say("oracle residuals", res, "reported", [p["rel_residual"] for p in per])
    # the library measures the residual of the correction system in its own
    # (FP64) arithmetic; the oracle's of I0 + E agrees to a few 1e-11
    assert res.max() <= 2e-10, res
    ref = linear.sp_solve(I0, I1, 0.01, method="cg")
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-8
    # a different answer from the 7-point one
    assert np.linalg.norm(ref - solvers.sp_dct(I0, I1, 0.01)) > 1e-5 * np.linalg.norm(ref)


def test_linear_sp_stack_as_one_grid(gd):
    """Linear SP of equal slices laid out as a stack runs as one 3-D grid
    (M_z = Id, w_z = 0, z never coarsened) with per-slice norms: by the
    oracle's own residual of the Linear system every slice meets the
    tolerance (FP32 storage; the library's residual is that of the FP32-stored
    correction system, so the oracle's may exceed it by FP32 rounding).  The
    same slices out of stack order take the slice-by-slice route: the same bar,
    and the two answers agree (loosely: at alpha = 0.01 the operator's
    smallest eigenvalue, alpha times the mass matrices', makes the residual a
    weak bound on the error)."""
    say("linear SP stack as one grid")
    nz, ny, nx = 6, 40, 72
    I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100432)).numpy()
    rng = np.random.default_rng(13100432)
    I1 = I0 * rng.uniform(0.95, 1.05, (nz, 1, 1)) + rng.uniform(-2, 2, (nz, 1, 1))
    x0, x1 = torch.from_numpy(I0).float().cuda(), torch.from_numpy(I1).float().cuda()
    q0, q1 = x0.double().cpu().numpy(), x1.double().cpu().numpy()
    out, rep, per = gd.screened_poisson_stack(x0, x1, 0.01, discretization=2, out_dtype=torch.float64)
    got = out.cpu().numpy()
    assert rep["status"] == 0 and max(p["rel_residual"] for p in per) <= 1e-6
    res = linear.sp_relative_residuals(got, q0, q1, 0.01)
    assert res.max() <= 2e-6, res
    order = np.arange(nz)[::-1]
    descs = gd.make_slice_descs(order * nx * ny, nx, ny, 0.01)
    out2, rep2, per2 = gd.screened_poisson_slices(x0.reshape(-1), x1.reshape(-1), descs, discretization=2,
                                                  out_dtype=torch.float64)
    got2 = out2.cpu().numpy().reshape(nz, ny, nx)
    assert max(p["rel_residual"] for p in per2) <= 1e-6
    assert linear.sp_relative_residuals(got2, q0, q1, 0.01).max() <= 2e-6
    for z in range(nz):
        assert np.linalg.norm(got2[z] - got[z]) / np.linalg.norm(got[z]) <= 1e-4, z


def test_linear_sp_fp32_uneven(gd):
    say("linear SP f32 batch")
    meta = synth.make_slice_batch(nslices=5, lo=16, hi=120, seed=82, dtype=torch.float32)
    descs = gd.make_slice_descs(meta["offset"], meta["w"], meta["h"], meta["alpha"])
    out, rep, per = gd.screened_poisson_slices(meta["I0"].cuda(), meta["I1"].cuda(), descs, discretization=2,
                                               out_dtype=torch.float64, check=False)
    a0, a1, got = meta["I0"].double().numpy(), meta["I1"].double().numpy(), out.cpu().numpy()
    for i in range(5):
        o, w, h = meta["offset"][i], meta["w"][i], meta["h"][i]
        s0, s1 = a0[o:o + w * h].reshape(1, h, w), a1[o:o + w * h].reshape(1, h, w)
        al = float(np.float32(meta["alpha"][i]))
        x = got[o:o + w * h].reshape(1, h, w)
        # a plain FP32 correction stops at its rounding floor when that is above 1e-6
        floor = linear.sp_relative_residuals(s0 + (linear.sp_solve(s0, s1, al) - s0).astype(np.float32), s0, s1,
                                             al)[0]
        assert linear.sp_relative_residuals(x, s0, s1, al)[0] <= max(1.01e-6, 3.0 * floor)
        ref = linear.sp_solve(s0, s1, al)
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-5, i


def test_linear_unsupported_cases(gd):
    I0 = torch.rand(3, 16, 32, device="cuda") * 100
    with pytest.raises(gd.GDError) as ei:
        gd.screened_poisson_stack(I0.half(), I0.float(), 0.01, storage=gd.F16, fp64_refine=1, discretization=2)
    assert ei.value.status == gd.ERR_UNSUPPORTED
    with pytest.raises(gd.GDError) as ei:
        gd.npr_filter(I0, discretization=2)
    assert ei.value.status == gd.ERR_UNSUPPORTED
    with pytest.raises(gd.GDError) as ei:
        gd.smooth_z(I0, (1.0, 1.0, 4.0), storage=gd.F16, fp64_refine=1, discretization=2)
    assert ei.value.status == gd.ERR_UNSUPPORTED
