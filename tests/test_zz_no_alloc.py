"""The no-allocation entry point gd_smooth_z_noalloc (its multigrid
hierarchy in the library's static scratch array) called through the C ABI
against gd_smooth_z on the same inputs: the same iterate bit for bit, two
calls in a row with the second on a smaller stack, no device memory taken,
and the FP64 oracle's answer to the plain FP32 bar."""

import numpy as np
import pytest
import torch

import synth
from oracle import solvers as osv

pytestmark = pytest.mark.gpu
BETA = (1.0, 1.0, 4.0)


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("storage", ["f32", "f64", "f16"])
def test_noalloc_matches_smooth_z_twice(gd, storage):
    kw = dict(rel_tol=1e-6, check=False)
    # FP64 iterates (refinement, FP64 storage) are solved far enough below
    # 1e-6 that the error bar of 1e-6 against the oracle holds
    if storage == "f16":
        kw.update(storage=gd.F16, fp64_refine=1, rel_tol=1e-8)
    if storage == "f64":
        kw.update(storage=gd.F64, rel_tol=1e-9)
    tin = {"f32": torch.float32, "f64": torch.float64, "f16": torch.float16}[storage]
    # set-up: the first call on a device loads the scratch array (the
    # library's device global, once per process); later calls take nothing
    tiny = torch.zeros((2, 4, 4), device="cuda", dtype=tin)
    gd.smooth_z_noalloc(tiny, torch.empty((2, 4, 4), device="cuda", dtype=torch.float64), BETA, **kw)
    # the larger stack first, then a smaller one: the scratch keeps the
    # first call's contents, which the second must not depend on
    for shape, seed in (((36, 150, 130), 11), ((20, 70, 97), 12)):
        nz, ny, nx = shape
        say("noalloc", storage, shape)
        I0 = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, seed), device="cuda", dtype=tin)
        ref, rref = gd.smooth_z(I0, BETA, out_dtype=torch.float64, **kw)
        out = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        rep = gd.smooth_z_noalloc(I0, out, BETA, **kw)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        say(f"status {rep['status']} / {rref['status']}, cycles {rep['cycles']} / {rref['cycles']}, "
            f"residual {rep['rel_residual']:.3g}, free memory change {free1 - free0} B")
        # the same status (a plain FP32 solve of a small smooth stack may stop
        # at its rounding floor above 1e-6: then both report it), cycles and
        # iterate, bit for bit; no device memory taken
        assert rep["status"] == rref["status"]
        assert rep["cycles"] == rref["cycles"] and rep["refine_steps"] == rref["refine_steps"]
        assert torch.equal(out, ref)
        assert free1 >= free0 - (4 << 20)
        a0 = I0.double().cpu().numpy()
        err = rel(out.cpu().numpy(), osv.ad_dct(a0, BETA))
        say(f"error vs the FP64 oracle {err:.2e}")
        if storage == "f32":
            assert rep["status"] in (0, gd.ERR_NOT_CONVERGED) and err <= 1e-5
        else:
            assert rep["status"] == 0 and err <= 1e-6


def test_noalloc_refuses_a_stack_beyond_its_scratch(gd):
    cap = gd.noalloc_scratch_bytes()
    assert cap == 128 << 20
    I0 = torch.zeros((1, 1, 1), device="cuda")
    out = torch.zeros((1, 1, 1), device="cuda")
    lib = gd.load()
    import ctypes

    # 512 x 512 x 256 FP32 (about 1.3 GB of hierarchy) is refused before any
    # device work: the pointers are never read
    st = lib.gd_smooth_z_noalloc(ctypes.c_void_p(I0.data_ptr()), gd.F32, ctypes.c_void_p(out.data_ptr()), gd.F32,
                                 512, 512, 256, 1.0, 1.0, 4.0, None, None, None)
    assert st == gd.ERR_UNSUPPORTED
    assert b"bytes of scratch" in lib.gd_last_error()
