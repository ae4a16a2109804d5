"""Spectral (DCT) solver on the GPU against the FP64 oracle.

The library's FFT-based DCT path and the oracle's scipy DCT solve the same
constant-coefficient Neumann systems exactly, so they agree to FP64
rounding (1e-12 relative); the multigrid solve of the same system agrees
to its tolerance.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import solvers

pytestmark = pytest.mark.gpu

# long y-lines (ny >= 512 with nx > 1) take the transposed path, with and
# without a z axis
SHAPES = [(8, 16, 32), (1, 1, 64), (4, 1, 8), (16, 64, 64), (2, 2, 2), (1, 1, 1), (32, 8, 4), (1, 4096, 2),
          (2, 1, 4096), (4, 512, 64), (1, 512, 1024), (2, 1024, 1)]
SYSTEMS = [(0.0, (1.0, 1.0, 4.0)), (0.01, (1.0, 1.0, 0.0)), (0.3, (2.0, 0.5, 1.0)), (0.001, (1.0, 1.0, 0.1))]


def say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("alpha,beta", SYSTEMS)
def test_dct_solve_matches_oracle(gd, shape, alpha, beta):
    say("dct solve", shape, alpha, beta)
    b = np.random.default_rng(5).standard_normal(shape)
    if alpha == 0.0:
        b -= b.mean()
    ref = solvers.dct_solve(b, alpha, beta)
    x, st = gd.dct_solve(torch.from_numpy(b).cuda(), alpha, beta)
    x = x.cpu().numpy()
    assert st == 0
    assert np.abs(x - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("shape", [(16, 64, 64), (8, 128, 32), (1, 256, 256), (4, 512, 32), (1, 1024, 64)])
@pytest.mark.parametrize("tin", [torch.float32, torch.float16])
def test_dct_ad_closed_form(gd, shape, tin):
    say("dct AD", shape, tin)
    nz, ny, nx = shape
    I0t = synth.make_stack(synth.StackSpec(nx, ny, nz, (4.0, 40.0), True, 13100426)).to(tin)
    I0 = I0t.double().numpy()
    ref = solvers.ad_dct(I0, (1.0, 1.0, 4.0))
    out, st = gd.dct_smooth_z(I0t.cuda(), (1.0, 1.0, 4.0), out_dtype=torch.float64)
    assert st == 0
    x = out.cpu().numpy()
    assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()


def test_dct_agrees_with_multigrid(gd):
    say("dct vs MG")
    I0 = synth.make_stack(synth.StackSpec(64, 64, 16, (4.0, 40.0), True, 13100427)).cuda()
    mg, rep = gd.smooth_z(I0, (1.0, 1.0, 4.0), storage=gd.F64, rel_tol=1e-11)
    sp, st = gd.dct_smooth_z(I0, (1.0, 1.0, 4.0))
    assert rep["status"] == 0 and st == 0
    assert (torch.linalg.norm(mg - sp) / torch.linalg.norm(sp)).item() <= 1e-8


def test_dct_sizes_must_be_powers_of_two(gd):
    b = torch.zeros(3, 8, 8, device="cuda", dtype=torch.float64)
    _, st = gd.dct_solve(b, 0.1, (1.0, 1.0, 1.0), check=False)
    assert st == gd.ERR_UNSUPPORTED
    b = torch.zeros(1, 8, 8192, device="cuda", dtype=torch.float32)
    _, st = gd.dct_solve(b, 0.1, (1.0, 1.0, 1.0), check=False)
    assert st == gd.ERR_UNSUPPORTED
