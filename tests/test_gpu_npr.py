"""Gradient-modulation filter of Sec. 6 on the GPU against the FP64 oracle.

The oracle builds the modulated gradient field and solves the filter's
normal equations exactly (DCT); the HIP path builds the correction-form
right-hand side in one kernel and runs V-cycles.  Bars: the canonical
relative residual of the output, recomputed by the oracle, within 1 % of the
tolerance asked for (with FP32 storage the tolerance is raised to three times
the residual of the exact answer with its correction I1 - I0 rounded to
FP32, the floor of any FP32 iterate); the relative L2 error within
max(1e-5, 1.01 ||r|| / (alpha ||x*||)) for FP32 and 1e-8 for FP64 storage.
The second term is the exact bound the residual gives: the operator's
smallest eigenvalue is alpha (the constant field; the Laplacians are PSD),
so ||x - x*|| <= ||r|| / alpha, which at the paper's alpha = 0.001 exceeds
1e-5 of ||x*|| for a 1e-6 residual.
"""

import numpy as np
import pytest
import torch

import synth
from oracle import grid as og
from oracle import npr

pytestmark = pytest.mark.gpu

PAPER = dict(alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.25, sigma=5.0)
OTHER = dict(alpha=0.05, beta=(1.0, 0.5, 2.0), lam=0.8, sigma=12.0)


def say(*a):
    print("[case]", *a, flush=True)


def video(shape, seed=13100416):
    nt, ny, nx = shape
    return synth.make_video(synth.VideoSpec(nx, ny, nt, seed))


def canon_residual(x, I0, p):
    b = npr.rhs(I0, p["alpha"], p["beta"], p["lam"], p["sigma"])
    r = b - og.apply_A(x, p["alpha"], p["beta"])
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def err_bar(x, I0, ref, p):
    r = npr.rhs(I0, p["alpha"], p["beta"], p["lam"], p["sigma"]) - og.apply_A(x, p["alpha"], p["beta"])
    return max(1e-5, 1.01 * np.linalg.norm(r) / (p["alpha"] * np.linalg.norm(ref)))


def fp32_floor(I0, ref, p):
    E = (ref - I0).astype(np.float32).astype(np.float64)
    return canon_residual(I0 + E, I0, p)


@pytest.mark.parametrize("shape", [(12, 40, 70), (7, 45, 99), (1, 33, 200), (5, 1, 64), (3, 2, 1), (1, 1, 1),
                                   (24, 96, 160)])
@pytest.mark.parametrize("params", ["paper", "other"])
def test_npr_fp32_matches_oracle(gd, shape, params):
    p = PAPER if params == "paper" else OTHER
    say("npr f32", shape, params)
    I0 = video(shape).float().double().numpy()  # the FP32 input both sides see
    ref = npr.npr_filter(I0, p["alpha"], p["beta"], p["lam"], p["sigma"])
    tol = max(1e-6, 3.0 * fp32_floor(I0, ref, p))
    out, rep = gd.npr_filter(torch.from_numpy(I0).float().cuda(), p["alpha"], p["beta"], p["lam"], p["sigma"],
                             out_dtype=torch.float64, rel_tol=tol)
    x = out.cpu().numpy()
    assert rep["status"] == 0 and rep["rel_residual"] <= tol, rep
    assert canon_residual(x, I0, p) <= 1.01 * tol
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= err_bar(x, I0, ref, p)


@pytest.mark.parametrize("shape", [(6, 30, 50), (1, 17, 33), (9, 1, 1)])
def test_npr_fp64_matches_oracle(gd, shape):
    say("npr f64", shape)
    p = PAPER
    I0 = video(shape, seed=13100417).numpy()
    ref = npr.npr_filter(I0, p["alpha"], p["beta"], p["lam"], p["sigma"])
    out, rep = gd.npr_filter(torch.from_numpy(I0).cuda(), p["alpha"], p["beta"], p["lam"], p["sigma"],
                             storage=gd.F64, rel_tol=1e-11)
    x = out.cpu().numpy()
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-11, rep
    assert canon_residual(x, I0, p) <= 1.01e-11
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-8


@pytest.mark.parametrize("tin", [torch.float16, torch.bfloat16])
def test_npr_16bit_input(gd, tin):
    """A 16-bit input volume: both sides see the same rounded values."""
    say("npr input", tin)
    p = PAPER
    I0t = video((6, 36, 64), seed=13100418).to(tin)
    I0 = I0t.double().numpy()
    ref = npr.npr_filter(I0, p["alpha"], p["beta"], p["lam"], p["sigma"])
    out, rep = gd.npr_filter(I0t.cuda(), p["alpha"], p["beta"], p["lam"], p["sigma"], out_dtype=torch.float64,
                             rel_tol=max(1e-6, 3.0 * fp32_floor(I0, ref, p)))
    x = out.cpu().numpy()
    assert rep["status"] == 0
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= err_bar(x, I0, ref, p)


def test_npr_identity_limit(gd):
    """lambda = 1 and sigma -> 0 keep every gradient: the output is the input."""
    say("npr identity")
    I0 = video((4, 20, 30)).numpy()
    out, rep = gd.npr_filter(torch.from_numpy(I0).cuda(), 0.001, (1.0, 1.0, 0.1), 1.0, 1e-9, storage=gd.F64,
                             rel_tol=1e-12)
    assert rep["status"] == 0
    assert np.abs(out.cpu().numpy() - I0).max() <= 1e-8 * np.abs(I0).max()
