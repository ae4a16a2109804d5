"""The windowed relaxation behind the streamed levels (Sec. 4.1: every
V-cycle is two streaming passes through the data with a window of slices),
checked on the oracle's own multigrid steps on the CPU.

A slab [z0, z1) is processed in the window [z0 - h, z1 + h), clipped to the
grid and treated as a grid of its own (natural boundary at its cut faces),
with h = 2 nu + 2 and windows starting on even planes.  Then nu red-black
sweeps, the residual and the pairwise restriction of the window agree with
those of the whole grid on the slab (down pass), and so do the
interpolated coarse correction followed by nu sweeps (up pass).  A halo two
planes too thin fails: an error at a cut face moves two planes inwards per
sweep.
"""

import numpy as np
import pytest

from oracle import mgsteps as om


def windows(nz, slab, halo):
    slab = min(nz, max(slab + slab % 2, halo))
    out = []
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        out.append((max(0, z0 - halo), min(nz, z1 + halo), z0, z1))
    return out


def sweeps(x, b, alpha, w, nu):
    for _ in range(nu):
        x = om.rb_sweep(x, b, alpha, w)
    return x


CASES = [(21, 6, 1), (30, 8, 2), (27, 6, 2), (16, 16, 2), (33, 10, 3)]
ALPHA, W, C = 0.01, (1.0, 0.7, 4.0), (1, 1, 2)


@pytest.mark.parametrize("nz,slab,nu", CASES)
def test_down_pass_windows_reproduce_the_whole_grid(nz, slab, nu):
    rng = np.random.default_rng(nz * 100 + slab)
    shape = (nz, 5, 6)
    x, b = rng.standard_normal(shape), rng.standard_normal(shape)
    xs = sweeps(x, b, ALPHA, W, nu)
    bc = om.restrict_sum(om.residual(xs, b, ALPHA, W), C)
    halo = 2 * nu + 2
    covered = np.zeros(nz, bool)
    for a, e, z0, z1 in windows(nz, slab, halo):
        assert a % 2 == 0
        xw = sweeps(x[a:e], b[a:e], ALPHA, W, nu)
        assert np.array_equal(xw[z0 - a:z1 - a], xs[z0:z1])
        bw = om.restrict_sum(om.residual(xw, b[a:e], ALPHA, W), C)
        c0, c1 = z0 // 2, (z1 + 1) // 2
        assert np.abs(bw[c0 - a // 2:c1 - a // 2] - bc[c0:c1]).max() <= 1e-13 * np.abs(bc).max()
        covered[z0:z1] = True
    assert covered.all()


@pytest.mark.parametrize("nz,slab,nu", CASES)
def test_up_pass_windows_reproduce_the_whole_grid(nz, slab, nu):
    rng = np.random.default_rng(nz * 100 + slab + 1)
    shape = (nz, 5, 6)
    x, b = rng.standard_normal(shape), rng.standard_normal(shape)
    ec = rng.standard_normal(om.coarse_shape(shape, C))
    xs = sweeps(x + om.prolong_trilinear(ec, shape, C), b, ALPHA, W, nu)
    halo = 2 * nu + 2
    for a, e, z0, z1 in windows(nz, slab, halo):
        cn = (e - a + 1) // 2  # coarse planes under the window
        ew = ec[a // 2:a // 2 + cn]
        xw = x[a:e] + om.prolong_trilinear(ew, (e - a,) + shape[1:], C)
        xw = sweeps(xw, b[a:e], ALPHA, W, nu)
        assert np.abs(xw[z0 - a:z1 - a] - xs[z0:z1]).max() <= 1e-12 * np.abs(xs).max()


def test_a_thinner_halo_is_not_enough():
    nz, slab, nu = 30, 8, 2
    rng = np.random.default_rng(7)
    shape = (nz, 5, 6)
    x, b = rng.standard_normal(shape), rng.standard_normal(shape)
    xs = sweeps(x, b, ALPHA, W, nu)
    worst = 0.0
    for a, e, z0, z1 in windows(nz, slab, 2 * nu - 2):
        xw = sweeps(x[a:e], b[a:e], ALPHA, W, nu)
        worst = max(worst, np.abs(xw[z0 - a:z1 - a] - xs[z0:z1]).max())
    assert worst > 1e-6
