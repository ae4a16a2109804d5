"""Pins of the gradient-modulation (NPR) filter oracle, Sec. 6.

Each check ties the oracle to something other than itself: a loop-by-loop
restatement of the modulation, the filter's limits (identity when every
gradient is kept, screened smoothing with a closed form when every gradient
is suppressed), a hand-computed step edge, and the energy minimum written
with plain loops.
"""

import numpy as np
import pytest

from oracle import grid, npr

SHAPES = [(3, 4, 5), (1, 1, 7), (2, 5, 1), (4, 1, 3), (1, 6, 6)]


def rnd(shape, seed=0, scale=20.0):
    return np.random.default_rng(seed).standard_normal(shape) * scale + 100.0


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("lam,sigma", [(1.25, 5.0), (0.5, 30.0), (2.0, 0.7)])
def test_modulation_matches_loops(shape, lam, sigma):
    I0 = rnd(shape)
    a = npr.modulate(I0, lam, sigma)
    b = npr.modulate_loops(I0, lam, sigma)
    for c in range(3):
        assert a[c].shape == b[c].shape
        if b[c].size:
            assert np.abs(a[c] - b[c]).max() <= 1e-12 * max(1.0, np.abs(b[c]).max())


def test_step_edge_by_hand():
    # one x-face carries a jump of 100 >> sigma: V = lambda * 100 there, 0 elsewhere
    I0 = np.array([[[0.0, 0.0, 0.0, 100.0, 100.0]]])
    gx, gy, gz = npr.modulate(I0, 1.25, 5.0)
    assert gx.shape == (1, 1, 4) and gy.size == 0 and gz.size == 0
    assert np.array_equal(gx, np.array([[[0.0, 0.0, 125.0, 0.0]]]))
    # a gradient of sigma keeps lambda (1 - e^{-1/2}) of itself
    I0 = np.array([[[0.0, 5.0]]])
    assert abs(npr.modulate(I0, 1.0, 5.0)[0][0, 0, 0] - 5.0 * (1.0 - np.exp(-0.5))) < 1e-14


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("method", ["dense", "dct"])
def test_identity_when_every_gradient_is_kept(shape, method):
    """lambda = 1 and sigma -> 0: V = grad I0, so I0 itself has zero energy."""
    I0 = rnd(shape, seed=1)
    x = npr.npr_filter(I0, alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.0, sigma=1e-9, method=method)
    assert np.abs(x - I0).max() <= 1e-8 * np.abs(I0).max()


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 1, 8), (6, 2, 3)])
def test_screened_smoothing_when_every_gradient_is_suppressed(shape):
    """sigma -> infinity: V -> 0 and (alpha + sum beta L) x = alpha I0.  A
    separable cosine cos(pi k (i + 1/2) / n) per axis is an eigenvector of
    the Neumann second difference with eigenvalue 2 - 2 cos(pi k / n), so
    for such an input x = alpha / (alpha + sum beta_a lambda_a) I0."""
    alpha, beta = 0.05, (1.0, 2.0, 0.3)
    nz, ny, nx = shape
    ks = (1 % nx, 1 % ny, 1 % nz)  # one non-constant mode per axis of length > 1
    cx = np.cos(np.pi * ks[0] * (np.arange(nx) + 0.5) / nx)
    cy = np.cos(np.pi * ks[1] * (np.arange(ny) + 0.5) / ny)
    cz = np.cos(np.pi * ks[2] * (np.arange(nz) + 0.5) / nz)
    I0 = 3.0 * cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    lam_sum = sum(beta[c] * (2.0 - 2.0 * np.cos(np.pi * ks[c] / n)) for c, n in enumerate((nx, ny, nz)))
    want = alpha / (alpha + lam_sum) * I0
    for method in ("dense", "dct"):
        x = npr.npr_filter(I0, alpha=alpha, beta=beta, lam=1.25, sigma=1e12, method=method)
        assert np.abs(x - want).max() <= 1e-10


@pytest.mark.parametrize("shape", [(2, 3, 4), (1, 4, 5), (3, 1, 3)])
def test_solution_minimises_the_energy(shape):
    """The energy written with loops (value term plus modulated-gradient
    term) has its minimum at the oracle's solution: every direction raises
    it, and its directional derivatives vanish there."""
    alpha, beta, lam, sigma = 0.001, (1.0, 1.0, 0.1), 1.25, 5.0
    I0 = rnd(shape, seed=3, scale=8.0)
    x = npr.npr_filter(I0, alpha, beta, lam, sigma, method="dense")
    e0 = npr.energy(x, I0, alpha, beta, lam, sigma)
    rng = np.random.default_rng(4)
    for _ in range(4):
        d = rng.standard_normal(shape)
        ep = npr.energy(x + 1e-3 * d, I0, alpha, beta, lam, sigma)
        em = npr.energy(x - 1e-3 * d, I0, alpha, beta, lam, sigma)
        assert ep > e0 and em > e0
        assert abs(ep - em) / 2e-3 <= 1e-6 * max(1.0, e0)


def test_right_hand_side_definition():
    """rhs = alpha I0 + sum_a beta_a D_a^T V_a, with D_a^T taken face by face."""
    I0 = rnd((2, 3, 4), seed=5)
    alpha, beta, lam, sigma = 0.01, (1.0, 0.5, 0.2), 1.25, 5.0
    V = npr.modulate_loops(I0, lam, sigma)
    want = alpha * I0.copy()
    steps = ((0, 0, 1), (0, 1, 0), (1, 0, 0))
    for c in range(3):
        dz, dy, dx = steps[c]
        for (k, j, i), v in np.ndenumerate(V[c]):
            # face from (k, j, i) to (k + dz, j + dy, i + dx): -v at the lower voxel, +v at the upper
            want[k, j, i] -= beta[c] * v
            want[k + dz, j + dy, i + dx] += beta[c] * v
    assert np.abs(npr.rhs(I0, alpha, beta, lam, sigma) - want).max() <= 1e-12


def test_oracle_header_names_the_reading():
    assert "Discrete reading" in npr.__doc__ and "owned" in npr.__doc__
    assert grid.AXIS == (2, 1, 0)
