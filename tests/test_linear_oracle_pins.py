"""Pins of the Linear (B-spline finite element) oracle of Sec. 4.2.

The mass and stiffness matrices are checked against Gauss quadrature of the
hat functions and their derivatives; the assembled AD right-hand side
against quadrature of the energy's linear term on a tiny grid; the solution
against a dense solve, the identity case (no cross-slice weight) and the
gauge; its energy against loops.
"""

import numpy as np
import pytest

from oracle import hybrid, linear

GP = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))  # 2-point Gauss on [0, 1], exact for cubics


def hat(i, t):
    return np.maximum(0.0, 1.0 - np.abs(t - i))


def dhat(i, t):
    return np.where(np.abs(t - i) < 1.0, -np.sign(t - i), 0.0)


@pytest.mark.parametrize("n", [2, 3, 6])
def test_mass_and_stiffness_by_quadrature(n):
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for e in range(n - 1):  # element [e, e + 1], integrands smooth inside
        for g in GP:
            t = e + g
            for i in range(n):
                for j in range(n):
                    M[i, j] += 0.5 * hat(i, t) * hat(j, t)
                    K[i, j] += 0.5 * dhat(i, t) * dhat(j, t)
    assert np.abs(linear.mass_1d(n) - M).max() < 1e-14
    assert np.abs(linear.stiffness_1d(n) - K).max() < 1e-14


def test_ad_rhs_by_quadrature():
    """b_v = integral (b_x dphi_v/dx dI0/dx + b_y dphi_v/dy dI0/dy) over the
    domain, I0 interpolated: tensor Gauss quadrature per cell."""
    nz, ny, nx = 2, 3, 4
    I0 = np.random.default_rng(1).standard_normal((nz, ny, nx))
    beta = (1.0, 0.5, 4.0)
    b = np.zeros_like(I0)
    for cz in range(nz - 1):
        for cy in range(ny - 1):
            for cx in range(nx - 1):
                for gz in GP:
                    for gy in GP:
                        for gx in GP:
                            z, y, x = cz + gz, cy + gy, cx + gx
                            w = 0.125
                            ix = [hat(i, x) for i in range(nx)]
                            iy = [hat(j, y) for j in range(ny)]
                            iz = [hat(k, z) for k in range(nz)]
                            dx = [dhat(i, x) for i in range(nx)]
                            dy = [dhat(j, y) for j in range(ny)]
                            ux = sum(I0[k, j, i] * dx[i] * iy[j] * iz[k] for k in range(nz) for j in range(ny)
                                     for i in range(nx))
                            uy = sum(I0[k, j, i] * ix[i] * dy[j] * iz[k] for k in range(nz) for j in range(ny)
                                     for i in range(nx))
                            for k in range(nz):
                                for j in range(ny):
                                    for i in range(nx):
                                        b[k, j, i] += w * (beta[0] * dx[i] * iy[j] * iz[k] * ux
                                                           + beta[1] * ix[i] * dy[j] * iz[k] * uy)
    assert np.abs(linear.rhs_ad(I0, beta) - b).max() < 1e-12


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 6, 7), (4, 1, 3), (2, 2, 2)])
def test_ad_solution(shape):
    beta = (1.0, 1.0, 4.0)
    I0 = np.random.default_rng(2).standard_normal(shape) * 10.0
    xd = linear.ad_solve(I0, beta, method="dense")
    xc = linear.ad_solve(I0, beta, method="cg")
    assert np.abs(xd - xc).max() < 1e-9 * np.abs(xd).max()
    assert abs(xd.mean() - I0.mean()) < 1e-12
    assert linear.relative_residual(xd, I0, beta) < 1e-11
    # no cross-slice weight: the input is a minimiser, and the slices decouple,
    # so the solution is I0 up to one constant per slice
    d = linear.ad_solve(I0, (1.0, 1.0, 0.0), method="dense") - I0
    assert np.abs(d - d.mean(axis=(1, 2), keepdims=True)).max() < 1e-9
    # a z-constant stack is a fixed point
    zc = np.broadcast_to(I0[:1], shape).copy()
    assert np.abs(linear.ad_solve(zc, beta, method="dense") - zc).max() < 1e-9


def test_differs_from_the_7_point_answer():
    from oracle import solvers
    I0 = np.random.default_rng(3).standard_normal((4, 6, 6)) * 10.0
    a = linear.ad_solve(I0, (1.0, 1.0, 4.0), method="dense")
    c = solvers.ad_dct(I0, (1.0, 1.0, 4.0))
    assert np.linalg.norm(a - c) > 1e-3 * np.linalg.norm(c)


def test_tables_are_the_hybrid_level0_with_mass():
    M, K = linear.tables((3, 4, 5))[0]
    assert np.array_equal(K, hybrid.laplace_1d(5))
    # hats sum to one, so a row sum is the hat's integral: 1 inside, 1/2 at the ends
    assert np.allclose(M.sum(axis=1), [0.5, 1.0, 1.0, 1.0, 0.5]) and np.isclose(M.sum(), 4.0)
