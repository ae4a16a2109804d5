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


# ---- per-slice screened Poisson (Eq. (2)) in the same space


def test_sp_rhs_by_quadrature():
    """b_v = integral alpha phi_v I1 + b_x dphi_v/dx dI0/dx + b_y dphi_v/dy dI0/dy
    over a slice, I0 and I1 interpolated: tensor Gauss quadrature per cell."""
    ny, nx = 3, 4
    rng = np.random.default_rng(2)
    I0 = rng.standard_normal((1, ny, nx))
    I1 = rng.standard_normal((1, ny, nx))
    alpha, beta = 0.3, (1.0, 0.5)
    b = np.zeros((ny, nx))
    for cy in range(ny - 1):
        for cx in range(nx - 1):
            for gy in GP:
                for gx in GP:
                    y, x = cy + gy, cx + gx
                    w = 0.25
                    hx = np.array([hat(i, x) for i in range(nx)])
                    hy = np.array([hat(j, y) for j in range(ny)])
                    dx = np.array([dhat(i, x) for i in range(nx)])
                    dy = np.array([dhat(j, y) for j in range(ny)])
                    v1 = hy @ I1[0] @ hx
                    g0x = hy @ I0[0] @ dx
                    g0y = dy @ I0[0] @ hx
                    for j in range(ny):
                        for i in range(nx):
                            b[j, i] += w * (alpha * hy[j] * hx[i] * v1 + beta[0] * hy[j] * dx[i] * g0x
                                            + beta[1] * dy[j] * hx[i] * g0y)
    assert np.abs(linear.rhs_sp(I0, I1, alpha, beta)[0] - b).max() < 1e-13


def _energy_sp(I, I0, I1, alpha, beta):
    """alpha |I - I1|^2_M + b_x |dI/dx - dI0/dx|^2 + b_y |dI/dy - dI0/dy|^2
    of one slice with the Kronecker-assembled Gram matrices (independent of
    the oracle's separable application)."""
    ny, nx = I.shape
    Mx, My = linear.mass_1d(nx), linear.mass_1d(ny)
    Kx, Ky = linear.stiffness_1d(nx), linear.stiffness_1d(ny)
    M = np.kron(My, Mx)
    K = beta[0] * np.kron(My, Kx) + beta[1] * np.kron(Ky, Mx)
    d1 = (I - I1).ravel()
    d0 = (I - I0).ravel()
    return alpha * d1 @ M @ d1 + d0 @ K @ d0


@pytest.mark.parametrize("shape", [(2, 5, 7), (1, 1, 6), (3, 4, 1)])
def test_sp_solution_minimises_the_energy(shape):
    rng = np.random.default_rng(3)
    I0 = rng.uniform(0, 50, shape)
    I1 = I0 + rng.standard_normal(shape) * 5
    alpha, beta = 0.05, (1.0, 0.7)
    x = linear.sp_solve(I0, I1, alpha, beta, method="dense")
    xc = linear.sp_solve(I0, I1, alpha, beta, method="cg")
    assert np.abs(x - xc).max() < 1e-9 * np.abs(x).max()
    for z in range(shape[0]):
        e0 = _energy_sp(x[z], I0[z], I1[z], alpha, beta)
        for _ in range(4):
            d = rng.standard_normal(x[z].shape) * 1e-3
            assert _energy_sp(x[z] + d, I0[z], I1[z], alpha, beta) > e0
    assert linear.sp_relative_residuals(xc, I0, I1, alpha, beta).max() < 1e-12


def test_sp_special_cases():
    rng = np.random.default_rng(4)
    I0 = rng.uniform(0, 50, (2, 6, 5))
    # target values equal to the input: the input comes back
    assert np.abs(linear.sp_solve(I0, I0, 0.01, method="dense") - I0).max() < 1e-10
    # a per-slice constant offset of the target is reproduced exactly (K kills constants)
    off = np.array([3.0, -7.0])[:, None, None]
    assert np.abs(linear.sp_solve(I0, I0 + off, 0.01, method="dense") - (I0 + off)).max() < 1e-9
    # large alpha: the value target wins
    I1 = rng.uniform(0, 50, I0.shape)
    assert np.abs(linear.sp_solve(I0, I1, 1e9, method="dense") - I1).max() < 1e-5
    # the answer differs from the 7-point (Constant) one
    from oracle import solvers

    assert np.abs(linear.sp_solve(I0, I1, 0.01, method="dense") - solvers.sp_dct(I0, I1, 0.01)).max() > 1e-3
