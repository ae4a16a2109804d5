"""The "Linear" discretisation of Sec. 4.2: first-order B-spline finite
elements (FP64, CPU).

Test infrastructure only (see the package header).

Each voxel value is the coefficient of a trilinear hat function centred on
the voxel (unit spacing, supports clipped to the domain [0, n - 1] per axis:
the natural, Neumann, boundary).  The energy of Sec. 4,
integral alpha (I - V)^2 + (grad I - G)^t W (grad I - G), restricted to
this space gives the normal equations

    (alpha Mx My Mz + b_x Kx My Mz + b_y Mx Ky Mz + b_z Mx My Kz) I = rhs,

with the 1-D mass matrix M (1/6, 4/6, 1/6; end rows 2/6, 1/6) and the 1-D
stiffness matrix K (-1, 2, -1; end rows 1, -1: the same matrix as the
3-point Neumann second difference), a 27-point stencil.

Readings (the paper names the discretisation only): the anisotropic
diffusion of Eq. (1) takes G = (d I0/dx, d I0/dy, 0) with I0 interpolated in
the same space, so its right-hand side is (b_x Kx My Mz + b_y Mx Ky Mz) I0;
alpha = 0 leaves the constants as null space and the solution is fixed by
mean(I1) = mean(I0) as for the 7-point system.  The answer differs from
the 7-point one: that is why this discretisation has an oracle of its own.
"""

import numpy as np

from . import grid, hybrid


def mass_1d(n):
    """Gram matrix of the n hat functions on [0, n - 1] (n = 1: the constant)."""
    if n == 1:
        return np.ones((1, 1))
    M = np.zeros((n, n))
    for i in range(n - 1):  # element [i, i + 1]
        M[i, i] += 2.0 / 6.0
        M[i + 1, i + 1] += 2.0 / 6.0
        M[i, i + 1] += 1.0 / 6.0
        M[i + 1, i] += 1.0 / 6.0
    return M


def stiffness_1d(n):
    """Gram matrix of the derivatives of the n hat functions."""
    return hybrid.laplace_1d(n)


def tables(shape):
    """Finest-level per-axis (M, K) pairs ordered (x, y, z)."""
    nz, ny, nx = shape
    return [(mass_1d(n), stiffness_1d(n)) for n in (nx, ny, nz)]


def apply(x, alpha, beta):
    """The Linear operator applied to x."""
    x = grid.as3d(x)
    return hybrid.apply(x, tables(x.shape), alpha, beta)


def rhs_ad(I0, beta):
    """Right-hand side of Eq. (1) in this space: the in-slice derivatives of
    the interpolated input, (b_x Kx My Mz + b_y Mx Ky Mz) I0."""
    I0 = grid.as3d(I0)
    return hybrid.apply(I0, tables(I0.shape), 0.0, (beta[0], beta[1], 0.0))


def ad_solve(I0, beta, method="cg", rtol=1e-13, maxiter=100000):
    """Anisotropic diffusion with the Linear discretisation, mean(I1) = mean(I0).
    method 'dense' (tiny grids) or 'cg' (conjugate gradients on the
    mean-free subspace, to relative residual rtol)."""
    I0 = grid.as3d(I0)
    b = rhs_ad(I0, beta)
    if method == "dense":
        A = hybrid.kron_operator(tables(I0.shape), 0.0, beta)
        x = np.linalg.lstsq(A, b.ravel(), rcond=None)[0].reshape(I0.shape)
    else:
        x = np.zeros(I0.shape)
        r = b - apply(x, 0.0, beta)
        r -= r.mean()
        p = r.copy()
        rr = float(np.sum(r * r))
        nb = np.linalg.norm(b)
        it = 0
        while it < maxiter and np.sqrt(rr) > rtol * nb:
            q = apply(p, 0.0, beta)
            a = rr / float(np.sum(p * q))
            x += a * p
            r -= a * q
            r -= r.mean()
            rn = float(np.sum(r * r))
            p = r + (rn / rr) * p
            rr = rn
            it += 1
    return x - x.mean() + I0.mean()


def relative_residual(x, I0, beta):
    """||b - A x|| / ||b|| of the Linear AD system."""
    b = rhs_ad(I0, beta)
    return float(np.linalg.norm(b - apply(x, 0.0, beta)) / np.linalg.norm(b))
