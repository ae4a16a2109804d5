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


# ---------------------------------------------------------------------------
# per-slice screened Poisson (Eq. (2)) in the same space


def _slice_tables(ny, nx):
    """(M, K) pairs (x, y, z) of one 2-D slice seen as a one-plane grid."""
    return tables((1, ny, nx))


def rhs_sp(I0, I1, alpha, beta_xy=(1.0, 1.0)):
    """Right-hand side of Eq. (2) per slice with the value target I1 and the
    gradient target grad I0 both interpolated in the hat-function space:
    alpha Mx My I1 + (b_x Kx My + b_y Mx Ky) I0."""
    I0 = grid.as3d(I0)
    I1 = grid.as3d(I1)
    out = np.empty(I0.shape)
    T = _slice_tables(I0.shape[1], I0.shape[2])
    for z in range(I0.shape[0]):
        out[z] = (hybrid.apply(I1[z:z + 1], T, alpha, (0.0, 0.0, 0.0))
                  + hybrid.apply(I0[z:z + 1], T, 0.0, (beta_xy[0], beta_xy[1], 0.0)))[0]
    return out


def apply_sp(x, alpha, beta_xy=(1.0, 1.0)):
    """The per-slice operator alpha Mx My + b_x Kx My + b_y Mx Ky."""
    x = grid.as3d(x)
    out = np.empty(x.shape)
    T = _slice_tables(x.shape[1], x.shape[2])
    for z in range(x.shape[0]):
        out[z] = hybrid.apply(x[z:z + 1], T, alpha, (beta_xy[0], beta_xy[1], 0.0))[0]
    return out


def sp_solve(I0, I1, alpha, beta_xy=(1.0, 1.0), method="cg", rtol=1e-13, maxiter=100000):
    """Eq. (2) with the Linear discretisation, slice by slice (SPD for
    alpha > 0): method 'dense' (tiny slices) or 'cg'."""
    I0 = grid.as3d(I0)
    I1 = grid.as3d(I1)
    b = rhs_sp(I0, I1, alpha, beta_xy)
    x = np.empty(I0.shape)
    ny, nx = I0.shape[1:]
    for z in range(I0.shape[0]):
        if method == "dense":
            A = hybrid.kron_operator(_slice_tables(ny, nx), alpha, (beta_xy[0], beta_xy[1], 0.0))
            x[z] = np.linalg.solve(A, b[z].ravel()).reshape(ny, nx)
            continue
        xs = np.zeros((1, ny, nx))
        bz = b[z:z + 1]
        r = bz - apply_sp(xs, alpha, beta_xy)
        p = r.copy()
        rr = float(np.sum(r * r))
        nb = np.linalg.norm(bz)
        it = 0
        while it < maxiter and np.sqrt(rr) > rtol * nb:
            q = apply_sp(p, alpha, beta_xy)
            a = rr / float(np.sum(p * q))
            xs += a * p
            r -= a * q
            rn = float(np.sum(r * r))
            p = r + (rn / rr) * p
            rr = rn
            it += 1
        x[z] = xs[0]
    return x


def sp_relative_residuals(x, I0, I1, alpha, beta_xy=(1.0, 1.0)):
    """Per-slice ||b - A x|| / ||b|| of the Linear SP system."""
    b = rhs_sp(I0, I1, alpha, beta_xy)
    r = b - apply_sp(x, alpha, beta_xy)
    return np.array([np.linalg.norm(r[z]) / np.linalg.norm(b[z]) for z in range(b.shape[0])])
