"""Discrete gradient-domain operators on a regular voxel grid (FP64, CPU).

Test infrastructure only (see the package header).

Discretisation (Sec. 4.2, "Constant"/"Hybrid" finest level): one unknown per
voxel, unit spacing.  The gradient along axis ``a`` lives on the faces between
face-adjacent voxels, ``(D_a I)_f = I[v + e_a] - I[v]``.  A face outside the
grid does not exist, which is the natural (Neumann) boundary condition of the
energy.  The continuous energy of Sec. 4,

    E(I) = integral  alpha (I - V)^2 + (grad I - G)^t W (grad I - G),

becomes

    E(I) = alpha * sum_v (I_v - V_v)^2
         + sum_a beta_a * sum_{faces f normal to a} ((D_a I)_f - G_{a,f})^2,

and its normal equations are

    (alpha Id + sum_a beta_a D_a^T D_a) I = alpha V + sum_a beta_a D_a^T G_a,

the discrete form of (alpha - div W grad) I = alpha V - div W G.  ``D_a^T D_a``
is the 3-point Neumann Laplacian along ``a`` (off-diagonal -1), so the operator
is the 7-point stencil of the "Constant" discretisation.

Axis convention: arrays are ``[nz][ny][nx]``; x is numpy axis 2, y axis 1,
z axis 0.  ``beta`` is always given as ``(beta_x, beta_y, beta_z)``.
"""

import numpy as np

# numpy axis of each gradient component (x, y, z)
AXIS = (2, 1, 0)


def as3d(a):
    """View a 1-, 2- or 3-D array as [nz][ny][nx] (missing leading axes = 1)."""
    a = np.asarray(a, dtype=np.float64)
    while a.ndim < 3:
        a = a[None]
    return a


def grad(I, comp):
    """Forward difference along component ``comp`` (0=x, 1=y, 2=z).

    Returns the face field of shape n_a - 1 along that axis."""
    return np.diff(as3d(I), axis=AXIS[comp])


def grad_T(g, comp, shape):
    """Adjoint of :func:`grad`: (D_a^T g)_v = g_{v - e_a} - g_v, with the
    values of missing (outside) faces taken as zero."""
    ax = AXIS[comp]
    g = np.asarray(g, dtype=np.float64)
    pad = [(0, 0)] * 3
    pad[ax] = (1, 1)
    gp = np.pad(g, pad)
    out = -np.diff(gp, axis=ax)
    assert out.shape == tuple(shape)
    return out


def laplace_axis(I, comp):
    """D_a^T D_a I: the Neumann second difference along one axis (PSD sign)."""
    I = as3d(I)
    return grad_T(grad(I, comp), comp, I.shape)


def apply_A(x, alpha, beta):
    """(alpha Id + sum_a beta_a D_a^T D_a) x  -- the operator of Sec. 4."""
    x = as3d(x)
    y = alpha * x
    for c in range(3):
        if beta[c] != 0.0 and x.shape[AXIS[c]] > 1:
            y = y + beta[c] * laplace_axis(x, c)
    return y


def rhs_general(V, G, alpha, beta, shape=None):
    """alpha V + sum_a beta_a D_a^T G_a  -- right-hand side of Sec. 4.

    ``G`` is a triple of face fields (each n_a - 1 long along its axis) or
    None entries for zero components; ``V`` may be None when alpha == 0."""
    if shape is None:
        shape = as3d(V).shape
    b = np.zeros(shape)
    if alpha != 0.0:
        b += alpha * as3d(V)
    for c in range(3):
        if G[c] is not None and beta[c] != 0.0 and shape[AXIS[c]] > 1:
            b += beta[c] * grad_T(G[c], c, shape)
    return b


def rhs_ad(I0, beta):
    """Right-hand side of the anisotropic diffusion, Eq. (1) / Sec. 3.1.1.

    The target field is G = (dI0/dx, dI0/dy, 0): the in-slice derivatives of
    the input and a zero cross-slice derivative; alpha = 0."""
    I0 = as3d(I0)
    G = (grad(I0, 0), grad(I0, 1), None)
    return rhs_general(None, G, 0.0, beta, shape=I0.shape)


def rhs_sp(I0, I1, alpha, beta_xy=(1.0, 1.0)):
    """Right-hand side of the per-slice screened Poisson, Eq. (2) / Sec. 3.1.2.

    alpha I1 - Delta_pi I0 with pi = Diag(1, 1, 0): value target I1, gradient
    target the in-slice gradient of I0, no coupling across slices."""
    I0 = as3d(I0)
    G = (grad(I0, 0), grad(I0, 1), None)
    return rhs_general(I1, G, alpha, (beta_xy[0], beta_xy[1], 0.0), shape=I0.shape)


def energy(I, V, G, alpha, beta):
    """Discrete energy of Sec. 4 written directly as sums over voxels and faces
    (pure-Python loops; tiny grids only).  Used to pin apply_A/rhs_general:
    its minimiser must solve their system."""
    I = as3d(I)
    nz, ny, nx = I.shape
    E = 0.0
    if alpha != 0.0:
        V = as3d(V)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    E += alpha * (I[k, j, i] - V[k, j, i]) ** 2
    steps = ((0, 0, 1), (0, 1, 0), (1, 0, 0))  # (dz, dy, dx) for x, y, z
    for c in range(3):
        dz, dy, dx = steps[c]
        if beta[c] == 0.0:
            continue
        for k in range(nz - dz):
            for j in range(ny - dy):
                for i in range(nx - dx):
                    d = I[k + dz, j + dy, i + dx] - I[k, j, i]
                    g = 0.0 if G[c] is None else G[c][k, j, i]
                    E += beta[c] * (d - g) ** 2
    return E
