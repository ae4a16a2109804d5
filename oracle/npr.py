"""Gradient-modulation ("NPR") filter of the discussion section (FP64, CPU).

Test infrastructure only (see the package header).

Sec. 6 applies the general solver of Sec. 4 to a video volume: the output
minimises

    alpha * sum_v (I_v - I0_v)^2 + sum_a beta_a * sum_{faces f normal to a} ((D_a I)_f - V_{a,f})^2,

the energy of Sec. 4 with value target I0 and gradient target the input's
gradient modulated by its magnitude (the non-photorealistic filter of Bhat
et al. that the paper cites):

    V = lambda * (1 - exp(-|grad I0|^2 / (2 sigma^2))) * grad I0.

Small gradients (|grad I0| << sigma) are suppressed, large ones scaled by
lambda.  The paper uses alpha = 0.001, W = Diag(1, 1, 0.1), lambda = 1.25 and
sigma = 5 on grey values in [0, 256).

Discrete reading (the paper states the filter in continuous form only): the
gradient of I0 at voxel v is its forward-difference vector
g_v = (I0[v+e_x] - I0[v], I0[v+e_y] - I0[v], I0[v+e_z] - I0[v]), a component
being 0 where the face v -> v+e_a leaves the grid; |grad I0|^2 at v is
|g_v|^2, and the face v -> v+e_a (the face "owned" by v) carries
V = lambda (1 - exp(-|g_v|^2 / (2 sigma^2))) g_{v,a}.

No pin from the paper's own numbers exists (its video is not available);
the functions are pinned by the identity and zero-target limits, by a
loop-by-loop restatement, and by the energy minimum (tests).
"""

import numpy as np

from . import grid, solvers

AXIS = grid.AXIS


def modulate(I0, lam, sigma):
    """The modulated gradient field V as three face fields (x, y, z), each
    one shorter than the grid along its own axis (the layout of grid.grad)."""
    I0 = grid.as3d(I0)
    g = [grid.grad(I0, c) for c in range(3)]
    # |g_v|^2: every face contributes to the voxel that owns it (its lower end)
    m2 = np.zeros(I0.shape)
    for c in range(3):
        n = I0.shape[AXIS[c]]
        if n > 1:
            own = [slice(None)] * 3
            own[AXIS[c]] = slice(0, n - 1)
            m2[tuple(own)] += g[c] ** 2
    factor = lam * (1.0 - np.exp(-m2 / (2.0 * sigma * sigma)))
    out = []
    for c in range(3):
        n = I0.shape[AXIS[c]]
        own = [slice(None)] * 3
        own[AXIS[c]] = slice(0, max(n - 1, 0))
        out.append(factor[tuple(own)] * g[c])
    return tuple(out)


def modulate_loops(I0, lam, sigma):
    """The same field computed voxel by voxel with plain loops (tiny grids)."""
    I0 = grid.as3d(I0)
    nz, ny, nx = I0.shape
    out = [np.zeros((nz, ny, nx - 1)), np.zeros((nz, ny - 1, nx)), np.zeros((nz - 1, ny, nx))]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                gx = I0[k, j, i + 1] - I0[k, j, i] if i + 1 < nx else 0.0
                gy = I0[k, j + 1, i] - I0[k, j, i] if j + 1 < ny else 0.0
                gz = I0[k + 1, j, i] - I0[k, j, i] if k + 1 < nz else 0.0
                f = lam * (1.0 - np.exp(-(gx * gx + gy * gy + gz * gz) / (2.0 * sigma * sigma)))
                if i + 1 < nx:
                    out[0][k, j, i] = f * gx
                if j + 1 < ny:
                    out[1][k, j, i] = f * gy
                if k + 1 < nz:
                    out[2][k, j, i] = f * gz
    return tuple(out)


def rhs(I0, alpha, beta, lam, sigma):
    """alpha I0 + sum_a beta_a D_a^T V_a: the right-hand side of the filter's
    normal equations (Sec. 4 with V = I0 and G = the modulated field)."""
    I0 = grid.as3d(I0)
    return grid.rhs_general(I0, modulate(I0, lam, sigma), alpha, beta, shape=I0.shape)


def npr_filter(I0, alpha=0.001, beta=(1.0, 1.0, 0.1), lam=1.25, sigma=5.0, method="dct", rtol=1e-13):
    """The filtered volume: the minimiser of the energy above (alpha > 0).
    method 'dct' (exact), 'dense' (tiny grids) or 'cg' (to relative residual rtol)."""
    I0 = grid.as3d(I0)
    return solvers.general_solve(I0, modulate(I0, lam, sigma), alpha, beta, method=method, shape=I0.shape,
                                 rtol=rtol)


def energy(I, I0, alpha, beta, lam, sigma):
    """The filter's discrete energy, written with loops (tiny grids)."""
    return grid.energy(I, I0, modulate_loops(I0, lam, sigma), alpha, beta)
