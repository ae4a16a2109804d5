"""Single multigrid steps of Sec. 4.1, written plainly (FP64, CPU).

Test infrastructure only (see the package header).

These are the reference for kernel-level parity: one red-black Gauss-Seidel
sweep, the residual, the restriction of a residual to the next coarser level,
and the up-sampling of a coarse correction.  Each takes every coefficient as
an explicit argument: a level's operator is alpha * Id + sum_a w_a * L_a with
L_a the 3-point Neumann second difference along axis a (the 7-point
"Constant" stencil of Sec. 4.2 with per-level weights w = (w_x, w_y, w_z)).

Coarsening factors ``c = (c_x, c_y, c_z)`` are 1 (axis kept) or 2 (axis
halved); a coarse grid has ceil(n / c) cells per axis, so an odd last fine
cell is the only child of its coarse cell.
"""

import numpy as np

from . import grid


def _neighbour_terms(x, w):
    """Per voxel: (sum of w_nb * x_nb over existing neighbours,
    sum of w_nb over existing neighbours)."""
    x = grid.as3d(x)
    s = np.zeros_like(x)
    d = np.zeros_like(x)
    for c, ax in enumerate(grid.AXIS):
        if w[c] == 0.0 or x.shape[ax] == 1:
            continue
        n = x.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        s[lo] += w[c] * x[hi]   # neighbour at +1
        s[hi] += w[c] * x[lo]   # neighbour at -1
        d[lo] += w[c]
        d[hi] += w[c]
    return s, d


def parity(shape):
    """0 for red voxels ((i + j + k) even), 1 for black."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (i + j + k) & 1


def rb_sweep(x, b, alpha, w):
    """One red-black Gauss-Seidel sweep: every red voxel is set to the value
    that zeroes its own residual given its (black) neighbours, then every
    black voxel likewise given the updated red ones (multi-coloured GS, the
    parallel relaxation of Sec. 4.1 "Parallelization").  A voxel with no
    coupling at all (alpha == 0, no neighbours) is set to 0."""
    x = grid.as3d(x).copy()
    b = grid.as3d(b)
    col = parity(x.shape)
    for colour in (0, 1):
        s, d = _neighbour_terms(x, w)
        den = alpha + d
        new = np.where(den > 0.0, (b + s) / np.where(den > 0.0, den, 1.0), 0.0)
        x = np.where(col == colour, new, x)
    return x


def residual(x, b, alpha, w):
    """r = b - (alpha Id + sum_a w_a L_a) x."""
    return grid.as3d(b) - grid.apply_A(x, alpha, w)


def coarse_shape(shape, c):
    """Coarse grid size: ceil(n / c) per axis; ``c`` is (c_x, c_y, c_z)."""
    nz, ny, nx = shape
    return (-(-nz // c[2]), -(-ny // c[1]), -(-nx // c[0]))


def restrict_sum(r, c):
    """Coarse constraints from a fine residual: each coarse cell receives the
    sum of its children (the transpose of piecewise-constant up-sampling,
    stencil (1,1) per halved axis; Sec. 4.2 "Constant")."""
    r = grid.as3d(r)
    nz, ny, nx = r.shape
    cs = coarse_shape(r.shape, c)
    out = np.zeros(cs)
    for k in range(nz):
        for j in range(ny):
            out[k // c[2], j // c[1], :] += np.bincount(
                np.arange(nx) // c[0], weights=r[k, j, :], minlength=cs[2]
            )
    return out


def prolong_constant(e, fine_shape, c):
    """Piecewise-constant up-sampling: each fine cell takes its parent's value
    (stencil (1,1) per halved axis; Sec. 4.2 "Constant")."""
    e = grid.as3d(e)
    nz, ny, nx = fine_shape
    k = np.arange(nz) // c[2]
    j = np.arange(ny) // c[1]
    i = np.arange(nx) // c[0]
    return e[k[:, None, None], j[None, :, None], i[None, None, :]]


def _trilinear_weights(n_fine, n_coarse, c):
    """1-D cell-centred linear interpolation matrix (n_fine x n_coarse).

    With c == 2 the fine cell centre i + 1/2 sits at coarse coordinate
    (i + 1/2) / 2; it takes 3/4 of its parent I = i // 2 and 1/4 of the
    nearer coarse neighbour (I - 1 for even i, I + 1 for odd i).  A neighbour
    outside the grid is replaced by the parent itself (mirror boundary,
    consistent with the natural boundary condition).  c == 1 is the identity."""
    P = np.zeros((n_fine, n_coarse))
    for i in range(n_fine):
        if c == 1:
            P[i, i] = 1.0
            continue
        I = i // 2
        J = I - 1 if i % 2 == 0 else I + 1
        if 0 <= J < n_coarse:
            P[i, I] += 0.75
            P[i, J] += 0.25
        else:
            P[i, I] += 1.0
    return P


def prolong_trilinear(e, fine_shape, c):
    """Cell-centred (bi/tri)linear up-sampling of a coarse correction, the
    tensor product of the 1-D weights of :func:`_trilinear_weights`."""
    e = grid.as3d(e)
    nz, ny, nx = fine_shape
    cz, cy, cx = e.shape
    Px = _trilinear_weights(nx, cx, c[0])
    Py = _trilinear_weights(ny, cy, c[1])
    Pz = _trilinear_weights(nz, cz, c[2])
    return np.einsum("ka,jb,ic,abc->kji", Pz, Py, Px, e, optimize=True)


def relative_residual(x, b, alpha, beta):
    """||b - A x||_2 / ||b||_2: the residual measure of the Table 1 caption
    (norm of the residual over the norm of the initial constraints, x0 = 0)."""
    b = grid.as3d(b)
    return float(np.linalg.norm(residual(x, b, alpha, beta)) / np.linalg.norm(b))
