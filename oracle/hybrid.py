"""Steps of the "Hybrid" discretisation of Sec. 4.2 (FP64, CPU).

Test infrastructure only (see the package header).

Hybrid keeps the 7-point ("Constant") operator on the finest level and moves
between levels with the prolongation of first-order B-splines, the stencil
(1/2, 1, 1/2) per halved axis; restriction is its transpose and every coarser
operator is the Galerkin product A_{l+1} = P^T A_l P (a 27-point stencil).

Reading of the nesting on a grid of n samples (the paper states the stencil
only): along a halved axis coarse sample c sits on fine sample 2c, so the
coarse axis has ceil(n / 2) samples; fine sample f takes e[f / 2] when f is
even and (e[(f - 1) / 2] + e[(f + 1) / 2]) / 2 when f is odd, and an odd last
fine sample with no coarse sample to its right takes e[(f - 1) / 2] alone,
so that constants stay constant (the null space of the pure-Neumann AD
system).  A kept axis has P = Id.

The finest operator is alpha Id + sum_a w_a L_a, L_a the Neumann 3-point
second difference along a; with P = P_x (x) P_y (x) P_z every level is

    A_l = alpha Mx My Mz + w_x Kx My Mz + w_y Mx Ky Mz + w_z Mx My Kz

(Kronecker products of 1-D matrices along x, y, z), M_0 = Id, K_0 = L and
M_{l+1} = P^T M_l P, K_{l+1} = P^T K_l P per axis: tridiagonal at every
level.  The relaxation of a 27-point level is 8-colour Gauss-Seidel: the
colour of sample (i, j, k) is (i mod 2) + 2 (j mod 2) + 4 (k mod 2), colours
in increasing order; samples of one colour are not coupled, so each colour
is updated at once.
"""

import numpy as np

from . import grid


def prolong_1d(n, halved):
    """Dense 1-D prolongation matrix, n fine samples x n_coarse."""
    if not halved:
        return np.eye(n)
    nc = (n + 1) // 2
    P = np.zeros((n, nc))
    for f in range(n):
        if f % 2 == 0:
            P[f, f // 2] = 1.0
        elif (f + 1) // 2 < nc:
            P[f, (f - 1) // 2] = 0.5
            P[f, (f + 1) // 2] = 0.5
        else:
            P[f, (f - 1) // 2] = 1.0
    return P


def laplace_1d(n):
    """Neumann 3-point second difference D^T D (PSD sign), n x n."""
    L = np.zeros((n, n))
    for i in range(n - 1):
        L[i, i] += 1.0
        L[i + 1, i + 1] += 1.0
        L[i, i + 1] -= 1.0
        L[i + 1, i] -= 1.0
    return L


def level_tables(n, halvings):
    """Per level l = 0 .. len(halvings): the 1-D pair (M_l, K_l) of one axis
    with n finest samples; halvings[l] says whether level l -> l + 1 halves
    this axis."""
    M, K = np.eye(n), laplace_1d(n)
    out = [(M, K)]
    for h in halvings:
        P = prolong_1d(M.shape[0], h)
        M, K = P.T @ M @ P, P.T @ K @ P
        out.append((M, K))
    return out


def kron_operator(mats, alpha, w):
    """Dense operator of one level from its per-axis (M, K) pairs ordered
    (x, y, z); unknowns in [nz][ny][nx] order (tiny grids only)."""
    (Mx, Kx), (My, Ky), (Mz, Kz) = mats
    k3 = lambda a, b, c: np.kron(c, np.kron(b, a))  # x fastest
    return alpha * k3(Mx, My, Mz) + w[0] * k3(Kx, My, Mz) + w[1] * k3(Mx, Ky, Mz) + w[2] * k3(Mx, My, Kz)


def _along(A, x, ax):
    """Apply the 1-D matrix A along array axis ax of x."""
    return np.moveaxis(np.tensordot(A, x, axes=([1], [ax])), 0, ax)


def apply(x, mats, alpha, w):
    """A_l x from the per-axis tables (separable products)."""
    x = grid.as3d(x)
    (Mx, Kx), (My, Ky), (Mz, Kz) = mats
    xm, xk = _along(Mx, x, 2), _along(Kx, x, 2)  # Mx x, Kx x
    mm = _along(My, xm, 1)                       # Mx My x
    out = alpha * _along(Mz, mm, 0) + w[2] * _along(Kz, mm, 0)
    out += w[0] * _along(Mz, _along(My, xk, 1), 0)
    out += w[1] * _along(Mz, _along(Ky, xm, 1), 0)
    return out


def diagonal(shape, mats, alpha, w):
    """The diagonal of A_l, per sample."""
    (Mx, Kx), (My, Ky), (Mz, Kz) = mats
    mx, kx = np.diag(Mx)[None, None, :], np.diag(Kx)[None, None, :]
    my, ky = np.diag(My)[None, :, None], np.diag(Ky)[None, :, None]
    mz, kz = np.diag(Mz)[:, None, None], np.diag(Kz)[:, None, None]
    return alpha * mx * my * mz + w[0] * kx * my * mz + w[1] * mx * ky * mz + w[2] * mx * my * kz


def colour(shape):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return (i & 1) + 2 * (j & 1) + 4 * (k & 1)


def gs8_sweep(x, b, mats, alpha, w):
    """One 8-colour Gauss-Seidel sweep of A_l x = b: colour by colour, every
    sample of the colour is set to zero its own residual.  A sample with a
    zero diagonal is set to 0."""
    x = grid.as3d(x).copy()
    b = grid.as3d(b)
    d = diagonal(x.shape, mats, alpha, w)
    col = colour(x.shape)
    for c in range(8):
        m = col == c
        if not m.any():
            continue
        r = b - apply(x, mats, alpha, w)
        upd = np.where(d != 0.0, x + r / np.where(d != 0.0, d, 1.0), 0.0)
        x[m] = upd[m]
    return x


def gs8_sweep_loops(x, b, A):
    """The same sweep from the dense operator with plain loops: each sample
    of a colour in turn, sequentially (tiny grids)."""
    x = grid.as3d(x).copy()
    shape = x.shape
    xf, bf = x.ravel(), grid.as3d(b).ravel()
    col = colour(shape).ravel()
    for c in range(8):
        for v in range(xf.size):
            if col[v] != c:
                continue
            s = bf[v] - A[v] @ xf + A[v, v] * xf[v]
            xf[v] = s / A[v, v] if A[v, v] != 0.0 else 0.0
    return xf.reshape(shape)


def transfer_mats(shape, halved):
    """Per-axis prolongation matrices (x, y, z) of a grid [nz][ny][nx]."""
    nz, ny, nx = shape
    return prolong_1d(nx, halved[0]), prolong_1d(ny, halved[1]), prolong_1d(nz, halved[2])


def restrict(r, P):
    """P^T r (the Galerkin restriction) with P = (Px, Py, Pz)."""
    r = grid.as3d(r)
    return _along(P[2].T, _along(P[1].T, _along(P[0].T, r, 2), 1), 0)


def prolong(e, P):
    """P e, the coarse correction up-sampled by the B-spline nesting."""
    e = grid.as3d(e)
    return _along(P[2], _along(P[1], _along(P[0], e, 2), 1), 0)
