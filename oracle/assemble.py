"""Explicit sparse assembly of the screened anisotropic operator (FP64, CPU).

Test infrastructure only (see the package header).

Built from the stencil description of the "Constant" discretisation in
Sec. 4.2: every pair of face-adjacent voxels along axis a is coupled with
off-diagonal -beta_a, and each voxel's diagonal is alpha plus the beta of
every neighbour it actually has (no neighbours outside the grid: natural
boundary).  This is written independently of ``grid.apply_A`` (which composes
difference operators) so that the two can pin each other.
"""

import numpy as np
import scipy.sparse as sp


def assemble(shape, alpha, beta):
    """CSR matrix of alpha Id + sum_a beta_a L_a for a [nz][ny][nx] grid."""
    nz, ny, nx = shape
    n = nz * ny * nx
    idx = np.arange(n).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.full(n, float(alpha))
    # (beta, slice of "lower" voxels, slice of their +1 neighbours) per axis
    pairs = (
        (beta[0], idx[:, :, :-1], idx[:, :, 1:]),
        (beta[1], idx[:, :-1, :], idx[:, 1:, :]),
        (beta[2], idx[:-1, :, :], idx[1:, :, :]),
    )
    for b, lo, hi in pairs:
        if b == 0.0 or lo.size == 0:
            continue
        lo = lo.ravel()
        hi = hi.ravel()
        rows += [lo, hi]
        cols += [hi, lo]
        vals += [np.full(lo.size, -b), np.full(lo.size, -b)]
        np.add.at(diag, lo, b)
        np.add.at(diag, hi, b)
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    A = sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(n, n),
    )
    A.sum_duplicates()
    return A


def closed_form_eigenvalues(shape, alpha, beta):
    """Eigenvalues of the assembled operator from the 1-D Neumann spectrum.

    The 3-point Neumann Laplacian on n points has eigenvalues
    2 - 2 cos(pi k / n), k = 0..n-1 (cosine eigenvectors); the operator is a
    Kronecker sum, so its spectrum is alpha + sum_a beta_a lambda_a(k_a)."""
    nz, ny, nx = shape
    lam = [2.0 - 2.0 * np.cos(np.pi * np.arange(m) / m) for m in (nx, ny, nz)]
    ev = (
        alpha
        + beta[0] * lam[0][None, None, :]
        + beta[1] * lam[1][None, :, None]
        + beta[2] * lam[2][:, None, None]
    )
    return np.sort(ev.ravel())
