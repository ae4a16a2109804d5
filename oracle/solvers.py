"""Solutions of the paper's linear systems (FP64, CPU).

Test infrastructure only (see the package header).

The multigrid of Sec. 4.1 reaches, up to rounding, the unique minimiser of the
discrete quadratic energy, so the oracle computes that minimiser directly:

* ``solve_dense``  assembled matrix + numpy dense solve (tiny grids);
* ``solve_cg``     conjugate gradients on the matrix-free operator, to a
                   relative residual of 1e-13 (any size that fits in RAM);
* ``dct_*``        the exact diagonalisation by the orthonormal DCT-II, the
                   discrete form of the frequency-space analysis of Sec. 3.2
                   (eigenvalues 2 - 2 cos(pi k / n) per axis instead of the
                   continuous k^2).

The anisotropic diffusion (Eq. (1)) has alpha = 0 and a pure-Neumann operator
whose null space is the constant field, and the frequency response of
Sec. 3.2.1 is undefined (0/0) at the zero frequency.  Reading used here: the
solution is the one with mean(I1) = mean(I0), i.e. unit gain at the zero
frequency; every other (0, 0, m) frequency has gain 0.
"""

import numpy as np
import scipy.fft as sfft

from . import grid
from .assemble import assemble

# ---------------------------------------------------------------------------
# generic system  (alpha + sum_a beta_a L_a) x = b


def solve_dense(b, alpha, beta):
    """Dense direct solve of the assembled system.  alpha == 0: the minimum
    norm (mean-zero) solution of the consistent part of b."""
    b = grid.as3d(b)
    A = assemble(b.shape, alpha, beta).toarray()
    if alpha > 0.0:
        x = np.linalg.solve(A, b.ravel())
    else:
        x = np.linalg.lstsq(A, b.ravel(), rcond=1e-12)[0]
    return x.reshape(b.shape)


def solve_cg(b, alpha, beta, rtol=1e-13, maxiter=100000, x0=None):
    """Jacobi-free plain conjugate gradients on the matrix-free operator.

    For alpha == 0 the right-hand side is projected onto the mean-zero
    subspace and the iterate is kept there (the operator is PSD with the
    constant null space).  Returns (x, iterations, relative residual)."""
    b = grid.as3d(b).copy()
    singular = alpha == 0.0
    if singular:
        b -= b.mean()
    x = np.zeros_like(b) if x0 is None else grid.as3d(x0).copy()
    if singular:
        x -= x.mean()
    r = b - grid.apply_A(x, alpha, beta)
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return x, 0, 0.0
    p = r.copy()
    rr = float(np.vdot(r, r))
    it = 0
    while it < maxiter and np.sqrt(rr) > rtol * nb:
        Ap = grid.apply_A(p, alpha, beta)
        a = rr / float(np.vdot(p, Ap))
        x += a * p
        r -= a * Ap
        if singular:
            r -= r.mean()
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    relres = np.linalg.norm(b - grid.apply_A(x, alpha, beta)) / nb
    return x, it, relres


def _lams(shape):
    """Per-axis Neumann eigenvalues broadcast to [nz][ny][nx] (x, y, z)."""
    nz, ny, nx = shape
    lx = (2.0 - 2.0 * np.cos(np.pi * np.arange(nx) / nx))[None, None, :]
    ly = (2.0 - 2.0 * np.cos(np.pi * np.arange(ny) / ny))[None, :, None]
    lz = (2.0 - 2.0 * np.cos(np.pi * np.arange(nz) / nz))[:, None, None]
    return lx, ly, lz


def dct_solve(b, alpha, beta):
    """Exact solve by DCT-II diagonalisation (alpha == 0: mean-zero solution)."""
    b = grid.as3d(b)
    lx, ly, lz = _lams(b.shape)
    den = alpha + beta[0] * lx + beta[1] * ly + beta[2] * lz
    bh = sfft.dctn(b, type=2, norm="ortho")
    with np.errstate(divide="ignore", invalid="ignore"):
        xh = np.where(den > 0.0, bh / np.where(den > 0.0, den, 1.0), 0.0)
    return sfft.idctn(xh, type=2, norm="ortho")


# ---------------------------------------------------------------------------
# the two systems of the paper


def ad_dct(I0, beta):
    """Anisotropic diffusion, Eq. (1), in closed form (Sec. 3.2.1).

    Gain (bx lx + by ly) / (bx lx + by ly + bz lz) per DCT frequency; the
    zero frequency keeps gain 1 (mean-preserving reading).  Where the
    denominator vanishes at a non-zero frequency (beta_z = 0) the gain is 1:
    with no cross-slice term the input already minimises the energy."""
    I0 = grid.as3d(I0)
    lx, ly, lz = _lams(I0.shape)
    num = beta[0] * lx + beta[1] * ly + 0.0 * lz
    den = num + beta[2] * lz
    gain = np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 1.0)
    h = sfft.dctn(I0, type=2, norm="ortho")
    return sfft.idctn(gain * h, type=2, norm="ortho")


def sp_dct(I0, I1, alpha, beta_xy=(1.0, 1.0)):
    """Per-slice screened Poisson, Eq. (2), in closed form (Sec. 3.2.2).

    Per slice and in-slice DCT frequency:
    (alpha I1^ + (bx lx + by ly) I0^) / (alpha + bx lx + by ly)."""
    I0 = grid.as3d(I0)
    I1 = grid.as3d(I1)
    lx, ly, _ = _lams(I0.shape)
    lxy = beta_xy[0] * lx + beta_xy[1] * ly
    h0 = sfft.dctn(I0, type=2, norm="ortho", axes=(1, 2))
    h1 = sfft.dctn(I1, type=2, norm="ortho", axes=(1, 2))
    h2 = (alpha * h1 + lxy * h0) / (alpha + lxy)
    return sfft.idctn(h2, type=2, norm="ortho", axes=(1, 2))


def ad_solve(I0, beta, method="cg", rtol=1e-13):
    """Anisotropic diffusion by an iterative/direct solve of Eq. (1) plus the
    gauge mean(I1) = mean(I0).  method: 'cg', 'dense' or 'dct'."""
    I0 = grid.as3d(I0)
    if method == "dct":
        return ad_dct(I0, beta)
    b = grid.rhs_ad(I0, beta)
    if method == "dense":
        x = solve_dense(b, 0.0, beta)
    else:
        x = solve_cg(b, 0.0, beta, rtol=rtol)[0]
    return x - x.mean() + I0.mean()


def sp_solve(I0, I1, alpha, beta_xy=(1.0, 1.0), method="cg", rtol=1e-13):
    """Per-slice screened Poisson, Eq. (2).  method: 'cg', 'dense' or 'dct'.

    The consolidated form with pi = Diag(1,1,0) has no cross-slice coupling,
    so one 3-D solve with beta_z = 0 equals the per-slice solves."""
    I0 = grid.as3d(I0)
    if method == "dct":
        return sp_dct(I0, I1, alpha, beta_xy)
    b = grid.rhs_sp(I0, I1, alpha, beta_xy)
    beta = (beta_xy[0], beta_xy[1], 0.0)
    if method == "dense":
        return solve_dense(b, alpha, beta)
    return solve_cg(b, alpha, beta, rtol=rtol)[0]


def general_solve(V, G, alpha, beta, method="cg", shape=None, rtol=1e-13):
    """The general screened gradient-domain system of Sec. 4."""
    b = grid.rhs_general(V, G, alpha, beta, shape=shape)
    if method == "dense":
        return solve_dense(b, alpha, beta)
    if method == "dct":
        return dct_solve(b, alpha, beta)
    return solve_cg(b, alpha, beta, rtol=rtol)[0]
