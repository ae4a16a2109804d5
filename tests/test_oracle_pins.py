"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check ties one oracle
function to an independent derivation (closed-form spectrum, brute-force
energy, DCT diagonalisation, invariants stated in Sec. 3, the Fig. 2 example).
"""

import os

import numpy as np
import pytest

from oracle import assemble, grid, mgsteps, solvers

BETA = (1.0, 1.0, 4.0)
SHAPES = [(4, 5, 7), (1, 1, 9), (3, 1, 5), (8, 8, 4), (2, 3, 1), (5, 2, 3)]


def rnd(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


# ---------------------------------------------------------------- operator


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(0.0, BETA), (0.3, (1.0, 2.0, 0.5)), (0.01, (1.0, 1.0, 0.0))])
def test_apply_matches_assembled_stencil(shape, alpha, beta):
    x = rnd(shape)
    A = assemble.assemble(shape, alpha, beta)
    assert np.abs(A @ x.ravel() - grid.apply_A(x, alpha, beta).ravel()).max() < 1e-12


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("alpha,beta", [(0.0, BETA), (0.01, (1.0, 1.0, 0.1)), (2.0, (0.5, 3.0, 1.0))])
def test_spectrum_symmetry_definiteness(shape, alpha, beta):
    """Sec. 4 operator: symmetric, spectrum = alpha + sum beta_a (2 - 2cos(pi k/n))."""
    A = assemble.assemble(shape, alpha, beta).toarray()
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    ref = assemble.closed_form_eigenvalues(shape, alpha, beta)
    assert np.abs(ev - ref).max() < 1e-12 * max(1.0, ref.max())
    if alpha > 0:
        assert ev.min() > 0.0 and abs(ev.min() - alpha) < 1e-12
    else:
        # pure Neumann: one zero eigenvalue, constant eigenvector
        assert abs(ev[0]) < 1e-12 and ev[1] > 1e-6
        assert np.abs(A @ np.ones(A.shape[0])).max() < 1e-12


def _num_grad(f, x, h=1e-5):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        xp = x.copy()
        xm = x.copy()
        xp[i] += h
        xm[i] -= h
        g[i] = (f(xp) - f(xm)) / (2 * h)
    return g


@pytest.mark.parametrize("case", ["ad", "sp", "general"])
def test_solution_minimises_brute_force_energy(case):
    """The solved system is the Euler-Lagrange equation of the Sec. 4 energy:
    the energy, written as explicit sums over voxels and faces, has zero
    gradient at the oracle's solution and grows in every random direction."""
    shape = (3, 4, 5)
    I0 = rnd(shape, 1) * 10
    if case == "ad":
        alpha, beta, V = 0.0, BETA, None
        G = (grid.grad(I0, 0), grid.grad(I0, 1), None)
        x = solvers.ad_solve(I0, beta, method="cg")
    elif case == "sp":
        alpha, beta = 0.01, (1.0, 1.0, 0.0)
        V = rnd(shape, 2) * 10
        G = (grid.grad(I0, 0), grid.grad(I0, 1), None)
        x = solvers.sp_solve(I0, V, alpha, method="cg")
    else:
        alpha, beta = 0.2, (1.0, 0.5, 2.0)
        V = rnd(shape, 3)
        G = tuple(grid.grad(rnd(shape, 4 + c), c) for c in range(3))
        x = solvers.general_solve(V, G, alpha, beta, method="cg")
    f = lambda I: grid.energy(I, V, G, alpha, beta)  # noqa: E731
    g = _num_grad(f, x)
    assert np.abs(g).max() < 1e-5 * max(1.0, np.abs(x).max())
    e0 = f(x)
    for s in range(5):
        d = rnd(shape, 100 + s)
        if alpha == 0.0:
            d -= d.mean()  # the constant direction is flat for alpha = 0
        assert f(x + 1e-3 * d) > e0


# ------------------------------------------------------------------ solvers


@pytest.mark.parametrize("shape", SHAPES)
def test_dct_matches_dense_ad(shape):
    I0 = rnd(shape, 5) * 50
    a = solvers.ad_solve(I0, BETA, method="dense")
    b = solvers.ad_dct(I0, BETA)
    assert np.abs(a - b).max() < 1e-11 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("shape", SHAPES)
def test_dct_matches_dense_sp(shape):
    I0 = rnd(shape, 6) * 50
    I1 = rnd(shape, 7) * 50
    a = solvers.sp_solve(I0, I1, 0.01, method="dense")
    b = solvers.sp_dct(I0, I1, 0.01)
    assert np.abs(a - b).max() < 1e-9 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("shape", [(4, 5, 7), (8, 8, 4)])
@pytest.mark.parametrize("alpha,beta", [(0.0, BETA), (0.05, (1.0, 2.0, 0.3))])
def test_cg_and_dct_match_dense_general(shape, alpha, beta):
    b = rnd(shape, 8)
    if alpha == 0.0:
        b -= b.mean()
    xd = solvers.solve_dense(b, alpha, beta)
    xc, _, rr = solvers.solve_cg(b, alpha, beta)
    xf = solvers.dct_solve(b, alpha, beta)
    assert rr < 1e-12
    s = max(1.0, np.abs(xd).max())
    assert np.abs(xd - xc).max() < 1e-10 * s
    assert np.abs(xd - xf).max() < 1e-10 * s


def test_ad_gauge_and_slice_means():
    """Mean-preserving reading of Eq. (1); the (0, 0, m) frequencies have
    gain 0, so every slice of I1 (and of I2) carries the global mean."""
    I0 = rnd((6, 9, 11), 9) * 30 + 100
    I1 = solvers.ad_dct(I0, BETA)
    assert abs(I1.mean() - I0.mean()) < 1e-10
    sm = I1.mean(axis=(1, 2))
    assert np.abs(sm - I0.mean()).max() < 1e-10
    I2 = solvers.sp_dct(I0, I1, 0.01)
    assert np.abs(I2.mean(axis=(1, 2)) - I0.mean()).max() < 1e-10


# -------------------------------------------------------- invariants (Sec. 3)


def test_identity_when_target_gradients_are_own_gradients():
    """Target gradients equal to the input's own full gradient: the energy is
    minimised by the input itself."""
    I0 = rnd((4, 6, 5), 10) * 20
    G = tuple(grid.grad(I0, c) for c in range(3))
    x = solvers.general_solve(None, G, 0.0, BETA, method="cg", shape=I0.shape)
    assert np.abs((x - x.mean() + I0.mean()) - I0).max() < 1e-9
    x = solvers.general_solve(I0, G, 0.01, BETA, method="dense")
    assert np.abs(x - I0).max() < 1e-9
    # SP with I1 = I0 returns I0
    assert np.abs(solvers.sp_dct(I0, I0, 0.01) - I0).max() < 1e-10
    assert np.abs(solvers.sp_solve(I0, I0, 0.01, method="cg") - I0).max() < 1e-9


def test_no_diffusion_or_no_screening_is_identity():
    """Sec. 3.2.3: beta_z -> 0 or alpha -> 0 leaves the signal unchanged."""
    I0 = rnd((5, 7, 6), 11) * 20
    assert np.abs(solvers.ad_dct(I0, (1.0, 1.0, 0.0)) - I0).max() < 1e-10
    I1 = solvers.ad_dct(I0, BETA)
    I2 = solvers.sp_dct(I0, I1, 1e-12)
    # alpha -> 0: only the per-slice mean of I1 survives (the Laplacian fixes
    # everything else), so I2 -> I0 + (mean(I1_i) - mean(I0_i))
    shift = I1.mean(axis=(1, 2)) - I0.mean(axis=(1, 2))
    assert np.abs(I2 - (I0 + shift[:, None, None])).max() < 1e-6
    # alpha -> infinity: I2 -> I1
    assert np.abs(solvers.sp_dct(I0, I1, 1e12) - I1).max() < 1e-6


def test_z_constant_stack_is_fixed_point():
    f = rnd((1, 8, 9), 12) * 20
    I0 = np.repeat(f, 5, axis=0)
    assert np.abs(solvers.ad_dct(I0, BETA) - I0).max() < 1e-10
    assert np.abs(solvers.ad_solve(I0, BETA, method="cg") - I0).max() < 1e-9


def test_per_slice_offsets_removed_exactly():
    """I0 = f(x, y) + c(z): AD then SP returns f + mean(c) (the slice-to-slice
    discontinuities the method is built to remove, Sec. 1 / Sec. 3)."""
    f = rnd((1, 10, 12), 13) * 20
    c = np.random.default_rng(14).uniform(-20, 20, 6)
    I0 = f + c[:, None, None]
    I1 = solvers.ad_solve(I0, BETA, method="cg")
    I2 = solvers.sp_solve(I0, I1, 0.01, method="cg")
    assert np.abs(I2 - (f + c.mean())).max() < 1e-9


def test_combined_filter_on_single_frequency():
    """Sec. 3.2.3: AD followed by SP multiplies each frequency by
    F = (alpha * H + k2l2) / (alpha + k2l2), H = k2l2 / (k2l2 + bz m2),
    with the discrete eigenvalues 2 - 2 cos(pi k / n) in place of k^2."""
    nz, ny, nx = 8, 12, 10
    k, l, m = 3, 2, 5
    x = np.cos(np.pi * k * (np.arange(nx) + 0.5) / nx)
    y = np.cos(np.pi * l * (np.arange(ny) + 0.5) / ny)
    z = np.cos(np.pi * m * (np.arange(nz) + 0.5) / nz)
    I0 = z[:, None, None] * y[None, :, None] * x[None, None, :]
    lk = 2 - 2 * np.cos(np.pi * k / nx)
    ll = 2 - 2 * np.cos(np.pi * l / ny)
    lm = 2 - 2 * np.cos(np.pi * m / nz)
    alpha = 0.01
    H = (lk + ll) / (lk + ll + BETA[2] * lm)
    F = (alpha * H + lk + ll) / (alpha + lk + ll)
    I1 = solvers.ad_solve(I0, BETA, method="cg")
    assert np.abs(I1 - H * I0).max() < 1e-10
    I2 = solvers.sp_solve(I0, I1, alpha, method="cg")
    assert np.abs(I2 - F * I0).max() < 1e-10


def test_discrete_response_tends_to_paper_continuous_response():
    """At low frequency the discrete AD gain approaches the continuous
    response (bx k^2 + by l^2) / (bx k^2 + by l^2 + bz m^2) of Sec. 3.2.1."""
    n = 512
    for k, l, m in [(1, 2, 1), (3, 1, 2), (2, 2, 4)]:
        w = [np.pi * q / n for q in (k, l, m)]
        cont = (w[0] ** 2 + w[1] ** 2) / (w[0] ** 2 + w[1] ** 2 + 4.0 * w[2] ** 2)
        lam = [2 - 2 * np.cos(v) for v in w]
        disc = (lam[0] + lam[1]) / (lam[0] + lam[1] + 4.0 * lam[2])
        assert abs(disc - cont) < 1e-4


# ------------------------------------------------------------ multigrid steps


def _load_fig2():
    p = os.path.join(os.path.dirname(__file__), "golden", "fig2_aliasing.txt")
    rows = [ln for ln in open(p) if ln.strip() and not ln.startswith("#")]
    return [np.array([float(v) for v in r.split()]) for r in rows]


def test_fig2_aliasing_of_constant_restriction():
    s, Ls, R = _load_fig2()
    lap = grid.apply_A(s[None, None, :], 0.0, (1.0, 0.0, 0.0))[0, 0]
    assert np.array_equal(lap, Ls)
    r = mgsteps.restrict_sum(Ls[None, None, :], (2, 1, 1))[0, 0]
    assert np.array_equal(r, R)


def _rb_brute(x, b, alpha, w):
    """Gauss-Seidel written as loops: all red voxels (any order, they do not
    touch each other), then all black voxels."""
    x = x.copy()
    nz, ny, nx = x.shape
    for colour in (0, 1):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    if (i + j + k) % 2 != colour:
                        continue
                    s, d = 0.0, alpha
                    for (dk, dj, di, ww) in ((0, 0, 1, w[0]), (0, 0, -1, w[0]), (0, 1, 0, w[1]),
                                             (0, -1, 0, w[1]), (1, 0, 0, w[2]), (-1, 0, 0, w[2])):
                        kk, jj, ii = k + dk, j + dj, i + di
                        if 0 <= kk < nz and 0 <= jj < ny and 0 <= ii < nx:
                            s += ww * x[kk, jj, ii]
                            d += ww
                    x[k, j, i] = (b[k, j, i] + s) / d if d > 0 else 0.0
    return x


@pytest.mark.parametrize("shape", [(3, 4, 5), (1, 6, 7), (4, 1, 1), (1, 1, 1)])
@pytest.mark.parametrize("alpha,w", [(0.0, BETA), (0.04, (2.0, 2.0, 2.0)), (1.5, (1.0, 1.0, 0.0))])
def test_rb_sweep_matches_loops_and_fixes_solution(shape, alpha, w):
    x = rnd(shape, 20)
    b = rnd(shape, 21)
    if alpha == 0.0:
        b -= b.mean()
    out = mgsteps.rb_sweep(x, b, alpha, w)
    assert np.abs(out - _rb_brute(x, b, alpha, w)).max() < 1e-12
    if alpha > 0:  # the exact solution is a fixed point
        xs = solvers.solve_dense(b, alpha, w)
        assert np.abs(mgsteps.rb_sweep(xs, b, alpha, w) - xs).max() < 1e-10


def test_rb_sweeps_converge_to_solution():
    shape = (4, 6, 6)
    b = rnd(shape, 22)
    x = np.zeros(shape)
    for _ in range(400):
        x = mgsteps.rb_sweep(x, b, 0.5, (1.0, 1.0, 2.0))
    assert np.abs(x - solvers.solve_dense(b, 0.5, (1.0, 1.0, 2.0))).max() < 1e-10


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 7, 3), (1, 9, 9), (3, 1, 1)])
@pytest.mark.parametrize("c", [(2, 2, 2), (1, 1, 2), (2, 2, 1)])
def test_transfer_operators(shape, c):
    r = rnd(shape, 23)
    rc = mgsteps.restrict_sum(r, c)
    assert rc.shape == mgsteps.coarse_shape(shape, c)
    assert abs(rc.sum() - r.sum()) < 1e-10
    # restriction is the transpose of constant up-sampling
    e = rnd(rc.shape, 24)
    lhs = float((rc * e).sum())
    rhs = float((r * mgsteps.prolong_constant(e, shape, c)).sum())
    assert abs(lhs - rhs) < 1e-10
    # brute-force restriction
    ref = np.zeros(rc.shape)
    for k in range(shape[0]):
        for j in range(shape[1]):
            for i in range(shape[2]):
                ref[k // c[2], j // c[1], i // c[0]] += r[k, j, i]
    assert np.abs(ref - rc).max() < 1e-12
    # trilinear: reproduces constants everywhere
    ones = mgsteps.prolong_trilinear(np.ones(rc.shape), shape, c)
    assert np.abs(ones - 1.0).max() < 1e-14


def test_trilinear_reproduces_linear_in_interior():
    """Cell-centred interpolation is exact for a linear function away from
    the boundary mirror cells: coarse cell I has centre 2I + 1/2."""
    nf = 16
    nc = 8
    ec = 3.0 * (2 * np.arange(nc) + 0.5) + 1.0
    ef = mgsteps.prolong_trilinear(ec[None, None, :], (1, 1, nf), (2, 1, 1))[0, 0]
    exact = 3.0 * np.arange(nf) + 1.0
    assert np.abs(ef[1:-1] - exact[1:-1]).max() < 1e-12


def test_relative_residual_definition():
    shape = (3, 4, 5)
    b = rnd(shape, 25)
    assert abs(mgsteps.relative_residual(np.zeros(shape), b, 0.1, BETA) - 1.0) < 1e-15
    xs = solvers.solve_dense(b, 0.1, BETA)
    assert mgsteps.relative_residual(xs, b, 0.1, BETA) < 1e-13
