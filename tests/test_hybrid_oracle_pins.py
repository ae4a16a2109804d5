"""Pins of the Hybrid-discretisation steps (Sec. 4.2) of the oracle.

The Galerkin coarse operators built from per-axis 1-D tables are checked
against P^T A P formed from the explicitly assembled finest matrix; the
separable operator application against the dense Kronecker operator; the
8-colour sweep against a sample-by-sample loop over the dense matrix; the
prolongation against the B-spline stencil written out by hand.
"""

import numpy as np
import pytest

from oracle import assemble, hybrid, mgsteps

CASES = [((3, 4, 5), (True, True, True)), ((4, 3, 6), (False, False, True)), ((1, 5, 7), (True, True, False)),
         ((2, 2, 2), (True, True, True)), ((5, 1, 4), (True, False, True))]


def rnd(shape, seed=0):
    return np.random.default_rng(seed).standard_normal(shape)


def mats_of(shape, halved, level):
    nz, ny, nx = shape
    return [hybrid.level_tables(n, [h] * level)[level] for n, h in zip((nx, ny, nz), halved)]


@pytest.mark.parametrize("n", [1, 2, 5, 6, 9])
def test_prolongation_is_the_bspline_nesting(n):
    P = hybrid.prolong_1d(n, True)
    assert P.shape == (n, (n + 1) // 2)
    assert np.allclose(P @ np.ones(P.shape[1]), 1.0)  # constants stay constant
    for c in range(P.shape[1]):
        col = P[:, c]
        want = np.zeros(n)
        want[2 * c] = 1.0
        if 2 * c - 1 >= 0:
            want[2 * c - 1] = 0.5
        if 2 * c + 1 < n:
            want[2 * c + 1] = 0.5 if c + 1 < P.shape[1] else 1.0
        assert np.array_equal(col, want), (n, c)
    # a linear function on the coarse samples is interpolated exactly inside
    if n % 2 == 1:
        e = np.arange(P.shape[1], dtype=float)
        assert np.allclose(P @ e, np.arange(n) / 2.0)


@pytest.mark.parametrize("shape,halved", CASES)
@pytest.mark.parametrize("alpha,w", [(0.0, (1.0, 1.0, 4.0)), (0.01, (1.0, 0.5, 2.0))])
def test_galerkin_tables_match_assembled_product(shape, halved, alpha, w):
    A0 = assemble.assemble(shape, alpha, w).toarray()
    P = [hybrid.prolong_1d(n, h) for n, h in zip(shape[::-1], halved)]
    P3 = np.kron(P[2], np.kron(P[1], P[0]))
    want = P3.T @ A0 @ P3
    got = hybrid.kron_operator(mats_of(shape, halved, 1), alpha, w)
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
    # and the level-0 tables reproduce the 7-point operator itself
    assert np.abs(hybrid.kron_operator(mats_of(shape, halved, 0), alpha, w) - A0).max() <= 1e-13


@pytest.mark.parametrize("shape,halved", CASES)
@pytest.mark.parametrize("level", [0, 1, 2])
def test_separable_apply_and_diagonal(shape, halved, level):
    mats = mats_of(shape, halved, level)
    n = tuple(m[0].shape[0] for m in mats)[::-1]
    A = hybrid.kron_operator(mats, 0.03, (1.0, 2.0, 0.5))
    x = rnd(n, 1)
    assert np.abs(hybrid.apply(x, mats, 0.03, (1.0, 2.0, 0.5)).ravel() - A @ x.ravel()).max() <= 1e-12
    assert np.abs(hybrid.diagonal(n, mats, 0.03, (1.0, 2.0, 0.5)).ravel() - np.diag(A)).max() <= 1e-13


@pytest.mark.parametrize("shape,halved", CASES)
def test_colours_are_uncoupled_and_sweep_matches_loops(shape, halved):
    mats = mats_of(shape, halved, 1)
    n = tuple(m[0].shape[0] for m in mats)[::-1]
    alpha, w = 0.02, (1.0, 1.0, 4.0)
    A = hybrid.kron_operator(mats, alpha, w)
    col = hybrid.colour(n).ravel()
    for u in range(A.shape[0]):
        for v in range(A.shape[0]):
            if u != v and col[u] == col[v]:
                assert A[u, v] == 0.0
    x, b = rnd(n, 2), rnd(n, 3)
    assert np.abs(hybrid.gs8_sweep(x, b, mats, alpha, w) - hybrid.gs8_sweep_loops(x, b, A)).max() <= 1e-12
    xs = np.linalg.solve(A, b.ravel()).reshape(n)
    assert np.abs(hybrid.gs8_sweep(xs, b, mats, alpha, w) - xs).max() <= 1e-10


@pytest.mark.parametrize("shape,halved", CASES)
def test_transfers_are_adjoint(shape, halved):
    P = hybrid.transfer_mats(shape, halved)
    nc = tuple(p.shape[1] for p in P)[::-1]
    r, e = rnd(shape, 4), rnd(nc, 5)
    assert abs(np.sum(hybrid.restrict(r, P) * e) - np.sum(r * hybrid.prolong(e, P))) <= 1e-12
    P3 = np.kron(P[2], np.kron(P[1], P[0]))
    assert np.abs(hybrid.prolong(e, P).ravel() - P3 @ e.ravel()).max() <= 1e-13
    assert mgsteps.coarse_shape(shape, tuple(2 if h else 1 for h in halved)) == nc


def test_two_grid_cycle_contracts():
    """A two-grid cycle (sweep, Galerkin coarse solve, prolongation, sweep)
    with these steps reduces the error of the AD-type system."""
    shape, halved, alpha, w = (4, 6, 8), (True, True, True), 0.0, (1.0, 1.0, 4.0)
    m0, m1 = mats_of(shape, halved, 0), mats_of(shape, halved, 1)
    A0, A1 = hybrid.kron_operator(m0, alpha, w), hybrid.kron_operator(m1, alpha, w)
    P = hybrid.transfer_mats(shape, halved)
    b = rnd(shape, 6)
    b -= b.mean()
    xs = np.linalg.lstsq(A0, b.ravel(), rcond=None)[0].reshape(shape)
    x = np.zeros(shape)
    err0 = np.linalg.norm((x - xs) - (x - xs).mean())
    for _ in range(3):
        x = hybrid.gs8_sweep(x, b, m0, alpha, w)
        r = hybrid.restrict(b - hybrid.apply(x, m0, alpha, w), P)
        ec = np.linalg.lstsq(A1, r.ravel(), rcond=None)[0].reshape(r.shape)
        x = hybrid.gs8_sweep(x + hybrid.prolong(ec, P), b, m0, alpha, w)
    err = np.linalg.norm((x - xs) - (x - xs).mean())
    assert err < 0.1 * err0  # about 0.3 per two-grid cycle here
