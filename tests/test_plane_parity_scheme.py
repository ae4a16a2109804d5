"""The block scheme of the plane-parity relaxation of the 27-point levels,
checked on the CPU before any kernel: an 8-colour Gauss-Seidel sweep (colour
(i mod 2) + 2 (j mod 2) + 4 (k mod 2), colours in increasing order) equals
two passes, even planes then odd planes, in which each block holds a tile of
its plane with a ring of four samples and the two neighbour planes, and runs
the four in-plane colours on the tile widened by 3, 2, 1 and 0 samples,
reading even planes' neighbours as they were before the sweep and odd planes'
as they are after it.  Reads at clamped indices resolve into the window; a
read outside the window, or of a window sample never loaded, fails the test.
The blocks run in random order, each plane's results only written to the
output buffer, as on the GPU.  The row arithmetic is a generic separable
27-point operator with random tridiagonal per-axis tables (no coupling past
the ends), rounded to FP32 after every update as FP32 storage is.
"""

import numpy as np
import pytest


def _tables(rng, n):
    M = [rng.uniform(0.1, 1, n), rng.uniform(1, 2, n), rng.uniform(0.1, 1, n)]
    K = [rng.uniform(-1, 0, n), rng.uniform(1, 3, n), rng.uniform(-1, 0, n)]
    M[0][0] = K[0][0] = 0.0
    M[2][-1] = K[2][-1] = 0.0
    return M, K


def _row(T, alpha, w, i, j, k, fetch, n):
    c = (i, j, k)
    m = [[T[a][0][d][c[a]] for d in range(3)] for a in range(3)]
    kk = [[T[a][1][d][c[a]] for d in range(3)] for a in range(3)]
    q = [[min(max(c[a] + d - 1, 0), n[a] - 1) for d in range(3)] for a in range(3)]
    s = 0.0
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                coef = ((alpha * m[0][dx] + w[0] * kk[0][dx]) * m[1][dy] * m[2][dz]
                        + m[0][dx] * (w[1] * kk[1][dy] * m[2][dz] + w[2] * m[1][dy] * kk[2][dz]))
                s += coef * fetch(q[0][dx], q[1][dy], q[2][dz])
    d = ((alpha * m[0][1] + w[0] * kk[0][1]) * m[1][1] * m[2][1]
         + m[0][1] * (w[1] * kk[1][1] * m[2][1] + w[2] * m[1][1] * kk[2][1]))
    return s, d


def _update(xc, bv, ax, d):
    return np.float32(xc + (bv - ax) / d) if d != 0 else np.float32(0)


def _colour_sweep(x, b, T, alpha, w):
    x = x.copy()
    nz, ny, nx = x.shape
    n = (nx, ny, nz)
    for col in range(8):
        ci, cj, ck = col & 1, (col >> 1) & 1, col >> 2
        for k in range(ck, nz, 2):
            for j in range(cj, ny, 2):
                for i in range(ci, nx, 2):
                    ax, d = _row(T, alpha, w, i, j, k, lambda a, bb, c: float(x[c, bb, a]), n)
                    x[k, j, i] = _update(float(x[k, j, i]), float(b[k, j, i]), ax, d)
    return x


def _parity_sweep(rng, x, b, T, alpha, w, HX, HY, HZ, R=4):
    nz, ny, nx = x.shape
    n = (nx, ny, nz)
    xin, xout = x.copy(), np.full_like(x, np.nan)
    WX, WY = HX + 2 * R, HY + 2 * R
    ntx, nty = (nx + HX - 1) // HX, (ny + HY - 1) // HY
    for ck in range(2):
        mz = (nz - ck + 1) // 2
        if mz == 0:
            continue
        xnb = xin if ck == 0 else xout
        blocks = [(t, c) for t in range(ntx * nty) for c in range((mz + HZ - 1) // HZ)]
        rng.shuffle(blocks)
        for t, ch in blocks:
            x0, y0 = (t % ntx) * HX, (t // ntx) * HY
            wx0, wy0 = x0 - R, y0 - R
            W = np.full((3, WY, WX), np.nan, dtype=np.float32)

            def load(sl, src, k):
                for wy in range(WY):
                    for wx in range(WX):
                        gx, gy = wx0 + wx, wy0 + wy
                        if 0 <= gx < nx and 0 <= gy < ny:
                            W[sl, wy, wx] = src[k, gy, gx]

            cen, lo, hi = 0, 1, 2
            kk0, kk1 = ch * HZ, min(ch * HZ + HZ, mz)
            for kk in range(kk0, kk1):
                k = 2 * kk + ck
                if kk > kk0:
                    lo, hi = hi, lo
                elif k > 0:
                    load(lo, xnb, k - 1)
                load(cen, xin, k)
                if k + 1 < nz:
                    load(hi, xnb, k + 1)
                ls = lo if k > 0 else cen
                hs = hi if k + 1 < nz else cen

                def fetch(qx, qy, qz):
                    sl = cen if qz == k else (ls if qz < k else hs)
                    assert 0 <= qy - wy0 < WY and 0 <= qx - wx0 < WX, "read outside the window"
                    v = W[sl, qy - wy0, qx - wx0]
                    assert not np.isnan(v), "read of a sample never loaded"
                    return float(v)

                for ph in range(4):
                    pi, pj, r = ph & 1, ph >> 1, 3 - ph
                    xa, xb = max(x0 - r, 0), min(x0 + HX + r, nx)
                    ya, yb = max(y0 - r, 0), min(y0 + HY + r, ny)
                    ia, ja = xa + ((xa & 1) ^ pi), ya + ((ya & 1) ^ pj)
                    nu = (xb - ia + 1) // 2 if xb > ia else 0
                    nv = (yb - ja + 1) // 2 if yb > ja else 0
                    for m in range(nu * nv):
                        v, u = divmod(m, nu)
                        i, j = ia + 2 * u, ja + 2 * v
                        ax, d = _row(T, alpha, w, i, j, k, fetch, n)
                        W[cen, j - wy0, i - wx0] = _update(float(W[cen, j - wy0, i - wx0]), float(b[k, j, i]), ax, d)
                for ty in range(HY):
                    for tx in range(HX):
                        gx, gy = x0 + tx, y0 + ty
                        if gx < nx and gy < ny:
                            xout[k, gy, gx] = W[cen, gy - wy0, gx - wx0]
    return xout


@pytest.mark.parametrize("shape,tile", [((5, 11, 13), (4, 2, 1)), ((7, 6, 3), (8, 4, 2)), ((4, 1, 10), (3, 5, 3)),
                                        ((1, 9, 17), (8, 4, 2)), ((2, 2, 2), (4, 2, 1))])
def test_parity_blocks_equal_colour_sweep(shape, tile):
    rng = np.random.default_rng(sum(shape) * 7 + tile[0])
    nz, ny, nx = shape
    T = [_tables(rng, nx), _tables(rng, ny), _tables(rng, nz)]
    x = rng.standard_normal(shape).astype(np.float32)
    b = rng.standard_normal(shape).astype(np.float32)
    ref = _colour_sweep(x, b, T, 0.3, (1.0, 0.7, 2.0))
    got = _parity_sweep(rng, x, b, T, 0.3, (1.0, 0.7, 2.0), *tile)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_a_thinner_ring_reads_outside_the_window():
    """With a ring of three the last colour's reads leave the window."""
    rng = np.random.default_rng(3)
    shape = (3, 12, 14)
    T = [_tables(rng, 14), _tables(rng, 12), _tables(rng, 3)]
    x = rng.standard_normal(shape).astype(np.float32)
    b = rng.standard_normal(shape).astype(np.float32)
    with pytest.raises(AssertionError):
        _parity_sweep(rng, x, b, T, 0.3, (1.0, 0.7, 2.0), 4, 4, 1, R=3)
