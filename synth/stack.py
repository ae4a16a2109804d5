"""Synthetic voxel stacks and slice batches (torch, FP64, any device).

All random parameters (blob centres, widths and amplitudes, per-slice gains,
offsets and jitters, Voronoi sites, slice sizes) are drawn on the host with
``numpy.random.default_rng(seed)``; the per-voxel noise is a counter-based
hash of (seed, voxel index), so a stack is the same whether it is evaluated on
the CPU or on a GPU (up to the last bit of exp/log/cos).

Recipe for slice z of an (nx, ny, nz) stack:

    I0[z] = g_z * (blobs_z + membranes_z) + o_z + N(0, 2^2)

* blobs_z: 20 Gaussians shared by all slices, centre U[0,nx) x U[0,ny),
  sigma U(sigma_lo, sigma_hi), amplitude U(0, 255); in every slice each centre
  moves by its own sub-pixel jitter U(-0.5, 0.5)^2.
* membranes_z (optional): one Voronoi site uniform in each 64 x 64 px cell,
  jittered per slice like the blob centres; a pixel whose distance to the
  bisector of its two nearest sites is below 1 px (a 2 px band) gets -60.
* g_z ~ U(0.8, 1.2), o_z ~ U(-20, 20).
"""

from dataclasses import dataclass

import numpy as np
import torch

_M32 = 0xFFFFFFFF
_MIX = 0x45D9F3B  # < 2^27, so 32-bit x 32-bit products stay inside int64


@dataclass(frozen=True)
class StackSpec:
    nx: int
    ny: int
    nz: int
    sigma: tuple = (2.0, 8.0)
    membranes: bool = False
    seed: int = 13100411
    nblobs: int = 20


# Workloads (seed for workload k, 1-based: 13100410 + k).
CONFIGS = {
    "stack64": StackSpec(64, 64, 16, (2.0, 8.0), False, 13100411),
    "stack1k": StackSpec(1024, 1024, 128, (4.0, 40.0), True, 13100412),
    "stack4k": StackSpec(4096, 4096, 256, (4.0, 40.0), True, 13100413),
    "stack2k": StackSpec(2048, 2048, 64, (4.0, 40.0), True, 13100415),
}


def _mix32(x):
    x = x & _M32
    x = x ^ (x >> 16)
    x = (x * _MIX) & _M32
    x = x ^ (x >> 16)
    x = (x * _MIX) & _M32
    x = x ^ (x >> 16)
    return x


def counter_normal(index, key, std=2.0):
    """N(0, std^2) samples from a counter-based hash of an int64 index tensor
    (Box-Muller on two independent 32-bit hashes)."""
    lo = index & _M32
    hi = index >> 32
    h1 = _mix32(lo ^ _mix32(hi ^ (key & _M32)))
    h2 = _mix32(lo ^ _mix32(hi ^ ((key * 7 + 0x2545F491) & _M32)))
    u1 = (h1.to(torch.float64) + 0.5) / 4294967296.0
    u2 = (h2.to(torch.float64) + 0.5) / 4294967296.0
    return std * torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * np.pi * u2)


class _Params:
    """Host-side random parameters of one stack."""

    def __init__(self, spec: StackSpec):
        rng = np.random.default_rng(spec.seed)
        nb = spec.nblobs
        self.cx = rng.uniform(0.0, spec.nx, nb)
        self.cy = rng.uniform(0.0, spec.ny, nb)
        self.sig = rng.uniform(spec.sigma[0], spec.sigma[1], nb)
        self.amp = rng.uniform(0.0, 255.0, nb)
        self.jit = rng.uniform(-0.5, 0.5, (spec.nz, nb, 2))
        self.gain = rng.uniform(0.8, 1.2, spec.nz)
        self.off = rng.uniform(-20.0, 20.0, spec.nz)
        self.key = int(rng.integers(0, 2**31))
        self.ncx = -(-spec.nx // 64)
        self.ncy = -(-spec.ny // 64)
        if spec.membranes:
            gy, gx = np.meshgrid(np.arange(self.ncy), np.arange(self.ncx), indexing="ij")
            self.site_x = (gx + rng.uniform(0.0, 1.0, gx.shape)) * 64.0
            self.site_y = (gy + rng.uniform(0.0, 1.0, gy.shape)) * 64.0
            self.site_jit = rng.uniform(-0.5, 0.5, (spec.nz, self.ncy, self.ncx, 2))


def _membranes(p, z, ny, nx, device):
    """-60 on a 2 px band around the Voronoi edges of slice z, else 0."""
    big = 1e30
    sx = np.full((p.ncy + 4, p.ncx + 4), big)
    sy = np.full((p.ncy + 4, p.ncx + 4), big)
    sx[2:-2, 2:-2] = p.site_x + p.site_jit[z, :, :, 0]
    sy[2:-2, 2:-2] = p.site_y + p.site_jit[z, :, :, 1]
    sx = torch.as_tensor(sx, device=device)
    sy = torch.as_tensor(sy, device=device)
    y = torch.arange(ny, device=device, dtype=torch.float64)[:, None]
    x = torch.arange(nx, device=device, dtype=torch.float64)[None, :]
    cyi = (torch.arange(ny, device=device) // 64)[:, None]
    cxi = (torch.arange(nx, device=device) // 64)[None, :]
    inf = torch.full((ny, nx), float("inf"), device=device, dtype=torch.float64)
    d1, d2 = inf.clone(), inf.clone()
    s1x, s1y = torch.zeros_like(inf), torch.zeros_like(inf)
    s2x, s2y = torch.zeros_like(inf), torch.zeros_like(inf)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            qx = sx[cyi + dy + 2, cxi + dx + 2]
            qy = sy[cyi + dy + 2, cxi + dx + 2]
            d = (qx - x) ** 2 + (qy - y) ** 2
            first = d < d1
            second = (~first) & (d < d2)
            # demote the old best where a new best arrives
            d2 = torch.where(first, d1, torch.where(second, d, d2))
            s2x = torch.where(first, s1x, torch.where(second, qx, s2x))
            s2y = torch.where(first, s1y, torch.where(second, qy, s2y))
            d1 = torch.where(first, d, d1)
            s1x = torch.where(first, qx, s1x)
            s1y = torch.where(first, qy, s1y)
    sep = torch.sqrt((s2x - s1x) ** 2 + (s2y - s1y) ** 2)
    dist = (d2 - d1) / (2.0 * sep)
    return torch.where(dist < 1.0, -60.0, 0.0).to(torch.float64)


def _slice(spec, p, z, device):
    ny, nx = spec.ny, spec.nx
    x = torch.arange(nx, device=device, dtype=torch.float64)
    y = torch.arange(ny, device=device, dtype=torch.float64)
    cx = torch.as_tensor(p.cx + p.jit[z, :, 0], device=device)
    cy = torch.as_tensor(p.cy + p.jit[z, :, 1], device=device)
    s2 = torch.as_tensor(2.0 * p.sig**2, device=device)
    amp = torch.as_tensor(p.amp, device=device)
    gx = torch.exp(-((x[None, :] - cx[:, None]) ** 2) / s2[:, None])  # [nb][nx]
    gy = torch.exp(-((y[None, :] - cy[:, None]) ** 2) / s2[:, None])  # [nb][ny]
    img = (gy * amp[:, None]).T @ gx  # separable sum of blobs, [ny][nx]
    if spec.membranes:
        img = img + _membranes(p, z, ny, nx, device)
    img = p.gain[z] * img + p.off[z]
    idx = (
        torch.arange(ny, device=device, dtype=torch.int64)[:, None] * nx
        + torch.arange(nx, device=device, dtype=torch.int64)[None, :]
        + z * ny * nx
    )
    return img + counter_normal(idx, p.key)


def make_stack(spec: StackSpec, device="cpu", dtype=torch.float64, z_range=None):
    """The [nz][ny][nx] stack of ``spec`` (or the slices ``z_range``), cast
    (round to nearest even) to ``dtype`` slice by slice."""
    p = _Params(spec)
    z0, z1 = (0, spec.nz) if z_range is None else z_range
    out = torch.empty((z1 - z0, spec.ny, spec.nx), dtype=dtype, device=device)
    for z in range(z0, z1):
        out[z - z0] = _slice(spec, p, z, device).to(dtype)
    return out


def quantize(t, dtype):
    """Round to ``dtype`` (nearest even) and return the exact float64 value of
    the rounded numbers, which is what both solvers see as input."""
    return t.to(dtype).to(torch.float64)


def make_slice_batch(nslices=2048, lo=256, hi=2048, seed=13100414, device="cpu",
                     dtype=torch.float32, sizes_only=False):
    """Independent 2-D slices of uneven size for the batched screened Poisson.

    Sizes: w, h independently log-uniform in [lo, hi] (rounded); alpha_i ~
    U(0.001, 0.1).  Slice i is a one-slice stack (sigma 4-40, membranes)
    with seed ``seed + 7919 * (i + 1)``; its value target I1_i is I0_i with a
    fresh gain U(0.8, 1.2), offset U(-20, 20) and a linear ramp of up to
    +-20 in each direction.  Slices are packed back to back (pitch = width).

    Returns dict(w, h, alpha, offset, I0, I1) with numpy metadata and flat
    torch tensors of ``dtype``."""
    rng = np.random.default_rng(seed)
    w = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), nslices))).astype(np.int64)
    h = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), nslices))).astype(np.int64)
    alpha = rng.uniform(0.001, 0.1, nslices)
    gain = rng.uniform(0.8, 1.2, nslices)
    off = rng.uniform(-20.0, 20.0, nslices)
    ramp = rng.uniform(-20.0, 20.0, (nslices, 2))
    offset = np.concatenate([[0], np.cumsum(w * h)[:-1]]).astype(np.int64)
    meta = dict(w=w, h=h, alpha=alpha, offset=offset)
    if sizes_only:
        return meta
    total = int((w * h).sum())
    I0 = torch.empty(total, dtype=dtype, device=device)
    I1 = torch.empty(total, dtype=dtype, device=device)
    for i in range(nslices):
        spec = StackSpec(int(w[i]), int(h[i]), 1, (4.0, 40.0), True, seed + 7919 * (i + 1))
        s0 = make_stack(spec, device=device)[0]
        xr = torch.linspace(-1.0, 1.0, int(w[i]), device=device, dtype=torch.float64)
        yr = torch.linspace(-1.0, 1.0, int(h[i]), device=device, dtype=torch.float64)
        s1 = gain[i] * s0 + off[i] + ramp[i, 0] * xr[None, :] + ramp[i, 1] * yr[:, None]
        n = int(w[i] * h[i])
        I0[offset[i]:offset[i] + n] = s0.reshape(-1).to(dtype)
        I1[offset[i]:offset[i] + n] = s1.reshape(-1).to(dtype)
    meta.update(I0=I0, I1=I1)
    return meta
