"""Seeded synthetic grey-level video volume (input generation only).

Stand-in for the 1920x1080x742 video of Sec. 6, which is not available:
frames [t][y][x] of Gaussian blobs moving at constant velocity over a smooth
background, plus per-pixel sensor noise from the counter-based generator,
values clipped to [0, 255].  The sharp blob rims give large gradients, the
noise small ones: the two regimes the gradient-modulation filter separates.
"""

from dataclasses import dataclass

import numpy as np
import torch

from .stack import counter_normal


@dataclass(frozen=True)
class VideoSpec:
    nx: int
    ny: int
    nt: int
    seed: int = 13100416
    nblobs: int = 24
    noise: float = 2.0


VIDEO_CONFIGS = {
    "video1080": VideoSpec(1920, 1080, 742, 13100416),
}


class _Params:
    def __init__(self, spec: VideoSpec):
        rng = np.random.default_rng(spec.seed)
        nb = spec.nblobs
        self.cx = rng.uniform(0.0, spec.nx, nb)
        self.cy = rng.uniform(0.0, spec.ny, nb)
        self.vx = rng.uniform(-3.0, 3.0, nb)
        self.vy = rng.uniform(-2.0, 2.0, nb)
        # blob widths scale with the frame (7.5 .. 46 px at 1920x1080)
        self.sig = 1.5 + rng.uniform(0.004, 0.03, nb) * 0.5 * (spec.nx + spec.ny)
        self.amp = rng.uniform(-70.0, 90.0, nb)
        self.key = int(rng.integers(0, 2**31))


def _frame(spec, p, t, device):
    nx, ny = spec.nx, spec.ny
    x = torch.arange(nx, device=device, dtype=torch.float64)
    y = torch.arange(ny, device=device, dtype=torch.float64)
    cx = torch.as_tensor(np.mod(p.cx + p.vx * t, nx), device=device)
    cy = torch.as_tensor(np.mod(p.cy + p.vy * t, ny), device=device)
    s2 = torch.as_tensor(2.0 * p.sig**2, device=device)
    amp = torch.as_tensor(p.amp, device=device)
    gx = torch.exp(-((x[None, :] - cx[:, None]) ** 2) / s2[:, None])
    gy = torch.exp(-((y[None, :] - cy[:, None]) ** 2) / s2[:, None])
    img = (gy * amp[:, None]).T @ gx
    img = img + 100.0 + 40.0 * torch.sin(2.0 * np.pi * x / nx)[None, :] * torch.cos(2.0 * np.pi * y / ny)[:, None]
    idx = (torch.arange(ny, device=device, dtype=torch.int64)[:, None] * nx
           + torch.arange(nx, device=device, dtype=torch.int64)[None, :] + t * ny * nx)
    img = img + counter_normal(idx, p.key, spec.noise)
    return torch.clamp(img, 0.0, 255.0)


def make_video(spec: VideoSpec, device="cpu", dtype=torch.float64, t_range=None):
    """The [nt][ny][nx] volume of ``spec`` (or frames ``t_range``), cast to
    ``dtype`` frame by frame."""
    p = _Params(spec)
    t0, t1 = (0, spec.nt) if t_range is None else t_range
    out = torch.empty((t1 - t0, spec.ny, spec.nx), dtype=dtype, device=device)
    for t in range(t0, t1):
        out[t - t0] = _frame(spec, p, t, device).to(dtype)
    return out
