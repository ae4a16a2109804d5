"""Seeded synthetic EM-like stacks (input generation only).

This package holds no arithmetic of the solver: it only draws the inputs that
both the HIP path and the FP64 oracle consume.  The paper's Mouse S1 stack and
its video example are not available, so these stacks stand in for them:
Gaussian blobs shared across slices with sub-pixel jitter, a jittered-lattice
Voronoi membrane pattern, a per-slice gain and offset (the slice-to-slice
discontinuities the method removes) and additive Gaussian noise.  A
grey-level video volume (moving blobs plus noise) stands in for the video
of the paper's gradient-modulation example.
"""

from .stack import (  # noqa: F401
    StackSpec,
    CONFIGS,
    make_stack,
    make_slice_batch,
    quantize,
    counter_normal,
)
from .video import VideoSpec, VIDEO_CONFIGS, make_video  # noqa: F401
