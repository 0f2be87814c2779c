"""MI355X-native PlenOctree renderer (arXiv 2103.14024).

Hand-written HIP kernels for gfx950 behind a C ABI (include/plenoctree.h,
libplenoctree.so); this package is the thin Python binding over it.  torch is
used for device memory and streams only.

    from paper_2103_14024_amd import Tree, Camera, render_camera
"""
from ._lib import PlenOctreeError, version  # noqa: F401
from .render import (AUX_DEPTH, AUX_SAMPLES, AUX_STEPS, AUX_T, AUX_WIDTH, Camera, Job,  # noqa: F401
                     camera_rays, device_errors, make_opts, render_batch, render_camera, render_camera_noalloc,
                     render_rays,
                     release_queues, reserve_queues, render_rays_backward, render_rays_backward_kept,
                     render_rays_differentiable, render_rays_keep, reset_device_errors,
                     traversal_stats)
from .tree import Tree, build_host, default_stride, validate_host  # noqa: F401
from . import optim, visibility  # noqa: F401
from .optim import Trainer, psnr  # noqa: F401
