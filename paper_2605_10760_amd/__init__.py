"""MI355X (gfx950) differentiable 3D Gaussian-splatting rasterizer.

The hot path is HIP kernels behind the C ABI in include/gsr.h (libgsr.so);
this package only marshals PyTorch tensors into those calls.
"""
from ._lib import GsrError, load  # noqa: F401
from .rasterizer import (Adam, Rasterizer, SceneTensors, ViewTensors, apply_pose_delta,  # noqa: F401
                         autotune, dedup, iso_grad, l1_loss_grad, normal_loss_grad, pairs_of,
                         prune, rasterize, seed, seed_noalloc, sim3_gaussians, sim3_views, ssim_grad)
from .optim import MAP_WEIGHTS, REFINE_WEIGHTS, Optimizer, Rates, Weights, refine  # noqa: F401
