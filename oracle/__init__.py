"""CPU oracle of the differentiable Gaussian-splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports, calls, links
or executes this package: only tests/, the package-level smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path;
the only common dependency is the seeded input generator in synth/.

Contents (each module cites the passage it follows):
  keypath32  FP32 key path: culling, depth bits, opacity-aware tile rects
  project64  FP64 EWA projection and its exact derivative
  binning    (tile, depth) keys, sort, tile ranges
  composite  per-pixel front-to-back compositing (0.99 / 1/255 / 1e-4 rules)
  render     whole-view tiled and brute-force forward, exact FP64 backward
  smooth     FP64-decided brute-force render for finite differences
  sh         real spherical harmonics to degree 3
  se3        SE(3) exponential, left pose update
  sim3       Sim(3) correction of Gaussians and the lift of keyframe poses
  refine     exposure-compensated L1 gradient, opacity pruning
  ssim       SSIM term of the refinement loss and its gradient
  dedup      occupancy-aware deduplication of borrowed Gaussians
  mapping    isotropy and depth-normal terms of the mapping loss, seeding

Parity status: every function is pinned by tests under tests/ (closed
forms, invariants, brute force, library routines, finite differences).
"""
from .render import Settings, render_view, render_backward, render_pixels  # noqa: F401
