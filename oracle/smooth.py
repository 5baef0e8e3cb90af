"""Brute-force FP64 render used for finite differences (test infrastructure
only).

Unlike render.py this path takes FP64 parameters and decides everything in
FP64: a Gaussian is kept when its camera depth exceeds z_near, its 2D
covariance has a positive determinant and 255*sigma > 1; kept Gaussians are
walked in ascending (FP64 depth, index) order for every pixel.  Gaussians
whose binning box misses the screen have alpha < 1/255 everywhere, so they are
skipped by the per-pixel rule and need no separate test.  This makes the
rendered outputs a piecewise-smooth function of the FP64 parameters whose
pieces are fixed by the decision signature returned alongside.
"""
from __future__ import annotations

import numpy as np

from .composite import composite, pixel_grid
from .project64 import project
from .se3 import apply_left


def render_smooth(params, sh_degree, viewmat, intrin, width, height, z_near=0.2,
                  bg=(0.0, 0.0, 0.0), pose_delta=None):
    """params: dict of FP64 arrays means, log_scales, quats, opacity_logits,
    colors.  Returns (color [3,H,W], depth, alpha, signature)."""
    vm = np.asarray(viewmat, np.float64).reshape(3, 4)
    if pose_delta is not None:
        vm = apply_left(np.asarray(pose_delta, np.float64), vm)
    pr = project(params["means"], params["log_scales"], params["quats"],
                 params["opacity_logits"], params["colors"], sh_degree, vm,
                 intrin, width, height)
    det = pr["S2"][:, 0, 0] * pr["S2"][:, 1, 1] - pr["S2"][:, 0, 1] ** 2
    keep = (pr["z"] > z_near) & (det > 0) & (255.0 * pr["sigma"] > 1.0)
    idx = np.nonzero(keep)[0]
    order = idx[np.lexsort((idx, pr["z"][idx]))]
    rec = dict(u=pr["u"], v=pr["v"], A=pr["conic"][:, 0], B=pr["conic"][:, 1],
               C=pr["conic"][:, 2], sigma=pr["sigma"], z=pr["z"], color=pr["color"])
    color = np.zeros((3, height, width))
    depth = np.zeros((height, width))
    alpha = np.zeros((height, width))
    sig_parts = [tuple(order)]
    for y in range(height):
        xx, yy, sx, sy = pixel_grid(0, y, width, y + 1)
        r = composite(sx, sy, rec, order, bg, keep=True)
        color[:, yy, xx] = r["color"].T
        depth[yy, xx] = r["depth"]
        alpha[yy, xx] = r["alpha"]
        sig_parts.append(r["blended"].tobytes())
        sig_parts.append(r["clamped"].tobytes())
        sig_parts.append(r["n_eval"].tobytes())
    if sh_degree > 0:
        sig_parts.append((pr["color_raw"] > 0).tobytes())
    sig_parts.append((np.abs(pr["rx"]) <= pr["limx"]).tobytes())
    sig_parts.append((np.abs(pr["ry"]) <= pr["limy"]).tobytes())
    return color, depth, alpha, hash(tuple(sig_parts))
