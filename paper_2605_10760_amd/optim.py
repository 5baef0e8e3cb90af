"""The two optimisation loops that drive the rasterizer, as thin drivers
over the library's entry points (every arithmetic step, the Adam update
included, runs in its kernels; torch supplies memory and streams):

* mapping (Sec. III-A, Eq. (map_loss)):
  alpha L1(I^, I) + beta L1(D^, D) + lambda_n L_normal + lambda_s L_iso,
  alpha = 0.95, beta = 0.25, lambda_n = 1e-2, lambda_s = 10;
* joint photometric refinement of the fused map (Sec. III-C,
  Eq. (refine_loss)): alpha' L1(I~, I) + lambda (1 - SSIM(I~, I))
  + beta L1(D^, D-bar) + lambda_n' L_normal on the exposure-compensated
  render I~ = exp(a_k) I^ + b_k, with each keyframe's pose delta and
  (a_k, b_k) optimised jointly, alpha' = 1.75, lambda = 0.2,
  lambda_n' = 10; 2,000 iterations at half the mapping learning rates,
  then pruning of the Gaussians with opacity below 0.005.

The paper gives no learning rates; the defaults are the usual 3DGS ones for
the Gaussian parameters and 1e-3 for pose deltas and exposure.  The L1
terms are means over the batch (pixels, channels, views), L_normal is a
mean over interior pixels and L_iso a sum over Gaussians.

A pose delta is applied as T <- Exp(xi) T: each step renders at the current
T, takes the left-perturbation gradient at xi = 0, lets Adam produce xi
(its moments persist across steps), folds it into T and resets xi.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import astuple, dataclass

import torch

from . import _lib as L
from .rasterizer import (Adam, Rasterizer, SceneTensors, ViewTensors, apply_pose_delta,
                         iso_grad, l1_loss_grad, normal_loss_grad, prune, ssim_grad)


@dataclass(frozen=True)
class Weights:
    color: float   # alpha (mapping) or alpha' (refinement)
    depth: float   # beta
    ssim: float    # lambda (refinement only)
    normal: float  # lambda_n or lambda_n'
    iso: float     # lambda_s (mapping only)


MAP_WEIGHTS = Weights(color=0.95, depth=0.25, ssim=0.0, normal=1e-2, iso=10.0)
REFINE_WEIGHTS = Weights(color=1.75, depth=0.25, ssim=0.2, normal=10.0, iso=0.0)


@dataclass(frozen=True)
class Rates:
    means: float = 1.6e-4
    log_scales: float = 5e-3
    quats: float = 1e-3
    opacity: float = 5e-2
    colors: float = 2.5e-3
    pose: float = 1e-3
    exposure: float = 1e-3

    def scaled(self, k: float) -> "Rates":
        return Rates(*(k * x for x in astuple(self)))


class Optimizer:
    """One optimisation step per `step()`: forward of every view, the loss
    gradients on the device, backward, Adam.  The scene tensors are updated
    in place; with `pose` the view matrices of `self.views` (a copy) are,
    with `exposure` the per-view (a, b) in `self.exposure`.  Buffers are
    allocated once, so a step enqueues work only (no allocation, no host
    synchronisation) and can be captured in a graph."""

    def __init__(self, rast: Rasterizer, scene: SceneTensors, views: ViewTensors,
                 target_color: torch.Tensor, target_depth: torch.Tensor | None = None,
                 normal_prior: torch.Tensor | None = None, weights: Weights = MAP_WEIGHTS,
                 rates: Rates = Rates(), pose: bool = False, exposure: bool = False):
        self.rast, self.scene, self.w = rast, scene, weights
        self.views = ViewTensors(views.viewmats.clone(), views.intrinsics, views.view_set,
                                 views.width, views.height, views.needs_grad)
        self.tc = target_color.contiguous()
        self.td = None if target_depth is None else target_depth.contiguous()
        self.prior = None if normal_prior is None else normal_prior.contiguous()
        dev = scene.means.device
        V, H, W = views.n, views.height, views.width
        self.params = [scene.means, scene.log_scales, scene.quats, scene.opacity_logits,
                       scene.colors]
        lrs = [rates.means, rates.log_scales, rates.quats, rates.opacity, rates.colors]
        groups = list(zip(self.params, lrs))
        self.pose = torch.zeros((V, 6), device=dev) if pose else None
        self.exposure = torch.zeros((V, 2), device=dev) if exposure else None
        if pose:
            groups.append((self.pose, rates.pose))
        if exposure:
            groups.append((self.exposure, rates.exposure))
        # one gsr_adam launch updates every array (device step count, moments)
        self.adam = Adam(groups, eps=1e-15)
        self.state = rast.new_state()
        self.img = (torch.empty((V, 3, H, W), device=dev), torch.empty((V, H, W), device=dev),
                    torch.empty((V, H, W), device=dev))
        need_dd = self.td is not None or (weights.normal and self.prior is not None)
        self.lg = dict(d_color=torch.empty((V, 3, H, W), device=dev),
                       d_depth=torch.zeros((V, H, W), device=dev) if need_dd else None,
                       d_exposure=torch.empty((V, 2), device=dev) if exposure else None)
        self.g = dict(d_means=torch.empty_like(scene.means),
                      d_log_scales=torch.empty_like(scene.log_scales),
                      d_quats=torch.empty_like(scene.quats),
                      d_opacity_logits=torch.empty_like(scene.opacity_logits),
                      d_colors=torch.empty_like(scene.colors),
                      d_pose=torch.empty((V, 6), device=dev))
        self.ssim_ws = None
        if weights.ssim:
            nb = C.c_size_t()
            st = L.load().gsr_ssim_workspace_bytes(V, W, H, C.byref(nb))
            if st != L.GSR_OK:
                raise L.GsrError(st, "gsr_ssim_workspace_bytes failed")
            self.ssim_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        self.vm_next = torch.empty_like(self.views.viewmats)

    def gradients(self) -> dict:
        """Forward, loss gradients and backward at the current parameters.
        Returns the gradient buffers (parameter gradients, d_pose, and the
        exposure gradient under "d_exposure")."""
        w, sc, vw = self.w, self.scene, self.views
        c, d, _, _ = self.rast.forward(sc, vw, state=self.state, out=self.img)
        l1_out = dict(self.lg)
        if self.td is None:
            l1_out["d_depth"] = None
        l1_loss_grad(c, self.tc, d if self.td is not None else None, self.td, self.exposure,
                     w.color, w.depth, out=l1_out)
        if w.ssim:
            ssim_grad(c, self.tc, self.lg["d_color"], self.exposure, self.lg["d_exposure"],
                      w.ssim, workspace=self.ssim_ws)
        gd = self.lg["d_depth"]
        if w.normal and self.prior is not None:
            if self.td is None:
                gd.zero_()  # no depth L1 term wrote it
            normal_loss_grad(d, self.prior, vw.intrinsics, gd, w.normal)
        g = self.rast.backward(sc, vw, self.state, self.lg["d_color"], gd, None, out=self.g)
        if w.iso:
            iso_grad(sc.log_scales, g["d_log_scales"], w.iso)
        out = dict(g)
        out["d_exposure"] = self.lg["d_exposure"]
        return out

    def step(self) -> None:
        g = self.gradients()
        names = ["d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors"]
        for p, k in zip(self.params, names):
            p.grad = g[k]
        if self.pose is not None:
            self.pose.grad = g["d_pose"]
        if self.exposure is not None:
            self.exposure.grad = g["d_exposure"]
        with torch.no_grad():
            self.adam.step()
            if self.pose is not None:
                apply_pose_delta(self.views.viewmats, self.pose, out=self.vm_next)
                self.views.viewmats.copy_(self.vm_next)
                self.pose.zero_()


def refine(rast: Rasterizer, scene: SceneTensors, views: ViewTensors,
           target_color: torch.Tensor, target_depth: torch.Tensor | None = None,
           normal_prior: torch.Tensor | None = None, iters: int = 2000,
           rates: Rates = Rates(), min_opacity: float = 0.005):
    """Joint photometric refinement of a fused map (Sec. III-C): `iters`
    steps of Eq. (refine_loss) at half the mapping rates over the Gaussians,
    the pose deltas and the exposure, then opacity pruning.  Returns (pruned
    scene, refined view matrices, exposure [V,2])."""
    opt = Optimizer(rast, scene, views, target_color, target_depth, normal_prior,
                    REFINE_WEIGHTS, rates.scaled(0.5), pose=True, exposure=True)
    for _ in range(iters):
        opt.step()
    with torch.no_grad():
        pruned = prune(scene, min_opacity)
    return pruned, opt.views.viewmats, opt.exposure
