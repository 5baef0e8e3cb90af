"""Mapping-loss extras and Gaussian seeding (test infrastructure only).

Sec. III-A, Eq. (map_loss): besides the L1 terms, the mapping loss has
lambda_s L_iso, L_iso = sum_i |s_i - s_bar_i| (each Gaussian's scale
components pulled toward their mean; lambda_s = 10), and
lambda_n L_normal, L_normal = sum_k |1 - N^_k . N-bar_k| (a cosine loss
between the depth-induced normal of the rendered depth and a normal prior;
lambda_n = 1e-2).  New keyframes seed Gaussians at mu = T_k^{-1}
pi^{-1}(u, d_k) with the pixel's colour and a scale from the local
neighbourhood.

Readings (the paper gives no more):
  * L_iso: |s_i - s_bar_i| is the L1 norm over the three components, with
    s = exp(log_scales) and s_bar the mean of the three; summed over the
    Gaussians.
  * Normals: camera-space points P(u) = D(u) K^{-1} (u + 0.5, v + 0.5, 1);
    at an interior pixel N^ = normalize((P(u, v+1) - P(u, v-1)) x
    (P(u+1, v) - P(u-1, v))) (central differences; a surface facing the
    camera gets a normal toward it, -z).  Pixels on the image border, with
    a non-positive depth among the four neighbours, or with a zero cross
    product contribute nothing.  |1 - N^.N-bar| = 1 - N^.N-bar for unit
    vectors; L_normal is its mean over the interior pixels (V (H-2) (W-2))
    of the batch.
  * Seeding: one Gaussian per pixel with d > 0 on a grid of stride `stride`
    (pixels (stride j, stride i)), in row-major order; colour = the pixel's
    RGB; isotropic scale = the mean distance from the pixel's point to the
    points of its (up to four) grid neighbours with d > 0, or, without
    such a neighbour, the pixel footprint d stride / fx; identity rotation;
    the opacity logit is the caller's.

Everything is FP64 from the FP32 inputs.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ L_iso
def iso_loss(log_scales):
    s = np.exp(np.asarray(log_scales, np.float64))
    return float(np.sum(np.abs(s - s.mean(axis=1, keepdims=True))))


def iso_loss_grad(log_scales):
    """d L_iso / d log_scales [N,3]; the subgradient of |.| at 0 is 0."""
    s = np.exp(np.asarray(log_scales, np.float64))
    g = np.sign(s - s.mean(axis=1, keepdims=True))
    return s * (g - g.mean(axis=1, keepdims=True))


# --------------------------------------------------------------- normals
def _points(depth, intr):
    """Camera-space points [V,H,W,3] of depth maps [V,H,W]."""
    d = np.asarray(depth, np.float64)
    V, H, W = d.shape
    out = np.empty((V, H, W, 3))
    for k in range(V):
        fx, fy, cx, cy = (float(x) for x in intr[k])
        u = (np.arange(W) + 0.5 - cx) / fx
        v = (np.arange(H) + 0.5 - cy) / fy
        out[k, :, :, 0] = d[k] * u[None, :]
        out[k, :, :, 1] = d[k] * v[:, None]
        out[k, :, :, 2] = d[k]
    return out


def depth_normals(depth, intr):
    """(normals [V,H,W,3], valid [V,H,W]) of the depth-induced normal."""
    d = np.asarray(depth, np.float64)
    P = _points(d, intr)
    V, H, W = d.shape
    n = np.zeros((V, H, W, 3))
    valid = np.zeros((V, H, W), bool)
    a = P[:, 2:, 1:-1] - P[:, :-2, 1:-1]      # P(u, v+1) - P(u, v-1)
    b = P[:, 1:-1, 2:] - P[:, 1:-1, :-2]      # P(u+1, v) - P(u-1, v)
    c = np.cross(a, b)
    nrm = np.linalg.norm(c, axis=-1)
    pos = ((d[:, 2:, 1:-1] > 0) & (d[:, :-2, 1:-1] > 0) & (d[:, 1:-1, 2:] > 0)
           & (d[:, 1:-1, :-2] > 0) & (nrm > 0))
    n[:, 1:-1, 1:-1] = np.where(pos[..., None], c / np.where(nrm > 0, nrm, 1.0)[..., None], 0.0)
    valid[:, 1:-1, 1:-1] = pos
    return n, valid


def normal_loss(depth, prior, intr):
    """Mean over the interior pixels of 1 - N^ . N-bar (prior [V,H,W,3])."""
    n, valid = depth_normals(depth, intr)
    V, H, W = np.asarray(depth).shape
    cos = np.sum(n * np.asarray(prior, np.float64), axis=-1)
    return float(np.sum(np.where(valid, 1.0 - cos, 0.0)) / (V * (H - 2) * (W - 2)))


def normal_loss_grad(depth, prior, intr):
    """d normal_loss / d depth [V,H,W], by the chain rule: with c = a x b,
    a = P(u, v+1) - P(u, v-1), b = P(u+1, v) - P(u-1, v) and n = c / |c|,
    dl/dc = (-N-bar + (n . N-bar) n) / |c|, dl/da = b x dl/dc,
    dl/db = dl/dc x a, and dl/dD(q) = ray(q) . dl/dP(q)."""
    d = np.asarray(depth, np.float64)
    V, H, W = d.shape
    P = _points(d, intr)
    n, valid = depth_normals(d, intr)
    pr = np.asarray(prior, np.float64)
    a = P[:, 2:, 1:-1] - P[:, :-2, 1:-1]
    b = P[:, 1:-1, 2:] - P[:, 1:-1, :-2]
    c = np.cross(a, b)
    nrm = np.linalg.norm(c, axis=-1)
    ni = n[:, 1:-1, 1:-1]
    pi = pr[:, 1:-1, 1:-1]
    w = valid[:, 1:-1, 1:-1] / (V * (H - 2) * (W - 2))
    gc = (-pi + np.sum(ni * pi, axis=-1, keepdims=True) * ni) / np.where(nrm > 0, nrm, 1.0)[..., None]
    gc = gc * w[..., None]
    ga = np.cross(b, gc)
    gb = np.cross(gc, a)
    gP = np.zeros((V, H, W, 3))
    gP[:, 2:, 1:-1] += ga
    gP[:, :-2, 1:-1] -= ga
    gP[:, 1:-1, 2:] += gb
    gP[:, 1:-1, :-2] -= gb
    ray = _points(np.ones_like(d), intr)
    return np.sum(gP * ray, axis=-1)


# ---------------------------------------------------------------- seeding
def seed(depth, color, viewmat, intr, stride=1, opacity_logit=0.0):
    """Gaussians seeded from one keyframe: dict of means [M,3], log_scales
    [M,3], quats [M,4], opacity_logits [M], colors [M,3]."""
    d = np.asarray(depth, np.float64)
    H, W = d.shape
    vm = np.asarray(viewmat, np.float64).reshape(3, 4)
    R, t = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = (float(x) for x in intr)
    js, is_ = np.arange(0, H, stride), np.arange(0, W, stride)
    means, scales, cols = [], [], []

    def cam_point(j, i):
        z = d[j, i]
        return np.array([z * (i + 0.5 - cx) / fx, z * (j + 0.5 - cy) / fy, z])

    for j in js:
        for i in is_:
            if not d[j, i] > 0:
                continue
            p = cam_point(j, i)
            dists = []
            for dj, di in ((0, -stride), (0, stride), (-stride, 0), (stride, 0)):
                jj, ii = j + dj, i + di
                if 0 <= jj < H and 0 <= ii < W and d[jj, ii] > 0:
                    dists.append(np.linalg.norm(cam_point(jj, ii) - p))
            sc = np.mean(dists) if dists else d[j, i] * stride / fx
            means.append(R.T @ (p - t))
            scales.append(sc)
            cols.append(np.asarray(color, np.float64)[:, j, i])
    M = len(means)
    return dict(means=np.array(means).reshape(M, 3),
                log_scales=np.repeat(np.log(np.array(scales)).reshape(M, 1), 3, axis=1),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (M, 1)),
                opacity_logits=np.full(M, float(opacity_logit)),
                colors=np.array(cols).reshape(M, 3))
