"""Sim(3) correction of a Gaussian submap and the lift of its keyframe poses
into the global frame (test infrastructure only).

Once the pose graph has converged, every submap has a similarity correction
C = (s, R, t) (Sec. III-C).  Eq. (gauss_update) gives its action on a Gaussian: the mean
maps to s R mu + t, the covariance to s^2 R Sigma R^T and the scale vector to
s times itself, with opacity and colour unchanged.  With the factorisation
Sigma = Rg diag(sg)^2 Rg^T this is: log-scales + ln s, and the Gaussian's
rotation composed on the left with R (quaternion q_R * q).  Colour is left
as it is for every SH degree (the paper states colour is unchanged; for
degree >= 1 this keeps the coefficients in the submap's frame, a reading).

Eq. (mapgba_lift) carries a keyframe's world-to-camera pose T_k into the
global frame as T_k o C^{-1}.  That map is a similarity with scale 1/s; the
rasterizer takes rigid world-to-camera matrices, so the lifted camera is
written as s (T_k o C^{-1}) = [R_k R^T | s t_k - R_k R^T t]: the same camera
with its length unit multiplied by s.  Pixels are unchanged and camera
depths scale by s (the near plane must scale with them).

Everything is FP64.
"""
from __future__ import annotations

import numpy as np

from .project64 import quat_to_rot


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a * b of quaternions (w, x, y, z); a is [4] or [n,4],
    b is [n,4]."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    a = np.broadcast_to(a, b.shape)
    w1, x1, y1, z1 = a[:, 0], a[:, 1], a[:, 2], a[:, 3]
    w2, x2, y2, z2 = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def _unpack(sim):
    """(s, unit q_R, R, t) of a similarity stored as (s, qw, qx, qy, qz, tx, ty, tz)."""
    sim = np.asarray(sim, np.float64)
    s = sim[0]
    q = sim[1:5] / np.linalg.norm(sim[1:5])
    R = quat_to_rot(q[None])[0]
    return s, q, R, sim[5:8]


def apply_gaussians(means, log_scales, quats, sim):
    """Eq. (gauss_update) on a set of Gaussians: returns (means', log_scales',
    quats') in FP64; opacity and colour are unchanged."""
    s, q, R, t = _unpack(sim)
    m = np.asarray(means, np.float64)
    return (s * m @ R.T + t,
            np.asarray(log_scales, np.float64) + np.log(s),
            quat_mul(q, np.asarray(quats, np.float64)))


def lift_viewmat(viewmat, sim):
    """Eq. (mapgba_lift) for one world-to-camera pose [3,4], in the rigid form
    s (T o C^{-1}) = [Rk R^T | s tk - Rk R^T t]."""
    s, _, R, t = _unpack(sim)
    vm = np.asarray(viewmat, np.float64).reshape(3, 4)
    Rk, tk = vm[:, :3], vm[:, 3]
    RkRt = Rk @ R.T
    return np.concatenate([RkRt, (s * tk - RkRt @ t)[:, None]], 1)


def apply_sets(means, log_scales, quats, set_offsets, sims):
    """apply_gaussians on every set of a concatenated scene, set k with sims[k]."""
    out = [np.empty((np.asarray(means).shape[0], 3)), np.empty((np.asarray(means).shape[0], 3)),
           np.empty((np.asarray(means).shape[0], 4))]
    for k in range(len(set_offsets) - 1):
        a, b = int(set_offsets[k]), int(set_offsets[k + 1])
        r = apply_gaussians(means[a:b], log_scales[a:b], quats[a:b], sims[k])
        for o, x in zip(out, r):
            o[a:b] = x
    return tuple(out)
