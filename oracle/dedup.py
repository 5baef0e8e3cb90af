"""Occupancy-aware deduplication of borrowed Gaussians (test infrastructure
only).

Sec. III-C: with voxel index kappa(x) = floor(x / v) (per axis, voxel size
v), the target map's occupied voxels are every voxel that meets the box
[mu_i - k s_i, mu_i + k s_i] of a target Gaussian, Eq. (envelope); the free
voxels are every voxel met by the segment from keyframe k's camera centre c_k
to the back-projected depth r_k(u), parameters t in [0, 1), over every pixel
u of every keyframe depth map, Eq. (free_carve); a borrowed Gaussian is kept
only if the voxel of its mean is in neither set, Eq. (dedup).  The paper
gives neither v nor k; the defaults below (0.05 m, 1) are a reading.

Readings: the scale vector is s = exp(log_scales); a pixel u is the ray
through its centre (u + 0.5, v + 0.5); r_k(u) = c_k + d(u) R_k^T K^{-1}
(u + 0.5, v + 0.5, 1)^T (world point at camera depth d); pixels with d <= 0
carve nothing.  Everything is FP64 from the FP32 inputs.

Definitions, written out: the box's voxels are the product of the per-axis
index ranges [floor(lo / v), floor(hi / v)]; the segment's voxels are the
start voxel and, walking the crossings of voxel planes in increasing t
(computed per axis as (plane - c) / (r - c)), every voxel entered at a
crossing with 0 <= t < 1 (a start on a plane, moving down, leaves its voxel
at t = 0).  Crossings of two planes closer than `tie_eps` in t
make the walk order ambiguous; such segments are reported.
"""
from __future__ import annotations

import numpy as np

VOXEL = 0.05
K_ENV = 1.0


def voxel_of(x, v=VOXEL):
    """Integer voxel indices [n,3] of points x [n,3]."""
    return np.floor(np.asarray(x, np.float64) / v).astype(np.int64)


def occupied(means, log_scales, v=VOXEL, k=K_ENV):
    """Eq. (envelope): set of voxel index triples met by the target boxes."""
    m = np.asarray(means, np.float64)
    s = np.exp(np.asarray(log_scales, np.float64))
    lo = np.floor((m - k * s) / v).astype(np.int64)
    hi = np.floor((m + k * s) / v).astype(np.int64)
    out = set()
    for a, b in zip(lo, hi):
        for x in range(a[0], b[0] + 1):
            for y in range(a[1], b[1] + 1):
                for z in range(a[2], b[2] + 1):
                    out.add((x, y, z))
    return out


def segment_voxels(c, r, v=VOXEL, tie_eps=1e-12):
    """Voxels met by the points c + t (r - c), t in [0, 1).  Returns (set,
    ambiguous)."""
    c = np.asarray(c, np.float64)
    r = np.asarray(r, np.float64)
    d = r - c
    start = np.floor(c / v).astype(np.int64)
    events = []
    for ax in range(3):
        if d[ax] == 0.0:
            continue
        i0 = int(np.floor(c[ax] / v))
        i1 = int(np.floor(r[ax] / v))
        step = 1 if d[ax] > 0 else -1
        # planes crossed between the start and end voxels along this axis
        planes = range(i0 + 1, i1 + 1) if step > 0 else range(i0, i1, -1)
        for p in planes:
            t = (p * v - c[ax]) / d[ax]
            # t = 0: the start lies on the plane and the segment leaves its
            # voxel at once (moving down); t in [0, 1) includes that crossing
            if 0.0 <= t < 1.0:
                events.append((t, ax, step))
    events.sort()
    ts = [e[0] for e in events]
    amb = any(b - a < tie_eps for a, b in zip(ts, ts[1:]))
    cur = start.copy()
    out = {tuple(cur)}
    for t, ax, step in events:
        cur[ax] += step
        out.add(tuple(cur))
    return out, amb


def ray_ends(depth_k, viewmat, intr):
    """Segments of one keyframe: camera centre c [3] and the back-projected
    end point r [H,W,3] of every pixel (pixels with depth <= 0 carve nothing:
    mask [H,W] of the others).  The R^T products are written out in a fixed
    order (left to right, no fused multiply-add), so that the camera centre
    and the end points are reproducible bit for bit."""
    dep = np.asarray(depth_k, np.float64)
    H, W = dep.shape
    vm = np.asarray(viewmat, np.float64).reshape(3, 4)
    R, tt = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = (float(x) for x in intr)
    c = np.array([-((R[0, a] * tt[0] + R[1, a] * tt[1]) + R[2, a] * tt[2]) for a in range(3)])
    ii, jj = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    rx, ry = (ii + 0.5 - cx) / fx, (jj + 0.5 - cy) / fy
    r = np.stack([c[a] + dep * ((R[0, a] * rx + R[1, a] * ry) + R[2, a] * 1.0)
                  for a in range(3)], axis=-1)
    return c, r, dep > 0.0


def free(depth, viewmats, intrinsics, v=VOXEL):
    """Eq. (free_carve) over keyframe depth maps depth [K,H,W]: (set,
    number of ambiguous segments)."""
    dep = np.asarray(depth, np.float64)
    out = set()
    n_amb = 0
    K, H, W = dep.shape
    for kf in range(K):
        c, r, ok = ray_ends(dep[kf], viewmats[kf], intrinsics[kf])
        for j in range(H):
            for i in range(W):
                if not ok[j, i]:
                    continue
                vox, amb = segment_voxels(c, r[j, i], v)
                out |= vox
                n_amb += int(amb)
    return out, n_amb


def dedup(src_means, tgt_means, tgt_log_scales, depth, viewmats, intrinsics, v=VOXEL,
          k=K_ENV):
    """Eq. (dedup): keep mask of the borrowed Gaussians, and the number of
    ambiguous carving segments."""
    occ = occupied(tgt_means, tgt_log_scales, v, k)
    fr, n_amb = free(depth, viewmats, intrinsics, v)
    keys = voxel_of(src_means, v)
    keep = np.array([tuple(q) not in occ and tuple(q) not in fr for q in keys], bool)
    return keep, n_amb
