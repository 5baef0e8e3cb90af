"""Seeded synthetic inputs for the Gaussian-splatting rasterizer.

This module only draws random numbers and builds camera matrices; it holds
none of the rasterizer's arithmetic.  Both the CPU oracle and the HIP path
read the FP32 arrays it returns, so the two sides always see identical inputs.

Shapes follow the paper's setting: indoor Replica-style rooms rendered by
pinhole cameras whose intrinsics come from a 90 degree horizontal field of
view (Appendix A, "Rendered modalities": 1200x680 frames, so f = 600), agents'
submaps of uneven sizes (Sec. III-A, submaps P^a_l) and a fused global map
(Sec. III-C).  The datasets themselves are not available, so these draws stand
in for them.

Conventions
-----------
* Camera space is x right, y down, z forward; a view matrix is the 3x4
  world-to-camera transform [R | t] (Sec. III-B: poses T_k map world to
  camera).  World space uses the same y-down axis so an upright camera has
  camera-y equal to world-y.
* Quaternions are (w, x, y, z), not normalised.
* "N(m, s)" draws use numpy ``normal(m, s)``, i.e. s is the standard
  deviation.  Draw order per scene: means, log-scales, quaternions, opacity
  normals, colours, then targets.  Draws are FP64 and cast to FP32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32

# Room used by the Replica-scale configurations: 6 m wide (x), 3 m tall
# (y, pointing down), 4 m deep (z), centred on the origin.
ROOM_LO = np.array([-3.0, -1.5, -2.0])
ROOM_HI = np.array([3.0, 1.5, 2.0])

# Real spherical harmonic Y_00 (constant band), used only to express a DC
# colour draw as an SH coefficient: c = 0.5 + Y00 * k00.
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclass
class Scene:
    """Gaussians of one or more sets (submaps), FP32 SoA, concatenated."""

    means: np.ndarray          # [N,3]
    log_scales: np.ndarray     # [N,3]
    quats: np.ndarray          # [N,4] (w,x,y,z), unnormalised
    opacity_logits: np.ndarray # [N]
    colors: np.ndarray         # [N,3] (sh_degree 0) or [N,16,3] (sh_degree 3)
    set_offsets: np.ndarray    # int64 [S+1]
    sh_degree: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_sets(self) -> int:
        return int(self.set_offsets.shape[0] - 1)

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx], self.log_scales[idx], self.quats[idx],
                     self.opacity_logits[idx], self.colors[idx],
                     np.array([0, idx.shape[0]], np.int64), self.sh_degree)


@dataclass
class Views:
    """Pinhole views; each view renders exactly one Gaussian set."""

    viewmats: np.ndarray       # [V,3,4] world->camera
    intrinsics: np.ndarray     # [V,4] fx, fy, cx, cy
    view_set: np.ndarray       # int32 [V]
    width: int
    height: int
    needs_grad: np.ndarray = field(default=None)  # bool [V]

    def __post_init__(self):
        if self.needs_grad is None:
            self.needs_grad = np.ones(self.viewmats.shape[0], bool)

    @property
    def n(self) -> int:
        return int(self.viewmats.shape[0])

    def select(self, idx) -> "Views":
        idx = np.asarray(idx)
        return Views(self.viewmats[idx], self.intrinsics[idx], self.view_set[idx],
                     self.width, self.height, self.needs_grad[idx])


@dataclass
class Workload:
    name: str
    scene: Scene
    views: Views
    target_color: np.ndarray   # [V,3,H,W]
    target_depth: np.ndarray   # [V,H,W] (or None)
    description: str = ""


# --------------------------------------------------------------------------
# primitive draws
# --------------------------------------------------------------------------

def random_unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations: normalised 4-D standard normal draws."""
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def draw_gaussians(rng, n, lo, hi, sh_degree=0, sh_rest_std=0.1):
    """Gaussians drawn as the small configuration prescribes.

    means U[lo,hi]^3, log-scales N(-3,0.5), random unit quaternions,
    opacity logits N(0,1) (so opacity = sigmoid(N(0,1))), RGB U[0,1].
    With sh_degree 3 the RGB draw becomes the DC coefficient
    (c - 0.5)/Y00 and the 45 higher coefficients are N(0, sh_rest_std).
    """
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    means = lo + (hi - lo) * rng.random((n, 3))
    log_scales = rng.normal(-3.0, 0.5, size=(n, 3))
    quats = random_unit_quats(rng, n)
    opac = rng.normal(0.0, 1.0, size=n)
    rgb = rng.random((n, 3))
    if sh_degree == 0:
        colors = rgb
    else:
        k = (sh_degree + 1) ** 2
        colors = np.empty((n, k, 3))
        colors[:, 0, :] = (rgb - 0.5) / _Y00
        colors[:, 1:, :] = rng.normal(0.0, sh_rest_std, size=(n, k - 1, 3))
    return (means.astype(F32), log_scales.astype(F32), quats.astype(F32),
            opac.astype(F32), colors.astype(F32))


def look_at(center, target, yaw_jitter=0.0, pitch=0.0) -> np.ndarray:
    """World->camera [R|t] for a camera at `center` looking at `target`.

    The forward direction is flattened to the horizontal (x,z) plane, turned
    by `yaw_jitter` radians about the (down) y axis and tilted by `pitch`.
    Rows of R are the camera's right, down and forward axes in world space.
    """
    center = np.asarray(center, np.float64)
    d = np.asarray(target, np.float64) - center
    yaw = math.atan2(d[0], d[2]) + yaw_jitter
    fwd = np.array([math.sin(yaw) * math.cos(pitch), -math.sin(pitch),
                    math.cos(yaw) * math.cos(pitch)])
    down0 = np.array([0.0, 1.0, 0.0])
    right = np.cross(down0, fwd)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ center
    return np.concatenate([R, t[:, None]], axis=1)


def identity_view() -> np.ndarray:
    return np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)


def pinhole(width, height, f):
    return np.array([f, f, width / 2.0, height / 2.0])


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def small_plain(seed: int = 0, n: int = 2000) -> Workload:
    """2,000 Gaussians in front of one 128x96 camera (fx=fy=100, c=(64,48)),
    identity pose; means U[-1,1]^2 x U[2,4]; L1 colour target U[0,1]."""
    rng = np.random.default_rng(seed)
    g = draw_gaussians(rng, n, (-1, -1, 2), (1, 1, 4))
    scene = Scene(*g, set_offsets=np.array([0, n], np.int64))
    W, H = 128, 96
    views = Views(identity_view()[None].astype(F32),
                  np.array([[100.0, 100.0, 64.0, 48.0]], F32),
                  np.zeros(1, np.int32), W, H)
    trng = np.random.default_rng(1000 + seed)
    tc = trng.random((1, 3, H, W)).astype(F32)
    return Workload("small-plain-2k-128x96", scene, views, tc, None,
                    "plain fwd+bwd, 2k Gaussians, one 128x96 view")


def room_plain(seed: int = 10, n: int = 300_000, width=1200, height=680,
               f=600.0) -> Workload:
    """Gaussians uniform in the 6x3x4 m room, one 1200x680 (f=600) camera at
    the origin with identity pose; colour U[0,1] and depth U[0.2,4] targets."""
    rng = np.random.default_rng(seed)
    g = draw_gaussians(rng, n, ROOM_LO, ROOM_HI)
    scene = Scene(*g, set_offsets=np.array([0, n], np.int64))
    views = Views(identity_view()[None].astype(F32),
                  pinhole(width, height, f)[None].astype(F32),
                  np.zeros(1, np.int32), width, height)
    tc = rng.random((1, 3, height, width)).astype(F32)
    td = (0.2 + 3.8 * rng.random((1, height, width))).astype(F32)
    return Workload(f"room-plain-{n // 1000}k-{width}x{height}", scene, views,
                    tc, td, "plain fwd+bwd, one view inside the room")


def fd_subcase(seed: int = 21, n: int = 500) -> Workload:
    """Finite-difference sub-case: 500 Gaussians, 64x48 view, f=50, c=(32,24),
    Gaussians drawn as in the small configuration."""
    rng = np.random.default_rng(seed)
    g = draw_gaussians(rng, n, (-1, -1, 2), (1, 1, 4))
    scene = Scene(*g, set_offsets=np.array([0, n], np.int64))
    views = Views(identity_view()[None].astype(F32),
                  np.array([[50.0, 50.0, 32.0, 24.0]], F32),
                  np.zeros(1, np.int32), 64, 48)
    tc = rng.random((1, 3, 48, 64)).astype(F32)
    td = (0.2 + 3.8 * rng.random((1, 48, 64))).astype(F32)
    return Workload("fd-500-64x48", scene, views, tc, td, "FD sub-case")


MULTI_AGENT_SIZES = (50_000, 120_000, 200_000, 300_000, 400_000, 600_000)


def multi_agent(seed: int = 300, sizes=MULTI_AGENT_SIZES, keyframes: int = 8,
                width=640, height=480, scale: float = 1.0) -> Workload:
    """Agents' submaps of uneven sizes, each rendered from its own keyframes.

    Each set is uniform in the room.  Its keyframes sit on a horizontal circle
    of radius 1.5 m around the room centre at angle U[0,2pi), looking at the
    centre with yaw jitter U[-15,15] degrees; 640x480 at f=320 (HFOV 90).
    `scale` shrinks every set size (for tests), keeping the unevenness.
    """
    sizes = [max(1, int(round(s * scale))) for s in sizes]
    parts = []
    for a, n in enumerate(sizes):
        rng = np.random.default_rng(seed + a)
        parts.append(draw_gaussians(rng, n, ROOM_LO, ROOM_HI))
    arrays = [np.concatenate([p[i] for p in parts]) for i in range(5)]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    scene = Scene(*arrays, set_offsets=offs)
    vm, intr, vs = [], [], []
    f = width / 2.0
    for a in range(len(sizes)):
        crng = np.random.default_rng(seed + 100 + a)
        for _ in range(keyframes):
            th = crng.uniform(0.0, 2 * math.pi)
            jit = math.radians(crng.uniform(-15.0, 15.0))
            c = np.array([1.5 * math.cos(th), 0.0, 1.5 * math.sin(th)])
            vm.append(look_at(c, (0.0, 0.0, 0.0), jit))
            intr.append(pinhole(width, height, f))
            vs.append(a)
    views = Views(np.array(vm, F32), np.array(intr, F32), np.array(vs, np.int32),
                  width, height)
    trng = np.random.default_rng(seed + 1000)
    V = views.n
    tc = trng.random((V, 3, height, width)).astype(F32)
    td = (0.2 + 3.8 * trng.random((V, height, width))).astype(F32)
    return Workload(f"multi-agent-{len(sizes)}x{keyframes}-{width}x{height}",
                    scene, views, tc, td,
                    "agents' submaps x keyframes in one batch")


def fused_map(seed: int = 500, n: int = 3_000_000, n_novel: int = 16,
              n_keyframes: int = 32, width=1200, height=680,
              sh_degree: int = 3) -> Workload:
    """Fused global map: Gaussians uniform in the room with SH degree 3;
    n_novel forward-only views then n_keyframes fwd+bwd views at 1200x680.
    Camera centres U over x in [-2,2], y in [-0.5,0.5], z in [-1.5,1.5]; yaw
    U[0,2pi); pitch U[-15,15] degrees."""
    rng = np.random.default_rng(seed)
    g = draw_gaussians(rng, n, ROOM_LO, ROOM_HI, sh_degree=sh_degree)
    scene = Scene(*g, set_offsets=np.array([0, n], np.int64), sh_degree=sh_degree)
    crng = np.random.default_rng(seed + 1)
    vm, intr = [], []
    for _ in range(n_novel + n_keyframes):
        c = np.array([crng.uniform(-2, 2), crng.uniform(-0.5, 0.5),
                      crng.uniform(-1.5, 1.5)])
        yaw = crng.uniform(0.0, 2 * math.pi)
        pitch = math.radians(crng.uniform(-15.0, 15.0))
        tgt = c + np.array([math.sin(yaw), 0.0, math.cos(yaw)])
        vm.append(look_at(c, tgt, 0.0, pitch))
        intr.append(pinhole(width, height, width / 2.0))
    V = n_novel + n_keyframes
    ng = np.zeros(V, bool)
    ng[n_novel:] = True
    views = Views(np.array(vm, F32), np.array(intr, F32), np.zeros(V, np.int32),
                  width, height, ng)
    trng = np.random.default_rng(seed + 1000)
    tc = trng.random((V, 3, height, width)).astype(F32)
    td = (0.2 + 3.8 * trng.random((V, height, width))).astype(F32)
    return Workload(f"fused-map-{n // 1000}k-sh{sh_degree}-{V}x{width}x{height}",
                    scene, views, tc, td, "fused map, novel + keyframe views")


def tiny_scene(seed: int, n: int = 24, width: int = 32, height: int = 24,
               f: float = 30.0, sh_degree: int = 0, pose_noise: float = 0.0):
    """Small random scene for property tests: Gaussians in front of one view."""
    rng = np.random.default_rng(seed)
    g = draw_gaussians(rng, n, (-1, -1, 1.5), (1, 1, 3.5), sh_degree=sh_degree,
                       sh_rest_std=0.3)
    means, ls, q, o, c = g
    ls = (ls + 1.2).astype(F32)   # larger footprints on the small image
    scene = Scene(means, ls, q, o, c, np.array([0, n], np.int64), sh_degree)
    vm = identity_view()
    if pose_noise:
        ang = rng.normal(0.0, pose_noise, 3)
        vm = look_at(rng.normal(0.0, pose_noise, 3), (ang[0], ang[1], 3.0))
    views = Views(vm[None].astype(F32),
                  np.array([[f, f, width / 2.0, height / 2.0]], F32),
                  np.zeros(1, np.int32), width, height)
    return scene, views


WORKLOADS = {
    0: small_plain,
    1: room_plain,
    2: lambda seed=20: room_plain(seed=seed, n=1_000_000),
    3: multi_agent,
    4: fused_map,
}


# --------------------------------------------------------------------------
# depth maps for the mapping-loss extras and seeding
# --------------------------------------------------------------------------

def slanted_depth(rng: np.random.Generator, n_views: int, width: int, height: int,
                  f: float = 600.0, hole_frac: float = 0.01, noise: float = 2e-3):
    """Piecewise-planar camera depth maps [V,H,W] standing in for rendered
    room depth: per view, the nearest of three random planes
    z = z0 / (1 - gx x - gy y) in normalised image coordinates, z0 in
    U[1.5, 4], gradients N(0, 0.3), plus N(0, noise) jitter and a fraction
    of zero-depth holes; and unit normal priors [V,3,H,W] that face the
    camera, (N(0, 0.3), N(0, 0.3), -1) normalised.  Intrinsics [V,4] use
    focal f and the image centre."""
    intr = np.array([pinhole(width, height, f)] * n_views)
    x = (np.arange(width) + 0.5 - width / 2.0) / f
    y = (np.arange(height) + 0.5 - height / 2.0) / f
    depth = np.empty((n_views, height, width))
    for v in range(n_views):
        best = np.full((height, width), np.inf)
        for _ in range(3):
            z0 = rng.uniform(1.5, 4.0)
            gx, gy = rng.normal(0, 0.3, 2)
            den = 1.0 - gx * x[None, :] - gy * y[:, None]
            z = np.where(den > 0.2, z0 / np.maximum(den, 0.2), np.inf)
            best = np.minimum(best, z)
        best = np.where(np.isfinite(best), best, 5.0)
        depth[v] = best + rng.normal(0, noise, best.shape)
    depth[rng.random(depth.shape) < hole_frac] = 0.0
    pr = np.stack([rng.normal(0, 0.3, depth.shape), rng.normal(0, 0.3, depth.shape),
                   -np.ones(depth.shape)], axis=1)
    pr /= np.linalg.norm(pr, axis=1, keepdims=True)
    return depth.astype(F32), pr.astype(F32), intr.astype(F32)
