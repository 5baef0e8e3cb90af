"""Pins of the oracle's Sim(3) correction and pose lift (Eq. (gauss_update),
Eq. (mapgba_lift)) against matrix algebra, the group law and the render
invariance of the smooth FP64 renderer."""
import math

import numpy as np

from oracle.project64 import quat_to_rot
from oracle.sim3 import apply_gaussians, apply_sets, lift_viewmat, quat_mul
from oracle.smooth import render_smooth
from synth.scenes import tiny_scene


def _rand_sim(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return np.concatenate([[math.exp(rng.normal(0, 0.4))], q, rng.normal(0, 1.0, 3)])


def test_quat_mul_is_rotation_product():
    """R(a * b) = R(a) R(b): the Hamilton product composes rotations."""
    rng = np.random.default_rng(0)
    a = rng.normal(size=(50, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.normal(size=(50, 4))
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    ab = np.concatenate([quat_mul(a[i], b[i:i + 1]) for i in range(50)])
    np.testing.assert_allclose(quat_to_rot(ab), quat_to_rot(a) @ quat_to_rot(b), atol=1e-13)


def test_covariance_maps_as_s2_R_Sigma_Rt():
    """Sigma' from the transformed log-scales and rotation equals
    s^2 R Sigma R^T (Eq. (gauss_update))."""
    rng = np.random.default_rng(1)
    n = 40
    m = rng.normal(size=(n, 3))
    ls = rng.normal(-2, 0.5, (n, 3))
    q = rng.normal(size=(n, 4))
    sim = _rand_sim(rng)
    m2, ls2, q2 = apply_gaussians(m, ls, q, sim)

    def cov(ls_, q_):
        R = quat_to_rot(q_ / np.linalg.norm(q_, axis=1, keepdims=True))
        S = np.exp(ls_)
        return R @ (S[:, :, None] ** 2 * np.transpose(R, (0, 2, 1)))

    s = sim[0]
    R = quat_to_rot(sim[None, 1:5])[0]
    np.testing.assert_allclose(cov(ls2, q2), s * s * R @ cov(ls, q) @ R.T, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(m2, s * m @ R.T + sim[5:], atol=1e-13)
    # |q'| = |q|: the rotation part is unchanged up to composition
    np.testing.assert_allclose(np.linalg.norm(q2, axis=1), np.linalg.norm(q, axis=1), rtol=1e-13)


def test_group_law():
    """Applying C1 then C2 equals applying C2 o C1 = (s2 s1, R2 R1, s2 R2 t1 + t2)."""
    rng = np.random.default_rng(2)
    m = rng.normal(size=(30, 3))
    ls = rng.normal(-2, 0.5, (30, 3))
    q = rng.normal(size=(30, 4))
    c1, c2 = _rand_sim(rng), _rand_sim(rng)
    r1 = apply_gaussians(*apply_gaussians(m, ls, q, c1), c2)
    R2 = quat_to_rot(c2[None, 1:5])[0]
    c21 = np.concatenate([[c2[0] * c1[0]], quat_mul(c2[1:5], c1[None, 1:5])[0],
                          c2[0] * R2 @ c1[5:] + c2[5:]])
    r2 = apply_gaussians(m, ls, q, c21)
    for x, y in zip(r1, r2):
        np.testing.assert_allclose(x, y, atol=1e-12)


def test_lift_keeps_pixels_and_scales_depth():
    """Camera coordinates of C(mu) under the lifted pose are s times those of
    mu under the original pose (Eq. (mapgba_lift) in rigid form)."""
    rng = np.random.default_rng(3)
    m = rng.normal(size=(25, 3))
    sim = _rand_sim(rng)
    Rk = quat_to_rot(rng.normal(size=(1, 4)) / 2.0)[0]
    Rk, _ = np.linalg.qr(Rk)
    vm = np.concatenate([Rk, rng.normal(size=(3, 1))], 1)
    vm2 = lift_viewmat(vm, sim)
    m2, _, _ = apply_gaussians(m, np.zeros((25, 3)), np.tile([1.0, 0, 0, 0], (25, 1)), sim)
    p1 = m @ vm[:, :3].T + vm[:, 3]
    p2 = m2 @ vm2[:, :3].T + vm2[:, 3]
    np.testing.assert_allclose(p2, sim[0] * p1, atol=1e-12)
    np.testing.assert_allclose(vm2[:, :3] @ vm2[:, :3].T, np.eye(3), atol=1e-13)


def test_render_invariance_through_oracle_sim3():
    """P11 with the oracle's own functions: the corrected Gaussians seen from
    the lifted keyframe render the same colour and alpha, and s times the
    depth (SH degree 0, near plane scaled by s)."""
    sc, vw = tiny_scene(9, n=40, width=32, height=24, pose_noise=0.2)
    p = {k: np.asarray(getattr(sc, k), np.float64).copy()
         for k in ("means", "log_scales", "quats", "opacity_logits", "colors")}
    sim = np.array([1.7, 0.8, 0.3, -0.4, 0.2, 0.3, -0.2, 0.5])
    p2 = dict(p)
    p2["means"], p2["log_scales"], p2["quats"] = apply_gaussians(p["means"], p["log_scales"],
                                                                 p["quats"], sim)
    vm2 = lift_viewmat(vw.viewmats[0], sim)
    c1, d1, a1, _ = render_smooth(p, 0, vw.viewmats[0], vw.intrinsics[0], vw.width, vw.height,
                                  z_near=0.2)
    c2, d2, a2, _ = render_smooth(p2, 0, vm2, vw.intrinsics[0], vw.width, vw.height,
                                  z_near=0.2 * sim[0])
    np.testing.assert_allclose(c2, c1, atol=1e-10)
    np.testing.assert_allclose(a2, a1, atol=1e-10)
    np.testing.assert_allclose(d2, sim[0] * d1, atol=1e-9)
    assert a1.max() > 0.5


def test_apply_sets_uses_each_sets_similarity():
    rng = np.random.default_rng(4)
    m = rng.normal(size=(30, 3))
    ls = rng.normal(size=(30, 3))
    q = rng.normal(size=(30, 4))
    offs = np.array([0, 7, 7, 30])
    sims = [_rand_sim(rng) for _ in range(3)]
    out = apply_sets(m, ls, q, offs, sims)
    for k in (0, 2):
        a, b = offs[k], offs[k + 1]
        ref = apply_gaussians(m[a:b], ls[a:b], q[a:b], sims[k])
        for x, y in zip(out, ref):
            np.testing.assert_allclose(x[a:b], y, atol=1e-14)
