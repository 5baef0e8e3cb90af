"""Pins of the oracle's analytic backward: FP64 central finite differences
(P9), the translation-pose identity (P10), Sim(3) invariance of the render
(P11), and the SH / SE(3) building blocks against scipy."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.special

from oracle.render import render_backward, render_view
from oracle.se3 import apply_left, exp_se3
from oracle.sh import sh_basis, sh_basis_grad
from oracle.smooth import render_smooth
from synth.scenes import Scene, fd_subcase, tiny_scene

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "colors")
GRAD_OF = dict(means="d_means", log_scales="d_log_scales", quats="d_quats",
               opacity_logits="d_opacity", colors="d_colors")


def params64(sc):
    return {k: np.asarray(getattr(sc, k), np.float64).copy() for k in PARAMS}


def smooth_loss(sc, vw, p, w, pose=None):
    c, d, a, sig = render_smooth(p, sc.sh_degree, vw.viewmats[0], vw.intrinsics[0],
                                 vw.width, vw.height, pose_delta=pose)
    return float(np.sum(w[0] * c) + np.sum(w[1] * d) + np.sum(w[2] * a)), sig


def weights(rng, H, W):
    return (rng.normal(size=(3, H, W)), rng.normal(size=(H, W)) * 0.3,
            rng.normal(size=(H, W)))


def fd_check(sc, vw, n_per_param=6, seed=0, rtol=1e-6):
    rng = np.random.default_rng(seed)
    H, W = vw.height, vw.width
    w = weights(rng, H, W)
    g = render_backward(sc, vw, w[0][None], w[1][None], w[2][None])
    p0 = params64(sc)
    L0, sig0 = smooth_loss(sc, vw, p0, w)
    # the FP64-decided render equals the oracle's render at the base point
    rv = render_view(sc, vw, 0)
    Lt = float(np.sum(w[0] * rv["color"]) + np.sum(w[1] * rv["depth"]) + np.sum(w[2] * rv["alpha"]))
    assert Lt == pytest.approx(L0, rel=1e-12, abs=1e-12)
    checked, skipped = 0, 0
    worst = 0.0
    for name in PARAMS:
        G = g[GRAD_OF[name]]
        flat = np.abs(G).reshape(G.shape[0], -1).max(1)
        cand = np.argsort(-flat)[: 4 * n_per_param]
        picks = rng.choice(cand, size=min(n_per_param, cand.size), replace=False)
        scale = float(np.abs(G).max())
        for i in picks:
            comp = tuple(rng.integers(0, s) for s in G.shape[1:])
            theta = p0[name][(i,) + comp]
            h = 1e-6 * max(1.0, abs(theta))
            pp, pm = params64(sc), params64(sc)
            pp[name][(i,) + comp] += h
            pm[name][(i,) + comp] -= h
            Lp, sp = smooth_loss(sc, vw, pp, w)
            Lm, sm = smooth_loss(sc, vw, pm, w)
            if not (sp == sig0 == sm):
                skipped += 1
                continue
            fd = (Lp - Lm) / (2 * h)
            an = G[(i,) + comp]
            err = abs(fd - an) / max(abs(an), 1e-3 * scale)
            worst = max(worst, err)
            assert err <= rtol, (name, i, comp, fd, an)
            checked += 1
    for j in range(6):
        xi = np.zeros(6)
        h = 1e-6
        xi[j] = h
        Lp, sp = smooth_loss(sc, vw, p0, w, pose=xi)
        Lm, sm = smooth_loss(sc, vw, p0, w, pose=-xi)
        if not (sp == sig0 == sm):
            skipped += 1
            continue
        fd = (Lp - Lm) / (2 * h)
        an = g["d_pose"][0, j]
        err = abs(fd - an) / max(abs(an), 1e-3 * np.abs(g["d_pose"]).max())
        worst = max(worst, err)
        assert err <= rtol, ("pose", j, fd, an)
        checked += 1
    return checked, skipped, worst


@pytest.mark.slow
def test_p9_fd_subcase():
    """P9: FP64 central differences on the 500-Gaussian 64x48 sub-case."""
    wl = fd_subcase()
    checked, skipped, worst = fd_check(wl.scene, wl.views, n_per_param=5)
    assert checked >= 25 and skipped <= checked // 3


@pytest.mark.parametrize("seed", [0, 1])
def test_p9_fd_tiny_sh3_posed(seed):
    """P9 on SH degree 3 with a non-identity pose (direction and pose terms)."""
    sc, vw = tiny_scene(40 + seed, n=16, width=24, height=20, sh_degree=3, pose_noise=0.2)
    checked, skipped, worst = fd_check(sc, vw, n_per_param=4, seed=seed)
    assert checked >= 15


def test_p9_fd_guard_clamp():
    """P9 with Gaussians far off-screen so the Jacobian guard clamp is active
    while their footprint still reaches the image."""
    rng = np.random.default_rng(5)
    n = 10
    means = np.stack([rng.uniform(1.0, 1.6, n), rng.uniform(-0.3, 0.3, n),
                      rng.uniform(1.5, 2.0, n)], 1).astype(np.float32)
    ls = np.log(rng.uniform(0.2, 0.6, (n, 3))).astype(np.float32)
    q = rng.normal(size=(n, 4)).astype(np.float32)
    sc = Scene(means, ls, q, rng.normal(1, 0.5, n).astype(np.float32),
               rng.random((n, 3)).astype(np.float32), np.array([0, n], np.int64))
    _, vw = tiny_scene(0, n=1, width=24, height=20)
    from oracle.project64 import project
    pr = project(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.colors, 0,
                 vw.viewmats[0], vw.intrinsics[0], vw.width, vw.height)
    assert np.any(np.abs(pr["rx"]) > pr["limx"])
    checked, skipped, worst = fd_check(sc, vw, n_per_param=4, seed=3)
    assert checked >= 10


def test_p10_translation_pose_identity():
    """P10: dL/drho = Rc sum_i dL/dmu_i (moving the camera by rho moves every
    mean by -Rc^T rho relative to it), SH view dependence included."""
    sc, vw = tiny_scene(7, n=30, width=32, height=24, sh_degree=3, pose_noise=0.3)
    rng = np.random.default_rng(1)
    w = weights(rng, vw.height, vw.width)
    g = render_backward(sc, vw, w[0][None], w[1][None], w[2][None])
    Rc = vw.viewmats[0][:, :3].astype(np.float64)
    lhs = g["d_pose"][0, :3]
    rhs = Rc @ g["d_means"].sum(0)
    # Rc is an FP32-rounded rotation, orthonormal only to ~1e-7
    assert np.abs(Rc @ Rc.T - np.eye(3)).max() < 3e-7
    np.testing.assert_allclose(lhs, rhs, rtol=1e-6, atol=1e-6 * np.abs(lhs).max())


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b.T
    return np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2], 1)


def test_p11_sim3_invariance():
    """P11 (Eq. gauss_update and the lift of Sec. III-B): applying a
    similarity to the Gaussians and the inverse to the camera leaves colour
    and alpha unchanged and scales depth by s (SH degree 0)."""
    sc, vw = tiny_scene(9, n=40, width=32, height=24, pose_noise=0.2)
    p = params64(sc)
    s = 1.7
    qR = np.array([0.8, 0.3, -0.4, 0.2])
    qR /= np.linalg.norm(qR)
    from oracle.project64 import quat_to_rot
    R = quat_to_rot(qR[None])[0]
    t = np.array([0.3, -0.2, 0.5])
    p2 = dict(p)
    p2["means"] = s * p["means"] @ R.T + t
    p2["log_scales"] = p["log_scales"] + math.log(s)
    p2["quats"] = _quat_mul(qR, p["quats"])
    vm = vw.viewmats[0].astype(np.float64)
    Rc, tc = vm[:, :3], vm[:, 3]
    vm2 = np.concatenate([Rc @ R.T, (s * tc - Rc @ R.T @ t)[:, None]], 1)
    c1, d1, a1, _ = render_smooth(p, 0, vm, vw.intrinsics[0], vw.width, vw.height, z_near=0.2)
    c2, d2, a2, _ = render_smooth(p2, 0, vm2, vw.intrinsics[0], vw.width, vw.height,
                                  z_near=0.2 * s)
    np.testing.assert_allclose(c2, c1, atol=1e-10)
    np.testing.assert_allclose(a2, a1, atol=1e-10)
    np.testing.assert_allclose(d2, s * d1, atol=1e-9)
    assert a1.max() > 0.5


def test_sh_basis_matches_scipy():
    """Real SH (CS phase) built from scipy's complex harmonics."""
    rng = np.random.default_rng(0)
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = sh_basis(d, 3)
    for l in range(4):
        for m in range(-l, l + 1):
            c = scipy.special.sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else (math.sqrt(2) * (c.real if m > 0 else c.imag))
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-13)


def test_sh_gradient_tangential_fd():
    """The tangential part of the polynomial gradients matches differences of
    the (scipy-pinned) basis along the sphere."""
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    dY = sh_basis_grad(d, 3)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        dp = (d + e) / np.linalg.norm(d + e, axis=1, keepdims=True)
        dm = (d - e) / np.linalg.norm(d - e, axis=1, keepdims=True)
        fd = (sh_basis(dp, 3) - sh_basis(dm, 3)) / (2 * h)
        tang = np.eye(3)[j][None] - d[:, j:j + 1] * d        # (I - dd^T) e_j
        an = np.einsum("nkj,nj->nk", dY, tang)
        np.testing.assert_allclose(fd, an, atol=1e-8)


def test_se3_exp_matches_matrix_exponential():
    rng = np.random.default_rng(2)
    for scale in (1e-9, 1e-3, 0.5, 2.0):
        xi = rng.normal(size=6) * scale
        tw = np.zeros((4, 4))
        tw[:3, :3] = np.array([[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]])
        tw[:3, 3] = xi[:3]
        np.testing.assert_allclose(exp_se3(xi), scipy.linalg.expm(tw), atol=1e-13)
    vm = np.concatenate([np.eye(3), np.ones((3, 1))], 1)
    np.testing.assert_allclose(apply_left(np.zeros(6), vm), vm, atol=0)
