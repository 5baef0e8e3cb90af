"""Pins of the oracle's mapping-loss extras and seeding (Sec. III-A, Eq.
(map_loss)): closed forms, central differences, a plane's normals, and
back-projection through the pose."""
import numpy as np

from oracle.mapping import (depth_normals, iso_loss, iso_loss_grad, normal_loss,
                            normal_loss_grad, seed)


def test_iso_closed_form_and_fd():
    ls = np.log(np.array([[1.0, 2.0, 3.0], [0.5, 0.5, 0.5]]))
    # |1-2| + |2-2| + |3-2| = 2; an isotropic Gaussian costs nothing
    assert abs(iso_loss(ls) - 2.0) < 1e-12
    rng = np.random.default_rng(0)
    ls = rng.normal(-2, 0.5, (30, 3))
    g = iso_loss_grad(ls)
    h = 1e-7
    for _ in range(20):
        idx = tuple(rng.integers(0, s) for s in ls.shape)
        p, m = ls.copy(), ls.copy()
        p[idx] += h
        m[idx] -= h
        fd = (iso_loss(p) - iso_loss(m)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(fd))


def test_plane_normals():
    """A plane through depth z = z0 + gx x + gy y (camera frame) has the
    normal -(-gx, -gy, 1)/|.| facing the camera, at every interior pixel."""
    H, W = 9, 12
    intr = np.array([[20.0, 22.0, 6.1, 4.3]])
    fx, fy, cx, cy = intr[0]
    gx, gy, z0 = 0.3, -0.2, 2.0
    u = (np.arange(W) + 0.5 - cx) / fx
    v = (np.arange(H) + 0.5 - cy) / fy
    # z = z0 + gx z u + gy z v  =>  z = z0 / (1 - gx u - gy v)
    d = z0 / (1 - gx * u[None, :] - gy * v[:, None])
    n, valid = depth_normals(d[None], intr)
    want = -np.array([-gx, -gy, 1.0]) / np.linalg.norm([-gx, -gy, 1.0])
    assert valid[0, 1:-1, 1:-1].all() and not valid[0, 0].any()
    np.testing.assert_allclose(n[0, 1:-1, 1:-1], np.broadcast_to(want, (H - 2, W - 2, 3)),
                               atol=1e-12)
    # the loss against that normal is 0 and against its opposite is 2
    prior = np.broadcast_to(want, (1, H, W, 3))
    assert abs(normal_loss(d[None], prior, intr)) < 1e-12
    assert abs(normal_loss(d[None], -prior, intr) - 2.0) < 1e-12


def test_normal_loss_grad_fd():
    rng = np.random.default_rng(1)
    V, H, W = 2, 7, 9
    intr = np.array([[15.0, 16.0, 4.5, 3.4], [14.0, 15.0, 4.4, 3.6]])
    d = 1.5 + 0.3 * rng.random((V, H, W))
    d[1, 0, 3] = 0.0  # a hole: neighbouring normals drop out
    pr = rng.normal(size=(V, H, W, 3))
    pr /= np.linalg.norm(pr, axis=-1, keepdims=True)
    g = normal_loss_grad(d, pr, intr)
    h = 1e-7
    for idx in [(0, 3, 4), (1, 1, 1), (0, 0, 5), (1, 6, 8), (1, 2, 3), (0, 4, 0)]:
        p, m = d.copy(), d.copy()
        p[idx] += h
        m[idx] -= h
        fd = (normal_loss(p, pr, intr) - normal_loss(m, pr, intr)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * np.abs(g).max(), idx


def test_seed_back_projects_through_the_pose():
    rng = np.random.default_rng(2)
    H, W = 6, 8
    d = 1 + rng.random((H, W))
    d[2, 3] = 0.0
    col = rng.random((3, H, W))
    ang = 0.4
    R = np.array([[np.cos(ang), 0, np.sin(ang)], [0, 1, 0], [-np.sin(ang), 0, np.cos(ang)]])
    t = np.array([0.1, -0.2, 0.3])
    vm = np.concatenate([R, t[:, None]], 1)
    intr = np.array([10.0, 11.0, 4.0, 3.0])
    g = seed(d, col, vm, intr, stride=1, opacity_logit=-2.0)
    assert g["means"].shape == (H * W - 1, 3)
    # every mean projects back to its pixel centre at its depth
    p = g["means"] @ R.T + t
    jj, ii = np.divmod(np.array([q for q in range(H * W) if q != 2 * W + 3]), W)
    np.testing.assert_allclose(p[:, 2], d[jj, ii], rtol=1e-12)
    np.testing.assert_allclose(p[:, 0] / p[:, 2] * intr[0] + intr[2], ii + 0.5, atol=1e-9)
    np.testing.assert_allclose(p[:, 1] / p[:, 2] * intr[1] + intr[3], jj + 0.5, atol=1e-9)
    np.testing.assert_array_equal(g["colors"], col[:, jj, ii].T)
    assert np.all(g["opacity_logits"] == -2.0)
    # interior pixel on a fronto-parallel patch: scale = footprint d / f average
    d2 = np.full((5, 5), 2.0)
    g2 = seed(d2, np.zeros((3, 5, 5)), np.concatenate([np.eye(3), np.zeros((3, 1))], 1),
              np.array([10.0, 10.0, 2.5, 2.5]))
    assert abs(np.exp(g2["log_scales"][12, 0]) - 0.2) < 1e-12
