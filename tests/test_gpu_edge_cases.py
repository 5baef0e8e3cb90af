"""GPU parity on the rasterizer's constructed edge cases, through the C ABI.

The oracle pins these scenes on the CPU (exact stack at alpha 1/2 with
equal-depth ties, the 0.99 clamp, the 1/255 skip boundary, culling of
behind-camera, NaN, off-screen and never-visible Gaussians, the Jacobian
guard clamp); here the HIP path renders them and its keys, images, last and
evaluation counts and gradients are compared with the oracle's, plus scenes
that exercise the same rules at larger sizes: equal camera depths across many
binning chunks and segments, and many Gaussians blended at the clamp inside a
gradient test.
"""
import math

import numpy as np
import pytest

from gpu_harness import (GMAP, GRAD_TOL, IMG_TOL, _check_images, _check_keys, _gpu_backward,
                         _oracle_views, _upstream, announce, gpu_forward, grad_rel_err)
from oracle.composite import A_MAX, A_MIN
from oracle.render import Settings, render_backward, render_view
from synth.scenes import Scene, Views, identity_view, multi_agent, tiny_scene

pytestmark = pytest.mark.gpu

F = np.float32
CULLED = 0xFFFFFFFF


def scene_of(means, log_scales, quats, opac, colors):
    n = len(means)
    return Scene(np.asarray(means, F), np.asarray(log_scales, F), np.asarray(quats, F),
                 np.asarray(opac, F), np.asarray(colors, F), np.array([0, n], np.int64), 0)


def one_view(W, H, fx, fy, cx, cy):
    return Views(identity_view().astype(F)[None], np.array([[fx, fy, cx, cy]], F),
                 np.zeros(1, np.int32), W, H)


def full_check(sc, vw, seed=7, grad=True):
    """Keys bit-exact, images (ambiguous pixels against the oracle's
    branches), last positions, and the gradients of random upstream images."""
    g = gpu_forward(sc, vw)
    orc = _oracle_views(sc, vw)
    _check_keys(sc, vw, g, orc)
    _check_images(vw, g, orc)
    for k, r in enumerate(orc):
        ok = ~r["ambiguous"]
        np.testing.assert_array_equal(g["dbg"]["last"][k][ok], r["last"][ok])
    if not grad:
        return g, orc, None, None
    gc, gd, ga = _upstream(vw, seed, orc)
    got = _gpu_backward(g, gc, gd, ga)
    ref = render_backward(sc, vw, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)
    return g, orc, got, ref


def test_half_alpha_stack_exact_and_ties():
    """16 identical Gaussians at sigma = 1/2 on a pixel centre (equal depths):
    exactly 13 blended (2^-13 >= 1e-4 > 2^-14), the 14th examined and not
    blended, the tile's list in ascending index order, colour the exact sum
    of c_j 2^-(j+1)."""
    announce("edge: half-alpha stack")
    K = 16
    cols = np.stack([np.linspace(0.05, 0.95, K), np.linspace(0.9, 0.1, K),
                     (np.arange(K) % 3) / 2.0], 1)
    sc = scene_of([[0, 0, 3.0]] * K, [[math.log(0.02)] * 3] * K, [[1, 0, 0, 0]] * K, [0.0] * K,
                  cols)
    vw = one_view(128, 96, 100, 100, 64.5, 48.5)
    g, orc, _, _ = full_check(sc, vw)
    px, py = 64, 48
    assert not orc[0]["ambiguous"].any()
    assert g["dbg"]["last"][0][py, px] == 13
    assert g["n_eval"][0][py, px] == 14
    assert g["alpha"][0][py, px] == F(1.0 - 2.0 ** -13)
    expect = sum(cols.astype(F)[j].astype(np.float64) * 2.0 ** -(j + 1) for j in range(13))
    assert np.abs(g["color"][0][:, py, px] - expect).max() <= 1e-6
    assert abs(g["depth"][0][py, px] - 3.0 * (1 - 2.0 ** -13)) <= 3e-6
    t = (py // 16) * 8 + px // 16
    lo, hi = g["dbg"]["ranges"][t]
    assert list(g["dbg"]["inst"][lo:hi]) == list(range(K))


def test_alpha_clamp_forward_and_zero_gradient():
    """sigma(20) rounds to 1: alpha = 0.99f at the centre; with two stacked,
    (1 - 0.99f)^2 < 1e-4f so only the first is blended.  An upstream colour
    gradient on the clamped pixel alone gives exactly zero gradients to every
    geometric parameter and the opacity (the clamp's derivative is zero), and
    a non-zero colour gradient to the first Gaussian only."""
    announce("edge: 0.99 clamp")
    sc = scene_of([[0, 0, 3.0]] * 2, [[math.log(0.02)] * 3] * 2, [[1, 0, 0, 0]] * 2,
                  [20.0] * 2, [[0.3, 0.6, 0.9], [1.0, 1.0, 1.0]])
    vw = one_view(128, 96, 100, 100, 64.5, 48.5)
    g, orc, _, _ = full_check(sc, vw)
    px, py = 64, 48
    assert g["dbg"]["last"][0][py, px] == 1 and g["n_eval"][0][py, px] == 2
    assert g["alpha"][0][py, px] == F(A_MAX)
    want = A_MAX * np.array([0.3, 0.6, 0.9], F).astype(np.float64)
    assert np.abs(g["color"][0][:, py, px] - want).max() <= 1e-7
    # the oracle's own record of the centre pixel: clamped and blended
    r = render_view(sc, vw, 0, keep=True)
    clamped_px = 0
    for xx, yy, p in r["pieces"]:
        if "clamped" in p:
            hit = (p["clamped"] & p["blended"]).any(axis=1)
            clamped_px += int(hit.sum())
            assert set(zip(xx[hit], yy[hit])) <= {(px, py)}
    assert clamped_px == 1
    gc = np.zeros((1, 3, 96, 128), F)
    gc[0, :, py, px] = [0.7, -1.3, 0.4]
    got = _gpu_backward(g, gc, np.zeros((1, 96, 128), F), np.zeros((1, 96, 128), F))
    for key in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_pose"):
        assert np.all(got[key] == 0), key
    assert np.all(got["d_colors"][1] == 0) and np.all(got["d_colors"][0] != 0)
    ref = render_backward(sc, vw, gc, None, None)
    np.testing.assert_allclose(got["d_colors"], ref["d_colors"], rtol=1e-6, atol=0)


@pytest.mark.parametrize("factor,expect_in", [(1.001, True), (0.999, False)])
def test_skip_threshold_boundary(factor, expect_in):
    """A pixel where sigma*G = (1/255)(1 +- 1e-3): blended above, skipped
    below (alpha exactly 0)."""
    announce(f"edge: 1/255 boundary x{factor}")
    W, H, f, z0, ss = 128, 96, 100.0, 3.0, 0.05
    ssf = math.exp(float(F(math.log(ss))))
    A = 1.0 / (ssf * ssf * (f / z0) ** 2 + 0.3)
    G = math.exp(-0.5 * A * 9.0)             # pixel 3 px right of the centre
    sig = A_MIN * factor / G
    o = math.log(sig / (1 - sig))
    sc = scene_of([[0, 0, z0]], [[math.log(ss)] * 3], [[1, 0, 0, 0]], [o], [[1, 1, 1]])
    vw = one_view(W, H, f, f, 64.5, 48.5)
    g, orc, _, _ = full_check(sc, vw)
    a = float(g["alpha"][0][48, 67])
    if expect_in:
        assert a == pytest.approx(A_MIN * factor, rel=1e-4)
        assert g["dbg"]["last"][0][48, 67] == 1
    else:
        assert a == 0.0 and g["dbg"]["last"][0][48, 67] == 0
    assert g["alpha"][0][48, 64] > 0


def test_culled_gaussians_no_keys_zero_gradients():
    """Behind the near plane, behind the camera, a NaN mean, far off-screen,
    and an opacity that can never reach 1/255: no keys and exactly zero
    gradients (no NaN); the one visible Gaussian gets non-zero gradients."""
    announce("edge: culling")
    W, H = 64, 48
    means = [[0, 0, 0.1], [0, 0, -2.0], [np.nan, 0, 2], [50.0, 0, 2.0], [0, 0, 2.0],
             [0.1, 0.1, 2.0]]
    n = len(means)
    sc = scene_of(means, [[-3.0, -2.6, -3.3]] * n, [[0.9, 0.1, -0.2, 0.3]] * n,
                  [0.5, 0.5, 0.5, 0.5, -6.0, 0.5], [[1, 1, 1]] * n)
    vw = one_view(W, H, 50, 50, 32, 24)
    g = gpu_forward(sc, vw)
    zk = g["dbg"]["zkeys"]
    assert np.all(zk[:5] == CULLED) and zk[5] != CULLED
    assert g["counts"]["visible_pairs"] == 1
    assert set(np.unique(g["dbg"]["inst"]).tolist()) == {5}
    ones = (np.ones((1, 3, H, W), F), np.ones((1, H, W), F), np.ones((1, H, W), F))
    got = _gpu_backward(g, *ones)
    ref = render_backward(sc, vw, *ones)
    for key in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors"):
        assert np.all(got[key][:5] == 0), key
        assert np.any(got[key][5] != 0), key
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


def test_guard_clamp_active():
    """Gaussians far outside the field of view (the Jacobian's x/z clamped to
    1.3 half-widths) whose footprints still reach the image."""
    announce("edge: guard clamp")
    from oracle.project64 import project
    rng = np.random.default_rng(5)
    n = 10
    means = np.stack([rng.uniform(1.0, 1.6, n), rng.uniform(-0.3, 0.3, n),
                      rng.uniform(1.5, 2.0, n)], 1)
    ls = np.log(rng.uniform(0.2, 0.6, (n, 3)))
    q = rng.normal(size=(n, 4))
    sc = scene_of(means, ls, q, rng.normal(1, 0.5, n), rng.random((n, 3)))
    _, vw = tiny_scene(0, n=1, width=24, height=20)
    pr = project(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.colors, 0,
                 vw.viewmats[0], vw.intrinsics[0], vw.width, vw.height)
    assert np.any(np.abs(pr["rx"]) > pr["limx"])
    g, orc, _, _ = full_check(sc, vw)
    assert g["counts"]["visible_pairs"] >= 5


def test_clamped_opacities_in_gradient_test():
    """The small multi-agent batch with 12% of the opacity logits in
    U[5, 9] (sigma > 0.99): the clamp is reached by hundreds of blended
    entries, and every gradient still matches the oracle's."""
    announce("edge: clamped opacities, multi-agent small")
    wl = multi_agent(scale=0.002, keyframes=3, width=160, height=120)
    sc, vw = wl.scene, wl.views
    rng = np.random.default_rng(13)
    sel = rng.random(sc.n) < 0.12
    sc.opacity_logits[sel] = rng.uniform(5.0, 9.0, int(sel.sum())).astype(F)
    n_clamped = 0
    for k in range(vw.n):
        r = render_view(sc, vw, k, keep=True)
        n_clamped += sum(int((p["clamped"] & p["blended"]).sum())
                         for _, _, p in r["pieces"] if "clamped" in p)
    assert n_clamped > 100
    full_check(sc, vw, seed=14)


def test_equal_depth_ties_across_chunks_and_segments():
    """12,000 Gaussians on four depth planes (camera z exactly 2, 2.5, 3 or
    3.5), two views of one set: most keys tie, and the order of equal keys
    (ascending Gaussian index) must survive the depth sort, the row binning's
    chunks and the tile binning's segments bit for bit."""
    announce("edge: equal-depth ties")
    rng = np.random.default_rng(17)
    n = 12000
    z = rng.choice([2.0, 2.5, 3.0, 3.5], n)
    xy = rng.uniform(-0.85, 0.85, (n, 2)) * z[:, None] * np.array([1.0, 0.75])
    sc = Scene(np.concatenate([xy, z[:, None]], 1).astype(F),
               rng.normal(-3.3, 0.3, (n, 3)).astype(F), rng.normal(size=(n, 4)).astype(F),
               rng.normal(0, 1, n).astype(F), rng.random((n, 3)).astype(F),
               np.array([0, n], np.int64))
    vm2 = identity_view().copy()
    vm2[0, 3] = 0.1                      # a sideways shift keeps camera z exact
    vw = Views(np.stack([identity_view(), vm2]).astype(F), np.array([[150, 150, 128, 96]] * 2, F),
               np.zeros(2, np.int32), 256, 192)
    g, orc, _, _ = full_check(sc, vw, grad=False)
    keys = np.concatenate([r["keys"] for r in orc])
    assert (np.diff(keys.astype(np.int64)) == 0).sum() > 30000
    # also with the smallest binning chunk (more chunk boundaries)
    g2 = gpu_forward(sc, vw, chunk=64)
    _check_keys(sc, vw, g2, orc)
