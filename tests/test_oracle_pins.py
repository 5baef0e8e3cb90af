"""Pins of the CPU oracle against closed forms, invariants, brute force and
library routines (no GPU).  Each test names what it pins."""
import math

import numpy as np
import pytest

from oracle.composite import A_MAX, A_MIN, T_MIN
from oracle.keypath32 import keypath
from oracle.project64 import project
from oracle.render import Settings, render_view, render_backward
from oracle.smooth import render_smooth
from synth.scenes import Scene, Views, identity_view, small_plain, tiny_scene

F = np.float32


def one_view(W, H, fx, fy, cx, cy, vm=None):
    vm = identity_view() if vm is None else vm
    return Views(np.asarray(vm, F)[None], np.array([[fx, fy, cx, cy]], F),
                 np.zeros(1, np.int32), W, H)


def scene_of(means, log_scales, quats, opac, colors, sh_degree=0):
    n = len(means)
    return Scene(np.asarray(means, F), np.asarray(log_scales, F), np.asarray(quats, F),
                 np.asarray(opac, F), np.asarray(colors, F), np.array([0, n], np.int64),
                 sh_degree)


# ---------------------------------------------------------------- P1
@pytest.mark.parametrize("x0,y0,z0,ss,o", [(0.1, -0.05, 2.5, 0.03, 0.3),
                                           (-0.4, 0.3, 3.0, 0.05, -1.0),
                                           (0.0, 0.0, 2.0, 0.02, 4.0)])
def test_p1_single_isotropic_closed_form(x0, y0, z0, ss, o):
    """P1: one isotropic Gaussian, identity pose, guard clamp inactive.
    Sigma2 = ss^2 J J^T + 0.3 I with J J^T in closed form; every pixel has
    alpha = min(0.99, sigma exp(-d^T Sigma2^-1 d / 2)) if >= 1/255 else 0."""
    W, H, f = 96, 72, 80.0
    sc = scene_of([[x0, y0, z0]], [[math.log(ss)] * 3], [[1, 0, 0, 0]], [o], [[0.2, 0.5, 0.9]])
    vw = one_view(W, H, f, f, W / 2, H / 2)
    r = render_view(sc, vw, 0)
    x0, y0, z0, ss = (float(F(v)) for v in (x0, y0, z0, ss))
    ss = math.exp(float(F(math.log(ss))))
    JJ = np.array([[f * f * (1 + x0 * x0 / z0 ** 2) / z0 ** 2, f * f * x0 * y0 / z0 ** 4],
                   [f * f * x0 * y0 / z0 ** 4, f * f * (1 + y0 * y0 / z0 ** 2) / z0 ** 2]])
    S2 = ss * ss * JJ + 0.3 * np.eye(2)
    Q = np.linalg.inv(S2)
    sig = 1 / (1 + math.exp(-float(F(o))))
    u, v = f * x0 / z0 + W / 2, f * y0 / z0 + H / 2
    yy, xx = np.mgrid[0:H, 0:W]
    d = np.stack([u - (xx + 0.5), v - (yy + 0.5)], -1)
    q = np.einsum("hwi,ij,hwj->hw", d, Q, d)
    a = np.minimum(A_MAX, sig * np.exp(-0.5 * q))
    a = np.where(a >= A_MIN, a, 0.0)
    np.testing.assert_allclose(r["alpha"], a, atol=1e-12)
    np.testing.assert_allclose(r["depth"], z0 * a, atol=1e-11)
    for c, val in enumerate((0.2, 0.5, 0.9)):
        np.testing.assert_allclose(r["color"][c], float(F(val)) * a, atol=1e-12)


# ---------------------------------------------------------------- P2
def test_p2_exact_half_alpha_stack_and_ties():
    """P2: 16 identical Gaussians with sigma = 1/2 centred on a pixel centre:
    T halves exactly, 2^-13 >= 1e-4 > 2^-14, so exactly 13 are blended; equal
    depths are ordered by index, so colour = sum_{j<13} c_j 2^-(j+1)."""
    K = 16
    W, H = 128, 96
    cols = np.stack([np.linspace(0.05, 0.95, K), np.linspace(0.9, 0.1, K),
                     (np.arange(K) % 3) / 2.0], 1)
    sc = scene_of([[0, 0, 3.0]] * K, [[math.log(0.02)] * 3] * K, [[1, 0, 0, 0]] * K,
                  [0.0] * K, cols)
    vw = one_view(W, H, 100, 100, 64.5, 48.5)
    r = render_view(sc, vw, 0)
    px, py = 64, 48
    assert r["last"][py, px] == 13
    assert r["n_eval"][py, px] == 14
    assert r["alpha"][py, px] == 1 - 2.0 ** -13
    expect = sum(cols.astype(F)[j].astype(float) * 2.0 ** -(j + 1) for j in range(13))
    assert np.all(r["color"][:, py, px] == expect)
    assert r["depth"][py, px] == 3.0 * (1 - 2.0 ** -13)
    # the sorted list of that tile: equal keys, ascending Gaussian index
    t = (py // 16) * 8 + px // 16
    lo, hi = r["ranges"][t]
    assert list(r["vals"][lo:hi]) == list(range(K))


# ---------------------------------------------------------------- P3
def test_p3_alpha_clamp():
    """P3: sigma(20) rounds to 1 so alpha = 0.99f at the centre; with two
    stacked, T' = (1 - 0.99f)^2 < 1e-4f and only the first is blended."""
    W, H = 128, 96
    sc = scene_of([[0, 0, 3.0]] * 2, [[math.log(0.02)] * 3] * 2, [[1, 0, 0, 0]] * 2,
                  [20.0] * 2, [[0.3, 0.6, 0.9], [1.0, 1.0, 1.0]])
    vw = one_view(W, H, 100, 100, 64.5, 48.5)
    r = render_view(sc, vw, 0)
    assert (1 - A_MAX) ** 2 < T_MIN
    assert r["last"][48, 64] == 1 and r["n_eval"][48, 64] == 2
    np.testing.assert_array_equal(r["color"][:, 48, 64],
                                  A_MAX * np.array([0.3, 0.6, 0.9], F).astype(float))
    assert r["alpha"][48, 64] == A_MAX


# ---------------------------------------------------------------- P4
@pytest.mark.parametrize("factor,expect_in", [(1.001, True), (0.999, False)])
def test_p4_skip_rule(factor, expect_in):
    """P4: a pixel where sigma*G = (1/255)(1 +- 1e-3) is included / skipped."""
    W, H, f, z0, ss = 128, 96, 100.0, 3.0, 0.05
    ssf = math.exp(float(F(math.log(ss))))
    A = 1.0 / (ssf * ssf * (f / z0) ** 2 + 0.3)
    G = math.exp(-0.5 * A * 9.0)             # pixel 3 px right of the centre
    sig = A_MIN * factor / G
    o = math.log(sig / (1 - sig))
    sc = scene_of([[0, 0, z0]], [[math.log(ss)] * 3], [[1, 0, 0, 0]], [o], [[1, 1, 1]])
    vw = one_view(W, H, f, f, 64.5, 48.5)
    r = render_view(sc, vw, 0)
    a = r["alpha"][48, 67]
    if expect_in:
        assert a == pytest.approx(A_MIN * factor, rel=1e-6)
    else:
        assert a == 0.0
    assert r["alpha"][48, 64] > 0


# ---------------------------------------------------------------- P5 / P6 / P7
def _check_invariants(sc, vw, r):
    a, d, c = r["alpha"], r["depth"], r["color"]
    assert np.all(a <= 1 - T_MIN + 1e-15)
    assert np.all(r["T_final"] >= T_MIN)
    cmax = float(np.max(sc.colors)) if sc.sh_degree == 0 else np.inf
    assert np.all(c <= a[None] * cmax + 1e-12)
    zmax = float(np.max(r["setup"]["pr"]["z"], initial=0.0))
    assert np.all(d <= a * zmax + 1e-12)
    assert np.all(r["n_eval"] >= r["last"])


@pytest.mark.parametrize("seed", range(6))
def test_p5_p6_invariants_and_brute_force(seed):
    """P5 (T non-increasing, alpha <= 1-1e-4, colour/depth bounds) and P6
    (per-pixel walk over all Gaussians == per-tile walk, exactly)."""
    sc, vw = tiny_scene(seed, n=40, width=32, height=24, pose_noise=0.1 * (seed % 2))
    rt = render_view(sc, vw, 0, mode="tiled", keep=True)
    rb = render_view(sc, vw, 0, mode="brute")
    _check_invariants(sc, vw, rt)
    for key in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_array_equal(rt[key], rb[key])
    for _, _, piece in rt["pieces"]:
        Tb = piece["T_before"]
        if Tb.shape[1] > 1:
            w = piece["blended"]
            # transmittance never grows along the walk (up to the stop)
            assert np.all(np.diff(Tb, axis=1)[w[:, 1:]] <= 0)


def test_p6_brute_force_small_workload():
    wl = small_plain(0)
    rt = render_view(wl.scene, wl.views, 0, mode="tiled")
    rb = render_view(wl.scene, wl.views, 0, mode="brute")
    ok = ~rt["ambiguous"]
    for key in ("color", "depth", "alpha"):
        np.testing.assert_array_equal(rt[key][..., ok], rb[key][..., ok])
    assert rt["ambiguous"].sum() <= 5


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (32, 8), (32, 16)])
def test_p7_tile_shape_invariance(tile):
    """P7: images do not depend on the tile shape (exact in FP64)."""
    sc, vw = tiny_scene(3, n=50, width=48, height=40)
    r0 = render_view(sc, vw, 0, Settings())
    r1 = render_view(sc, vw, 0, Settings(tile_w=tile[0], tile_h=tile[1]))
    for key in ("color", "depth", "alpha", "T_final"):
        np.testing.assert_array_equal(r0[key], r1[key])


# ---------------------------------------------------------------- P8
def test_p8_key_list_independent_construction():
    """P8: sorted keys equal a per-tile construction (filter by rect, sort by
    (depth bits, index)); ascending; I = sum of tiles; ranges partition."""
    sc, vw = tiny_scene(11, n=60, width=64, height=48)
    r = render_view(sc, vw, 0)
    kp = r["setup"]["kp"]
    keys, vals, rng = r["keys"], r["vals"], r["ranges"]
    TX, TY = kp["TX"], kp["TY"]
    assert keys.shape[0] == int(kp["tiles"].sum())
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    pos = 0
    for t in range(TX * TY):
        tx, ty = t % TX, t // TX
        members = [(int(kp["zbits"][i]), i) for i in range(sc.n)
                   if kp["visible"][i] and kp["rect"][i][0] <= tx < kp["rect"][i][2]
                   and kp["rect"][i][1] <= ty < kp["rect"][i][3]]
        members.sort()
        lo, hi = rng[t]
        if not members:
            assert (lo, hi) == (0, 0)
            continue
        assert lo == pos and hi == pos + len(members)
        assert [m[1] for m in members] == list(vals[lo:hi])
        assert all(int(k) == (t << 32) | m[0] for k, m in zip(keys[lo:hi], members))
        pos = hi
    assert pos == keys.shape[0]


def test_keypath_matches_fp64_projection():
    """The FP32 key path agrees with the FP64 projection to FP32 accuracy,
    and culls exactly what the definition culls."""
    wl = small_plain(1)
    sc, vw = wl.scene, wl.views
    kp = keypath(sc.means, sc.log_scales, sc.quats, sc.opacity_logits,
                 vw.viewmats[0], vw.intrinsics[0], vw.width, vw.height)
    vis = kp["visible"]
    pr = project(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.colors, 0,
                 vw.viewmats[0], vw.intrinsics[0], vw.width, vw.height)
    np.testing.assert_allclose(kp["u"][vis], pr["u"][vis], rtol=1e-6)
    np.testing.assert_allclose(kp["v"][vis], pr["v"][vis], rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(kp["a"][vis], pr["S2"][vis, 0, 0], rtol=1e-5)
    np.testing.assert_allclose(kp["c"][vis], pr["S2"][vis, 1, 1], rtol=1e-5)
    np.testing.assert_allclose(kp["p"][vis], pr["p"][vis], rtol=1e-6, atol=1e-7)
    assert np.all(kp["zbits"][vis] == kp["p"][vis, 2].view(np.uint32))


# ---------------------------------------------------------------- P12
def test_p12_mass_integral():
    """P12: sum over pixels of alpha ~= 2 pi sqrt(det Sigma2) (sigma - 1/255),
    the exact integral of sigma exp(-d^T Q d/2) over the alpha >= 1/255
    ellipse, for a large unclamped footprint."""
    W, H = 256, 256
    sc = scene_of([[0.02, -0.01, 2.0]], [[math.log(0.15), math.log(0.08), math.log(0.1)]],
                  [[0.9, 0.2, -0.3, 0.1]], [0.5], [[1, 1, 1]])
    vw = one_view(W, H, 100, 100, 128, 128)
    r = render_view(sc, vw, 0)
    pr = r["setup"]["pr"]
    S2 = pr["S2"][0]
    sig = pr["sigma"][0]
    expect = 2 * math.pi * math.sqrt(np.linalg.det(S2)) * (sig - A_MIN)
    assert r["alpha"].sum() == pytest.approx(expect, rel=1e-3)


# ---------------------------------------------------------------- P13
def test_p13_culling():
    """P13: behind the near plane, NaN parameters, off-screen, and opacity
    that can never reach 1/255 produce no keys and zero gradients."""
    W, H = 64, 48
    means = [[0, 0, 0.1], [0, 0, -2.0], [np.nan, 0, 2], [50.0, 0, 2.0], [0, 0, 2.0],
             [0.1, 0.1, 2.0]]
    n = len(means)
    sc = scene_of(means, [[-3.0, -2.6, -3.3]] * n, [[0.9, 0.1, -0.2, 0.3]] * n,
                  [0.5, 0.5, 0.5, 0.5, -6.0, 0.5], [[1, 1, 1]] * n)
    vw = one_view(W, H, 50, 50, 32, 24)
    r = render_view(sc, vw, 0)
    assert set(np.unique(r["vals"])) == {5}
    g = render_backward(sc, vw, np.ones((1, 3, H, W)), np.ones((1, H, W)), np.ones((1, H, W)))
    for key in ("d_means", "d_log_scales", "d_quats", "d_colors"):
        assert np.all(g[key][:5] == 0) and np.any(g[key][5] != 0)
    assert np.all(g["d_opacity"][:5] == 0)


# ---------------------------------------------------------------- ambiguous branches
def _tile_pixels(r, st, W, H):
    """(pixel x, pixel y, list order) of every pixel of a rendered view."""
    su = r["setup"]
    TX = su["kp"]["TX"]
    for t in range(TX * su["kp"]["TY"]):
        tx, ty = t % TX, t // TX
        lo, hi = r["ranges"][t]
        order = su["local"][r["vals"][lo:hi] - su["g0"]]
        for y in range(ty * st.tile_h, min((ty + 1) * st.tile_h, H)):
            for x in range(tx * st.tile_w, min((tx + 1) * st.tile_w, W)):
                yield x, y, order


@pytest.mark.parametrize("seed", range(3))
def test_branches_reduce_to_composite(seed):
    """With no decision inside the ambiguity band the branch walk has one
    branch, equal to composite() exactly; with one, composite()'s outcome is
    among the branches."""
    from oracle.composite import composite_branches
    sc, vw = tiny_scene(seed, n=40, width=32, height=24, pose_noise=0.1 * (seed % 2))
    st = Settings()
    r = render_view(sc, vw, 0, st)
    rec = r["setup"]["rec"]
    for x, y, order in _tile_pixels(r, st, vw.width, vw.height):
        br = composite_branches(x + 0.5, y + 0.5, rec, order, np.zeros(3))
        want = (r["color"][:, y, x], r["depth"][y, x], r["alpha"][y, x], r["last"][y, x],
                r["n_eval"][y, x])
        hits = [b for b in br if np.all(b["color"] == want[0]) and b["depth"] == want[1]
                and b["alpha"] == want[2] and b["last"] == want[3] and b["n_eval"] == want[4]]
        if r["ambiguous"][y, x]:
            assert len(br) >= 2 and hits
        else:
            assert len(br) == 1 and len(hits) == 1


def test_branches_at_skip_and_stop_thresholds():
    """A pixel whose sigma*G sits 1e-6 (relative) above 1/255 yields the
    blended and the skipped outcome; a pixel whose transmittance after a
    blend sits 1e-6 above 1e-4 yields the stopped and the continued one."""
    from oracle.composite import composite_branches
    rec = dict(u=np.array([0.0]), v=np.array([0.0]), A=np.array([0.5]), B=np.array([0.0]),
               C=np.array([0.5]), sigma=np.array([0.5]), z=np.array([2.0]),
               color=np.array([[1.0, 0.5, 0.25]]))
    # sigma exp(-x^2/4) = (1/255)(1 + 1e-6) at sample point (x, 0)
    x = math.sqrt(-4.0 * math.log(A_MIN * (1 + 1e-6) / 0.5))
    br = composite_branches(x, 0.0, rec, [0], np.zeros(3))
    assert sorted(b["last"] for b in br) == [0, 1]
    a = [b["alpha"] for b in br if b["last"] == 1][0]
    assert a == pytest.approx(A_MIN * (1 + 1e-6), rel=1e-12)
    assert all(b["alpha"] == 0.0 for b in br if b["last"] == 0)
    # stop: T after the third blend equals 1e-4 (1 + 1e-6); no alpha near 0.99
    a1 = 0.95
    a3 = 1.0 - T_MIN * (1 + 1e-6) / (1.0 - a1) ** 2
    rec2 = dict(u=np.zeros(4), v=np.zeros(4), A=np.full(4, 1.0), B=np.zeros(4),
                C=np.full(4, 1.0), sigma=np.array([a1, a1, a3, 0.5]),
                z=np.array([1.0, 2.0, 3.0, 4.0]), color=np.eye(4)[:, :3])
    br = composite_branches(0.0, 0.0, rec2, [0, 1, 2, 3], np.zeros(3))
    got = sorted((b["last"], b["n_eval"]) for b in br)
    # continuing past the third entry, the fourth stops either way:
    # 1e-4 (1 + 1e-6) (1 - 0.5) < 1e-4
    assert got == [(2, 3), (3, 4)]
    cont = [b for b in br if b["last"] == 3][0]
    assert cont["T_final"] == pytest.approx(T_MIN * (1 + 1e-6), rel=1e-9)
    stop = [b for b in br if b["last"] == 2][0]
    assert stop["T_final"] == pytest.approx((1.0 - a1) ** 2, rel=1e-12)


def test_branches_cover_ambiguous_pixels_of_small_workload():
    """On the 2,000-Gaussian workload every pixel flagged ambiguous has two
    or more branches, one of them composite()'s own outcome; a sample of the
    other pixels has exactly that one."""
    from oracle.composite import composite_branches
    wl = small_plain(0)
    st = Settings()
    r = render_view(wl.scene, wl.views, 0, st)
    rec = r["setup"]["rec"]
    rng = np.random.default_rng(0)
    n_amb = 0
    for x, y, order in _tile_pixels(r, st, wl.views.width, wl.views.height):
        amb = r["ambiguous"][y, x]
        if not amb and rng.random() > 0.02:
            continue
        br = composite_branches(x + 0.5, y + 0.5, rec, order, np.zeros(3))
        hit = [b for b in br if np.all(b["color"] == r["color"][:, y, x])
               and b["alpha"] == r["alpha"][y, x] and b["n_eval"] == r["n_eval"][y, x]]
        assert hit and (len(br) >= 2 if amb else len(br) == 1)
        n_amb += int(amb)
    assert n_amb == int(r["ambiguous"].sum()) > 0
