"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact: culling, depth keys, tile rects, the sorted instance list and
tile ranges.  Images: colour and alpha within 1e-5 absolute, depth within
1e-5 * max(1, z_max), on pixels without an ambiguous FP32/FP64 decision.
Gradients: per tensor, max-abs and 2-norm of the error within 1e-3 of the
reference's max-abs and 2-norm, upstream gradients zeroed on ambiguous
pixels."""
import numpy as np
import pytest

from gpu_harness import (GMAP, GRAD_TOL, IMG_TOL, RERUN_TOL, _check_images, _check_keys,
                         _gpu_backward, _oracle_views, _upstream, announce, check_ambiguous_samples,
                         gpu_forward, grad_rel_err, oracle_blend_count, pair_to_gauss,
                         to_gpu)
from oracle.render import Settings, render_backward, render_pixels, render_view
from oracle.keypath32 import keypath
from synth.scenes import fused_map, multi_agent, room_plain, small_plain, tiny_scene

pytestmark = pytest.mark.gpu


def _scene_case(name):
    if name == "small-plain":
        wl = small_plain(0)
        return wl.scene, wl.views
    if name.startswith("tiny"):
        seed = int(name.split("-")[1])
        return tiny_scene(seed, n=60, width=70, height=45, pose_noise=0.15 * (seed % 2))
    if name == "multi-agent-small":
        wl = multi_agent(scale=0.002, keyframes=3, width=160, height=120)
        return wl.scene, wl.views
    if name.startswith("sh"):
        # SH degrees 1..3 (each its own kernel instantiation), rows of
        # exactly (degree + 1)^2 coefficients
        deg = int(name[2:])
        seed = {1: 11, 2: 12, 3: 5}[deg]
        return tiny_scene(seed, n=80, width=96, height=64, sh_degree=deg, pose_noise=0.2)
    raise KeyError(name)


CASES = ["small-plain", "tiny-0", "tiny-1", "tiny-2", "multi-agent-small", "sh1", "sh2", "sh3"]


@pytest.mark.parametrize("case", CASES)
def test_binning_bit_exact(case):
    announce(f"binning {case}")
    scene, views = _scene_case(case)
    g = gpu_forward(scene, views)
    orc = _oracle_views(scene, views)
    _check_keys(scene, views, g, orc)


@pytest.mark.parametrize("case", CASES)
def test_forward_images(case):
    announce(f"forward {case}")
    scene, views = _scene_case(case)
    g = gpu_forward(scene, views)
    orc = _oracle_views(scene, views)
    _check_images(views, g, orc)
    dbg = g["dbg"]
    for k, r in enumerate(orc):
        ok = ~r["ambiguous"]
        np.testing.assert_array_equal(dbg["last"][k][ok], r["last"][ok])
        # final transmittance, relative: a blended entry left out anywhere in
        # a pixel's list would change it by a factor (1 - alpha) <= 254/255
        tf, to = dbg["t_final"][k][ok].astype(np.float64), r["T_final"][ok]
        assert np.all(np.abs(tf - to) <= 1e-4 * to + 1e-9), f"T_final view {k}"


@pytest.mark.parametrize("case", CASES)
def test_backward_gradients(case):
    announce(f"backward {case}")
    scene, views = _scene_case(case)
    g = gpu_forward(scene, views, export=False)
    orc = _oracle_views(scene, views)
    gc, gd, ga = _upstream(views, 7, orc)
    got = _gpu_backward(g, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


def test_batched_equals_per_view():
    """All views in one call == one call per view (bit-identical forward)."""
    announce("batched vs per-view")
    scene, views = _scene_case("multi-agent-small")
    gb = gpu_forward(scene, views, export=False)
    for k in range(views.n):
        gk = gpu_forward(scene, views.select([k]), export=False)
        np.testing.assert_array_equal(gb["color"][k], gk["color"][0])
        np.testing.assert_array_equal(gb["depth"][k], gk["depth"][0])
        np.testing.assert_array_equal(gb["alpha"][k], gk["alpha"][0])


@pytest.mark.parametrize("tile", [(8, 8), (16, 8), (8, 16), (32, 8), (32, 16), (16, 32)])
def test_tile_shape_bit_identical(tile):
    announce(f"tile shape {tile}")
    scene, views = _scene_case("small-plain")
    g0 = gpu_forward(scene, views, export=False)
    g1 = gpu_forward(scene, views, tile=tile, export=False)
    for key in ("color", "depth", "alpha"):
        np.testing.assert_array_equal(g0[key], g1[key])


def test_tile_shape_keys_bit_exact():
    announce("tile shape 8x8 keys")
    scene, views = _scene_case("tiny-0")
    g = gpu_forward(scene, views, tile=(8, 8))
    orc = _oracle_views(scene, views, Settings(tile_w=8, tile_h=8))
    _check_keys(scene, views, g, orc, Settings(tile_w=8, tile_h=8))


def test_forward_deterministic():
    announce("determinism")
    scene, views = _scene_case("multi-agent-small")
    a = gpu_forward(scene, views, export=False)
    b = gpu_forward(scene, views, export=False, rast=a["rast"])
    for key in ("color", "depth", "alpha", "n_eval"):
        np.testing.assert_array_equal(a[key], b[key])


def test_edge_cases_empty_and_ragged():
    """Everything culled; an empty set; a ragged 37x23 image; one Gaussian."""
    announce("edge cases")
    sc, vw = tiny_scene(2, n=10, width=37, height=23)
    sc.means[:, 2] = -5.0                       # all behind the camera
    g = gpu_forward(sc, vw)
    assert g["counts"]["visible_pairs"] == 0 and g["counts"]["instances"] == 0
    assert np.all(g["alpha"] == 0) and np.all(g["color"] == 0)
    # one Gaussian, ragged image, plus an empty set rendered by a second view
    sc1, vw1 = tiny_scene(4, n=1, width=37, height=23)
    sc1.set_offsets = np.array([0, 1, 1], np.int64)
    from synth.scenes import Views
    vw2 = Views(np.concatenate([vw1.viewmats] * 2), np.concatenate([vw1.intrinsics] * 2),
                np.array([0, 1], np.int32), 37, 23)
    g = gpu_forward(sc1, vw2)
    orc = _oracle_views(sc1, vw2)
    _check_keys(sc1, vw2, g, orc)
    _check_images(vw2, g, orc)
    assert np.all(g["alpha"][1] == 0)


def test_overflow_reported():
    """A plan too small for the binning's (pair, tile row) entries reports
    GSR_E_OVERFLOW via poll; fit_capacity re-plans to the measured need."""
    announce("overflow")
    from paper_2605_10760_amd import Rasterizer
    scene, views = _scene_case("small-plain")
    st_, vt = to_gpu(scene, views)
    r = Rasterizer(views.width, views.height, scene.n, 1, max_instances=100)
    c, d, a, state = r.forward(st_, vt)
    cnt = r.poll(state, raise_on_overflow=False)
    assert cnt["overflow"] and cnt["row_entries"] > 100 and cnt["instances"] >= cnt["row_entries"]
    from paper_2605_10760_amd import GsrError
    with pytest.raises(GsrError):
        r.poll(state)
    r.fit_capacity(st_, vt)
    c, d, a, state = r.forward(st_, vt)
    assert not r.poll(state)["overflow"]


def test_pose_delta_kernel():
    announce("pose delta")
    import torch
    from oracle.se3 import apply_left
    from paper_2605_10760_amd import apply_pose_delta
    rng = np.random.default_rng(3)
    vm = np.stack([np.concatenate([np.linalg.qr(rng.normal(size=(3, 3)))[0],
                                   rng.normal(size=(3, 1))], 1) for _ in range(5)]).astype(np.float32)
    xi = (rng.normal(size=(5, 6)) * np.array([[0.1, 0.1, 0.1, 0.3, 0.3, 0.3]])).astype(np.float32)
    xi[0] = 0
    xi[1, 3:] = 1e-6
    out = apply_pose_delta(torch.from_numpy(vm).cuda(), torch.from_numpy(xi).cuda()).cpu().numpy()
    for k in range(5):
        np.testing.assert_allclose(out[k], apply_left(xi[k], vm[k]), atol=2e-6)


def test_autograd_function_matches_backward():
    announce("autograd")
    import torch
    from paper_2605_10760_amd import rasterize
    scene, views = _scene_case("tiny-1")
    g = gpu_forward(scene, views, export=False)
    st_, vt = g["scene_t"], g["views_t"]
    params = [p.clone().requires_grad_(True) for p in
              (st_.means, st_.log_scales, st_.quats, st_.opacity_logits, st_.colors)]
    pose = torch.zeros((views.n, 6), device="cuda", requires_grad=True)
    c, d, a = rasterize(g["rast"], *params, vt.viewmats, vt.intrinsics, scene.set_offsets,
                        views.view_set, views.width, views.height, pose_delta=pose)
    rng = np.random.default_rng(1)
    w = [torch.from_numpy(rng.normal(size=x.shape).astype(np.float32)).cuda() for x in (c, d, a)]
    loss = (c * w[0]).sum() + (d * w[1]).sum() + (a * w[2]).sum()
    loss.backward()
    ref = g["rast"].backward(st_, vt, g["state"], w[0], w[1], w[2])
    for p, key in zip(params, ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors")):
        e_inf, e_2 = grad_rel_err(p.grad.cpu().numpy(), ref[key].cpu().numpy())
        assert e_inf <= RERUN_TOL, (key, e_inf)
    e_inf, _ = grad_rel_err(pose.grad.cpu().numpy(), ref["d_pose"].cpu().numpy())
    assert e_inf <= RERUN_TOL


# ----------------------------------------------------------------- full size
def _sampled_full_size_checks(scene, views, view_ids, n_gauss=3000, n_pix=192, seed=0):
    g = gpu_forward(scene, views)
    dbg = g["dbg"]
    rng = np.random.default_rng(seed)
    so = scene.set_offsets
    T = dbg["TX"] * dbg["TY"]
    inst = dbg["inst"].astype(np.int64)
    # global properties: I = sum of rect areas; each tile's list ascending in
    # (depth bits, pair id); ranges partition [0, I)
    r = dbg["rects"].astype(np.int64)
    vis = dbg["zkeys"] != 0xFFFFFFFF
    areas = ((r[:, 2] - r[:, 0]) * (r[:, 3] - r[:, 1]))[vis]
    assert areas.sum() == g["counts"]["instances"] == inst.shape[0]
    rg = dbg["ranges"].astype(np.int64)
    nz = rg[:, 1] > rg[:, 0]
    assert np.all(rg[nz][1:, 0] == rg[nz][:-1, 1]) and rg[nz][0, 0] == 0
    assert rg[nz][-1, 1] == inst.shape[0]
    z = dbg["zkeys"][inst].astype(np.uint64)
    key = (z << np.uint64(32)) | inst.astype(np.uint64)
    tile_of = np.repeat(np.nonzero(nz)[0], (rg[nz, 1] - rg[nz, 0]))
    same = tile_of[1:] == tile_of[:-1]
    assert np.all(key[1:][same] > key[:-1][same])
    off = np.concatenate([[0], np.cumsum([so[s + 1] - so[s] for s in views.view_set])])
    for k in view_ids:
        s = views.view_set[k]
        n = int(so[s + 1] - so[s])
        idx = rng.choice(n, size=min(n_gauss, n), replace=False)
        kp = keypath(scene.means[so[s] + idx], scene.log_scales[so[s] + idx],
                     scene.quats[so[s] + idx], scene.opacity_logits[so[s] + idx],
                     views.viewmats[k], views.intrinsics[k], views.width, views.height)
        zk = dbg["zkeys"][off[k] + idx]
        ok = ~kp["straddle"]
        np.testing.assert_array_equal((zk != 0xFFFFFFFF)[ok], kp["visible"][ok])
        both = kp["visible"] & ok
        np.testing.assert_array_equal(zk[both], kp["zbits"][both])
        np.testing.assert_array_equal(dbg["rects"][off[k] + idx][both].astype(np.int64),
                                      kp["rect"][both])
        px = rng.integers(0, views.width, n_pix)
        py = rng.integers(0, views.height, n_pix)
        ro = render_pixels(scene, views, k, px, py)
        ok = ~ro["ambiguous"]
        zmax = max(1.0, float(ro["depth"].max() / max(ro["alpha"].max(), 1e-9)))
        dc = np.abs(g["color"][k][:, py, px].T - ro["color"])[ok].max()
        da = np.abs(g["alpha"][k][py, px] - ro["alpha"])[ok].max()
        dd = np.abs(g["depth"][k][py, px] - ro["depth"])[ok].max()
        assert dc <= IMG_TOL and da <= IMG_TOL and dd <= IMG_TOL * 10 * zmax, (k, dc, da, dd)
        check_ambiguous_samples(g, k, scene, views, px, py, ro, zmax)
    return g


@pytest.mark.slow
def test_room_plain_full_size_sampled():
    """300k Gaussians, one 1200x680 view: global binning properties, sampled
    Gaussians' keys and sampled pixels against the oracle."""
    announce("room 300k 1200x680 full size")
    wl = room_plain()
    _sampled_full_size_checks(wl.scene, wl.views, [0])


@pytest.mark.slow
def test_multi_agent_full_size_sampled():
    """Six submaps (50k..600k) x 8 keyframes at 640x480 in one batch."""
    announce("multi-agent 1.67M x 8 640x480 full size")
    wl = multi_agent()
    _sampled_full_size_checks(wl.scene, wl.views, [0, 47], n_pix=96)


@pytest.mark.slow
def test_room_plain_window_gradients():
    """Full-size 1200x680 view, upstream gradient on a 40x24 window: the
    oracle's gradient of that window (every Gaussian reaching it)."""
    announce("room 300k gradient window")
    wl = room_plain(n=300_000)
    scene, views = wl.scene, wl.views
    g = gpu_forward(scene, views, export=False)
    rng = np.random.default_rng(4)
    H, W = views.height, views.width
    gc = np.zeros((1, 3, H, W), np.float32)
    gd = np.zeros((1, H, W), np.float32)
    ga = np.zeros((1, H, W), np.float32)
    y0, x0 = 320, 576
    gc[0, :, y0:y0 + 24, x0:x0 + 40] = rng.normal(size=(3, 24, 40))
    gd[0, y0:y0 + 24, x0:x0 + 40] = 0.3 * rng.normal(size=(24, 40))
    ga[0, y0:y0 + 24, x0:x0 + 40] = rng.normal(size=(24, 40))
    TX = -(-W // 16)
    tiles = sorted({(y // 16) * TX + x // 16 for y in range(y0, y0 + 24) for x in range(x0, x0 + 40)})
    rv = render_view(scene, views, 0, tiles=tiles)
    amb = rv["ambiguous"]
    gc[0][:, amb] = 0
    gd[0][amb] = 0
    ga[0][amb] = 0
    got = _gpu_backward(g, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


def _window_upstream(scene, views, k, y0, x0, h, w, seed, st=Settings()):
    """Upstream gradients that are zero except on an h x w window of view k,
    with the oracle's ambiguous pixels zeroed."""
    rng = np.random.default_rng(seed)
    V, H, W = views.n, views.height, views.width
    gc = np.zeros((V, 3, H, W), np.float32)
    gd = np.zeros((V, H, W), np.float32)
    ga = np.zeros((V, H, W), np.float32)
    gc[k, :, y0:y0 + h, x0:x0 + w] = rng.normal(size=(3, h, w))
    gd[k, y0:y0 + h, x0:x0 + w] = 0.3 * rng.normal(size=(h, w))
    ga[k, y0:y0 + h, x0:x0 + w] = rng.normal(size=(h, w))
    TX = -(-W // st.tile_w)
    tiles = sorted({(y // st.tile_h) * TX + x // st.tile_w
                    for y in range(y0, y0 + h) for x in range(x0, x0 + w)})
    amb = render_view(scene, views, k, st, tiles=tiles)["ambiguous"]
    gc[k][:, amb] = 0
    gd[k][amb] = 0
    ga[k][amb] = 0
    return gc, gd, ga


@pytest.mark.slow
def test_room_1m_autograd_full_size():
    """1M Gaussians, one 1200x680 view, through the autograd Function with a
    pose delta: sampled pixels against the oracle, and the gradients of an
    upstream window (every parameter and the pose) against the oracle's."""
    announce("room 1M 1200x680 autograd full size")
    import torch
    from paper_2605_10760_amd import rasterize
    wl = room_plain(seed=20, n=1_000_000)
    scene, views = wl.scene, wl.views
    g = gpu_forward(scene, views, export=False)
    st_, vt = g["scene_t"], g["views_t"]
    params = [p.clone().requires_grad_(True) for p in
              (st_.means, st_.log_scales, st_.quats, st_.opacity_logits, st_.colors)]
    pose = torch.zeros((1, 6), device="cuda", requires_grad=True)
    c, d, a = rasterize(g["rast"], *params, vt.viewmats, vt.intrinsics, scene.set_offsets,
                        views.view_set, views.width, views.height, pose_delta=pose)
    rng = np.random.default_rng(21)
    px = rng.integers(0, views.width, 96)
    py = rng.integers(0, views.height, 96)
    ro = render_pixels(scene, views, 0, px, py)
    ok = ~ro["ambiguous"]
    cn, dn, an = c.detach().cpu().numpy(), d.detach().cpu().numpy(), a.detach().cpu().numpy()
    assert np.abs(cn[0][:, py, px].T - ro["color"])[ok].max() <= IMG_TOL
    assert np.abs(an[0][py, px] - ro["alpha"])[ok].max() <= IMG_TOL
    gc, gd, ga = _window_upstream(scene, views, 0, 300, 560, 24, 40, seed=22)
    t = lambda x: torch.from_numpy(x).cuda()
    loss = (c * t(gc)).sum() + (d * t(gd)).sum() + (a * t(ga)).sum()
    loss.backward()
    ref = render_backward(scene, views, gc, gd, ga)
    got = dict(zip(("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors"),
                   (p.grad.cpu().numpy() for p in params)))
    got["d_pose"] = pose.grad.cpu().numpy()
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


@pytest.mark.slow
def test_fused_map_full_size_sampled():
    """3M Gaussians with SH degree 3, 16 forward-only + 32 fwd+bwd views at
    1200x680 in one batch: sampled tiles' sorted lists bit-exact and sampled
    pixels for a forward-only view and a keyframe, and a keyframe's window
    gradients against the oracle."""
    announce("fused map 3M SH3 48 x 1200x680 full size")
    wl = fused_map()
    scene, views = wl.scene, wl.views
    g = gpu_forward(scene, views)
    dbg = g["dbg"]
    TX, TY = dbg["TX"], dbg["TY"]
    T = TX * TY
    N = scene.n
    rng = np.random.default_rng(31)
    for k in (3, 20):
        assert bool(views.needs_grad[k]) == (k >= 16)
        kp = keypath(scene.means, scene.log_scales, scene.quats, scene.opacity_logits,
                     views.viewmats[k], views.intrinsics[k], views.width, views.height)
        vis = kp["visible"]
        rect = kp["rect"]
        for t in rng.choice(T, size=40, replace=False):
            ty, tx = divmod(int(t), TX)
            cov = vis & (rect[:, 0] <= tx) & (tx < rect[:, 2]) & (rect[:, 1] <= ty) & (ty < rect[:, 3])
            ids = np.nonzero(cov)[0]
            if kp["straddle"][ids].any():
                continue
            want = ids[np.lexsort((ids, kp["zbits"][ids]))]
            lo, hi = dbg["ranges"][k * T + t]
            got = dbg["inst"][lo:hi].astype(np.int64) - k * N
            np.testing.assert_array_equal(got, want, err_msg=f"view {k} tile {t}")
        px = rng.integers(0, views.width, 64)
        py = rng.integers(0, views.height, 64)
        ro = render_pixels(scene, views, k, px, py)
        ok = ~ro["ambiguous"]
        assert np.abs(g["color"][k][:, py, px].T - ro["color"])[ok].max() <= IMG_TOL
        assert np.abs(g["alpha"][k][py, px] - ro["alpha"])[ok].max() <= IMG_TOL
    gc, gd, ga = _window_upstream(scene, views, 20, 330, 600, 16, 32, seed=32)
    got = _gpu_backward(g, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga, view_ids=[20])
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


def test_profile_stages_and_autotune():
    announce("profile + autotune")
    from paper_2605_10760_amd import autotune
    scene, views = _scene_case("small-plain")
    g = gpu_forward(scene, views, export=False)
    r = g["rast"]
    r.profile(True)
    c, d, a, state = r.forward(g["scene_t"], g["views_t"])
    import torch
    gc = torch.ones_like(c)
    r.backward(g["scene_t"], g["views_t"], state, gc, None, None)
    ms = r.stage_ms()
    r.profile(False)
    assert all(v > 0 for v in ms.values()), ms
    best = autotune(g["scene_t"], g["views_t"])
    assert best["tile"] in [(16, 16), (16, 8), (8, 16), (8, 8), (32, 8), (32, 16), (16, 32)]
    assert best["ms"] > 0 and best["chunk"] in (0, 64, 128, 256)
    assert best["fwd_batch"] in (1, 2) and best["bwd_batch"] in (1, 2, 4)
    g2 = gpu_forward(scene, views, tile=best["tile"], chunk=best["chunk"], export=False,
                     fwd_batch=best["fwd_batch"], bwd_batch=best["bwd_batch"],
                     persistent=best["persistent"])
    np.testing.assert_array_equal(g2["color"], g["color"])


# (entries per lane in the forward, per lane in the backward, persistent queue,
# tiles per backward wave)
RENDER_OPTS = [(2, 2, False, 1), (1, 1, True, 1), (2, 4, True, 1), (1, 4, False, 1),
               (1, 2, True, 2)]


@pytest.mark.parametrize("case", ["multi-agent-small", "sh3"])
@pytest.mark.parametrize("opts", RENDER_OPTS)
def test_render_options(case, opts):
    """Every compositing batch size and the persistent tile queue: forward
    outputs bit-identical to the default launch (the per-pixel arithmetic
    and its order do not change), gradients against the oracle."""
    fb, bb, pers, cols = opts
    announce(f"render options fb={fb} bb={bb} persistent={pers} cols={cols} {case}")
    scene, views = _scene_case(case)
    g0 = gpu_forward(scene, views)
    g1 = gpu_forward(scene, views, fwd_batch=fb, bwd_batch=bb, persistent=pers, bwd_cols=cols)
    for key in ("color", "depth", "alpha", "n_eval"):
        np.testing.assert_array_equal(g0[key], g1[key], err_msg=key)
    for key in ("t_final", "last"):
        np.testing.assert_array_equal(g0["dbg"][key], g1["dbg"][key], err_msg=key)
    orc = _oracle_views(scene, views)
    gc, gd, ga = _upstream(views, 11, orc)
    got = _gpu_backward(g1, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)
    # a second backward on the same saved state (the persistent queue's
    # cursor restarts every call)
    got2 = _gpu_backward(g1, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got2[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


@pytest.mark.parametrize("case", ["tiny-0", "tiny-1", "multi-agent-small", "sh3"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8)])
def test_backward_two_tiles_per_wave(case, tile):
    """The backward on pairs of tiles of a tile row (each entry compared
    with its position in each tile's own list; 70-pixel-wide views leave an
    odd tile column at the row end): gradients against the oracle and
    against the one-tile backward of the same forward."""
    announce(f"backward two tiles per wave {case} {tile}")
    scene, views = _scene_case(case)
    g1 = gpu_forward(scene, views, tile=tile, export=False)
    g2 = gpu_forward(scene, views, tile=tile, export=False, bwd_cols=2)
    np.testing.assert_array_equal(g1["color"], g2["color"])
    orc = _oracle_views(scene, views)
    gc, gd, ga = _upstream(views, 11, orc)
    a = _gpu_backward(g1, gc, gd, ga)
    b = _gpu_backward(g2, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(b[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)
        e_inf, _ = grad_rel_err(b[k_gpu], a[k_gpu])
        assert e_inf <= RERUN_TOL, (k_gpu, e_inf)


@pytest.mark.parametrize("case", ["small-plain", "multi-agent-small", "sh3"])
def test_blend_count_matches_oracle(case):
    """The debug count of blended entries per pixel (the unit of the
    compositing arithmetic) equals the oracle's on unambiguous pixels."""
    announce(f"blend count {case}")
    scene, views = _scene_case(case)
    g = gpu_forward(scene, views, n_blend=True)
    orc = _oracle_views(scene, views, keep=True)
    want = oracle_blend_count(views, orc)
    for k, r in enumerate(orc):
        ok = ~r["ambiguous"]
        np.testing.assert_array_equal(g["dbg"]["n_blend"][k][ok], want[k][ok])
        assert np.all(g["dbg"]["n_blend"][k] <= g["dbg"]["last"][k])


def test_graph_replay_matches_eager():
    """forward+backward captured once in a HIP graph and replayed several
    times, with eager work in between, reproduce the eager results."""
    announce("graph replay")
    import torch
    scene, views = _scene_case("multi-agent-small")
    g = gpu_forward(scene, views, export=False)
    r, st_, vt = g["rast"], g["scene_t"], g["views_t"]
    V, H, W = views.n, views.height, views.width
    state = r.new_state()
    out = (torch.empty((V, 3, H, W), device="cuda"), torch.empty((V, H, W), device="cuda"),
           torch.empty((V, H, W), device="cuda"))
    rng = np.random.default_rng(2)
    gc = torch.from_numpy(rng.normal(size=(V, 3, H, W)).astype(np.float32)).cuda()
    gd = torch.from_numpy(rng.normal(size=(V, H, W)).astype(np.float32)).cuda()
    grads = r.backward(st_, vt, g["state"], gc, gd, None)
    ref = {k: v.clone() for k, v in grads.items()}
    eager_color = g["color"]

    def step():
        r.forward(st_, vt, state=state, out=out)
        r.backward(st_, vt, state, gc, gd, None, out=grads)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(4):
        for v_ in grads.values():
            v_.fill_(float("nan"))
        out[0].fill_(-1.0)
        r.forward(st_, vt)          # unrelated eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out[0].cpu().numpy(), eager_color)
        for k in ref:
            e_inf, _ = grad_rel_err(grads[k].cpu().numpy(), ref[k].cpu().numpy())
            assert e_inf <= RERUN_TOL, (rep, k, e_inf)


def test_backward_repeatable_and_needs_grad_mask():
    """Two backwards of one forward agree (the per-pair gradient rows are left
    clean); views with needs_grad = 0 contribute nothing and get zero pose
    gradients, matching the oracle restricted to the other views."""
    announce("backward repeat + needs_grad")
    import torch
    scene, views = _scene_case("multi-agent-small")
    views.needs_grad = (np.arange(views.n) % 3 != 1)
    g = gpu_forward(scene, views, export=False)
    orc = _oracle_views(scene, views)
    gc, gd, ga = _upstream(views, 11, orc)
    a = _gpu_backward(g, gc, gd, ga)
    b = _gpu_backward(g, gc, gd, ga)
    for k in a:
        e_inf, _ = grad_rel_err(a[k], b[k])
        assert e_inf <= RERUN_TOL, k
    assert np.all(a["d_pose"][~views.needs_grad] == 0)
    ref = render_backward(scene, views, gc, gd, ga, view_ids=np.nonzero(views.needs_grad)[0])
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(a[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)


@pytest.mark.slow
def test_multi_agent_full_size_backward_windows():
    """The benched batch at its own size (6 submaps of 50k..600k Gaussians x
    8 keyframes at 640x480): per-tile sorted lists of 48 sampled tiles in 4
    views against an independent construction from the oracle's key path;
    then upstream gradients on 24x40 windows of two keyframes of the largest
    submap and one keyframe of every other submap, and every parameter
    gradient plus all 48 pose rows against the oracle's (views without a
    window must get exactly zero pose gradient)."""
    announce("multi-agent 1.67M x 8 640x480 full-size backward windows")
    wl = multi_agent()
    scene, views = wl.scene, wl.views
    g = gpu_forward(scene, views)
    dbg = g["dbg"]
    TX, TY = dbg["TX"], dbg["TY"]
    T = TX * TY
    so = scene.set_offsets
    pair_off = np.concatenate([[0], np.cumsum([so[s + 1] - so[s] for s in views.view_set])])
    rng = np.random.default_rng(41)
    for k in (2, 13, 30, 45):
        s = views.view_set[k]
        sl = slice(so[s], so[s + 1])
        kp = keypath(scene.means[sl], scene.log_scales[sl], scene.quats[sl],
                     scene.opacity_logits[sl], views.viewmats[k], views.intrinsics[k],
                     views.width, views.height)
        vis, rect = kp["visible"], kp["rect"]
        for t in rng.choice(T, size=12, replace=False):
            ty, tx = divmod(int(t), TX)
            cov = vis & (rect[:, 0] <= tx) & (tx < rect[:, 2]) & (rect[:, 1] <= ty) & (ty < rect[:, 3])
            ids = np.nonzero(cov)[0]
            if kp["straddle"][ids].any():
                continue
            want = ids[np.lexsort((ids, kp["zbits"][ids]))]
            lo, hi = dbg["ranges"][k * T + t]
            got = dbg["inst"][lo:hi].astype(np.int64) - pair_off[k]
            np.testing.assert_array_equal(got, want, err_msg=f"view {k} tile {t}")
    # windows: keyframes 40 and 43 of the 600k submap, one of every other
    win_views = [40, 43, 0, 9, 18, 27, 36]
    V, H, W = views.n, views.height, views.width
    gc = np.zeros((V, 3, H, W), np.float32)
    gd = np.zeros((V, H, W), np.float32)
    ga = np.zeros((V, H, W), np.float32)
    for i, k in enumerate(win_views):
        y0 = int(rng.integers(0, H - 24))
        x0 = int(rng.integers(0, W - 40))
        a, b, c = _window_upstream(scene, views, k, y0, x0, 24, 40, seed=50 + i)
        gc[k], gd[k], ga[k] = a[k], b[k], c[k]
    got = _gpu_backward(g, gc, gd, ga)
    ref = render_backward(scene, views, gc, gd, ga, view_ids=win_views)
    for k_gpu, k_ref in GMAP.items():
        e_inf, e_2 = grad_rel_err(got[k_gpu], ref[k_ref])
        assert e_inf <= GRAD_TOL and e_2 <= GRAD_TOL, (k_gpu, e_inf, e_2)
    others = np.setdiff1d(np.arange(V), win_views)
    assert np.all(got["d_pose"][others] == 0)
    for k in win_views:
        e_inf, _ = grad_rel_err(got["d_pose"][k], ref["d_pose"][k])
        assert e_inf <= GRAD_TOL, (k, e_inf)
