"""Helpers for the GPU parity tests: run the HIP path through the C ABI on
synthetic scenes and bring its outputs back as numpy."""
from __future__ import annotations

import sys

import numpy as np

IMG_TOL = 1e-5
GRAD_TOL = 1e-3
# Two runs of the same backward: each pair's screen-space gradient is summed
# with float atomics from many tiles, in an order that differs between runs,
# so the parameter gradients agree to rounding of those sums (measured up to
# 2.3e-5 of a tensor's max-norm), not bit for bit.
RERUN_TOL = 1e-4


def announce(msg: str):
    """Name the GPU case about to run (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def to_gpu(scene, views):
    from paper_2605_10760_amd import SceneTensors, ViewTensors
    return SceneTensors.from_numpy(scene), ViewTensors.from_numpy(views)


def make_rasterizer(scene, views, tile=(16, 16), max_instances=None, chunk=0, **opts):
    """A Rasterizer planned for this call; `opts` are the compositing options
    (fwd_batch, bwd_batch, persistent)."""
    from paper_2605_10760_amd import Rasterizer
    so = scene.set_offsets
    P = int(sum(so[s + 1] - so[s] for s in views.view_set))
    return Rasterizer(views.width, views.height, max(P, 1), views.n,
                      max_instances=max_instances, tile=tile, chunk=chunk, **opts), P


def gpu_forward(scene, views, tile=(16, 16), z_near=0.2, bg=(0.0, 0.0, 0.0), export=True,
                rast=None, chunk=0, n_blend=False, **opts):
    """Forward on the GPU; returns dict of numpy outputs (+ binning export)."""
    import torch
    st_, vt = to_gpu(scene, views)
    if rast is None:
        rast, P = make_rasterizer(scene, views, tile, chunk=chunk, **opts)
    else:
        P = int(sum(scene.set_offsets[s + 1] - scene.set_offsets[s] for s in views.view_set))
    c, d, a, state, ne = rast.forward(st_, vt, z_near=z_near, bg=bg, n_eval=True)
    # the same forward without the per-pixel entry counts runs its own kernel
    # instantiation (the one the training step uses): bit-identical images
    c2, d2, a2, st2 = rast.forward(st_, vt, z_near=z_near, bg=bg)
    for x, y, name in ((c, c2, "color"), (d, d2, "depth"), (a, a2, "alpha")):
        assert torch.equal(x, y), f"forward without entry counts differs in {name}"
    del c2, d2, a2, st2
    counts = rast.poll(state)
    out = dict(color=c.cpu().numpy(), depth=d.cpu().numpy(), alpha=a.cpu().numpy(),
               n_eval=ne.cpu().numpy(), counts=counts, state=state, rast=rast, scene_t=st_,
               views_t=vt, P=P)
    if export:
        out["dbg"] = rast.debug_export(state, views.n, P, int(counts["instances"]),
                                       n_blend=n_blend)
    torch.cuda.synchronize()
    return out


def oracle_blend_count(views, orc_keep):
    """Entries blended per pixel [V,H,W] from oracle renders made with
    keep=True (a blended entry has a positive weight)."""
    out = np.zeros((views.n, views.height, views.width), np.int64)
    for k, r in enumerate(orc_keep):
        for xx, yy, piece in r["pieces"]:
            out[k, yy, xx] = (piece["w"] > 0).sum(axis=1)
    return out


def pair_to_gauss(scene, views):
    """Map pair id -> (view, global Gaussian index)."""
    so = scene.set_offsets
    vids, gids = [], []
    for v, s in enumerate(views.view_set):
        n = int(so[s + 1] - so[s])
        vids.append(np.full(n, v))
        gids.append(so[s] + np.arange(n))
    return np.concatenate(vids), np.concatenate(gids)


def grad_rel_err(got, ref):
    """(max-norm, 2-norm) errors relative to the reference's norms."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    d = got - ref
    ninf = np.abs(ref).max() if ref.size else 0.0
    n2 = np.linalg.norm(ref)
    return (np.abs(d).max() / ninf if ninf > 0 else np.abs(d).max(),
            np.linalg.norm(d) / n2 if n2 > 0 else np.linalg.norm(d))


# ---------------------------------------------------------------- oracle comparisons
from oracle.composite import composite_branches  # noqa: E402
from oracle.render import Settings, render_view  # noqa: E402


def _oracle_views(scene, views, st=Settings(), keep=False):
    return [render_view(scene, views, k, st, keep=keep) for k in range(views.n)]


def _check_keys(scene, views, g, orc, st=Settings()):
    dbg = g["dbg"]
    vid, gid = pair_to_gauss(scene, views)
    so = scene.set_offsets
    T = dbg["TX"] * dbg["TY"]
    off = 0
    straddle = set()
    for k, r in enumerate(orc):
        kp = r["setup"]["kp"]
        n = kp["visible"].shape[0]
        zk = dbg["zkeys"][off:off + n]
        vis = zk != 0xFFFFFFFF
        s0 = so[views.view_set[k]]
        straddle |= set((s0 + np.nonzero(kp["straddle"])[0]).tolist())
        ok = ~kp["straddle"]
        np.testing.assert_array_equal(vis[ok], kp["visible"][ok], err_msg=f"culling, view {k}")
        both = vis & kp["visible"] & ok
        np.testing.assert_array_equal(zk[both], kp["zbits"][both], err_msg=f"depth bits, view {k}")
        np.testing.assert_array_equal(dbg["rects"][off:off + n][both].astype(np.int64),
                                      kp["rect"][both], err_msg=f"rects, view {k}")
        off += n
    # sorted instances: (global tile, depth bits, Gaussian) per instance
    inst = dbg["inst"].astype(np.int64)
    tile_of = np.zeros(inst.shape[0], np.int64)
    for t in range(views.n * T):
        lo, hi = dbg["ranges"][t]
        tile_of[lo:hi] = t
    g_keys = (tile_of.astype(np.uint64) << np.uint64(32)) | dbg["zkeys"][inst].astype(np.uint64)
    g_vals = gid[inst]
    o_keys = np.concatenate([r["keys"] for r in orc])
    o_vals = np.concatenate([r["vals"] for r in orc])
    if straddle:
        sel_g = ~np.isin(g_vals, list(straddle))
        sel_o = ~np.isin(o_vals, list(straddle))
        g_keys, g_vals, o_keys, o_vals = g_keys[sel_g], g_vals[sel_g], o_keys[sel_o], o_vals[sel_o]
    else:
        assert g["counts"]["instances"] == o_keys.shape[0]
        # the oracle's ranges are per view; shift to global positions
        base = np.cumsum([0] + [r["keys"].shape[0] for r in orc])
        o_rng = np.concatenate([np.where(r["ranges"][:, 1:2] > r["ranges"][:, :1],
                                         r["ranges"] + base[k], 0) for k, r in enumerate(orc)])
        np.testing.assert_array_equal(dbg["ranges"].astype(np.int64), o_rng, err_msg="tile ranges")
    np.testing.assert_array_equal(g_keys, o_keys, err_msg="sorted keys")
    np.testing.assert_array_equal(g_vals, o_vals, err_msg="sorted values")


def _check_images(views, g, orc, st=Settings()):
    for k, r in enumerate(orc):
        ok = ~r["ambiguous"]
        zmax = max(1.0, float(np.max(r["setup"]["pr"]["z"], initial=0.0)))
        dc = np.abs(g["color"][k] - r["color"])[:, ok].max(initial=0.0)
        da = np.abs(g["alpha"][k] - r["alpha"])[ok].max(initial=0.0)
        dd = np.abs(g["depth"][k] - r["depth"])[ok].max(initial=0.0)
        assert dc <= IMG_TOL, f"colour err {dc} view {k}"
        assert da <= IMG_TOL, f"alpha err {da} view {k}"
        assert dd <= IMG_TOL * zmax, f"depth err {dd} view {k}"
        np.testing.assert_array_equal(g["n_eval"][k][ok], r["n_eval"][ok])
        assert r["ambiguous"].mean() <= 1e-3
        check_ambiguous_pixels(g, k, r, views, st, zmax)


def check_ambiguous_pixels(g, k, r, views, st, zmax):
    """A pixel with a decision inside the ambiguity band must equal one of
    the oracle's outcomes of that decision (both ways, every such decision)."""
    ys, xs = np.nonzero(r["ambiguous"])
    if ys.size == 0:
        return 0
    su = r["setup"]
    TX = su["kp"]["TX"]
    for y, x in zip(ys, xs):
        t = (y // st.tile_h) * TX + x // st.tile_w
        lo, hi = r["ranges"][t]
        order = su["local"][r["vals"][lo:hi] - su["g0"]]
        br = composite_branches(x + 0.5, y + 0.5, su["rec"], order, np.asarray(st.bg, float))
        assert len(br) >= 2
        hit = any(np.abs(g["color"][k][:, y, x] - b["color"]).max() <= IMG_TOL
                  and abs(g["alpha"][k][y, x] - b["alpha"]) <= IMG_TOL
                  and abs(g["depth"][k][y, x] - b["depth"]) <= IMG_TOL * zmax
                  and g["n_eval"][k][y, x] == b["n_eval"] for b in br)
        assert hit, f"ambiguous pixel ({x}, {y}) of view {k} matches none of {len(br)} branches"
    return ys.size


def _upstream(views, seed, orc):
    rng = np.random.default_rng(seed)
    V, H, W = views.n, views.height, views.width
    gc = rng.normal(size=(V, 3, H, W)).astype(np.float32)
    gd = (0.3 * rng.normal(size=(V, H, W))).astype(np.float32)
    ga = rng.normal(size=(V, H, W)).astype(np.float32)
    for k, r in enumerate(orc):
        amb = r["ambiguous"]
        gc[k][:, amb] = 0
        gd[k][amb] = 0
        ga[k][amb] = 0
    return gc, gd, ga


def _gpu_backward(g, gc, gd, ga):
    import torch
    t = lambda a: torch.from_numpy(a).cuda()
    out = g["rast"].backward(g["scene_t"], g["views_t"], g["state"], t(gc), t(gd), t(ga))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


GMAP = dict(d_means="d_means", d_log_scales="d_log_scales", d_quats="d_quats",
            d_opacity_logits="d_opacity", d_colors="d_colors", d_pose="d_pose")




def check_ambiguous_samples(g, k, scene, views, px, py, ro, zmax, st=Settings()):
    """Sampled pixels (render_pixels output `ro`) with a decision inside the
    ambiguity band must equal one of the oracle's branches, walked over every
    visible Gaussian of the view in (depth bits, index) order."""
    from oracle.render import setup_view
    amb = np.nonzero(ro["ambiguous"])[0]
    if amb.size == 0:
        return 0
    su = setup_view(scene, views, k, st)
    vis = su["vis"]
    order = np.lexsort((vis, su["kp"]["zbits"][vis]))
    for i in amb:
        x, y = int(px[i]), int(py[i])
        br = composite_branches(x + 0.5, y + 0.5, su["rec"], order, np.asarray(st.bg, float))
        hit = any(np.abs(g["color"][k][:, y, x] - b["color"]).max() <= IMG_TOL
                  and abs(g["alpha"][k][y, x] - b["alpha"]) <= IMG_TOL
                  and abs(g["depth"][k][y, x] - b["depth"]) <= 10 * IMG_TOL * zmax
                  for b in br)
        assert hit, f"ambiguous sample ({x}, {y}) of view {k} matches none of {len(br)} branches"
    return amb.size
