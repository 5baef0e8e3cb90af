"""Whole-view forward and backward of the rasterizer (test infrastructure
only): key path -> FP64 projection -> binning -> compositing, and the exact
FP64 gradient of the outputs with respect to the Gaussian parameters and the
camera pose.

Views render the Gaussian set they are tagged with (one submap per agent,
Sec. III-A; the fused map of Sec. III-C is a single set).  Gradients of
Gaussians seen by several views of their set are summed over those views.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .binning import duplicate, sort_keys, tile_ranges
from .composite import composite, pixel_grid
from .keypath32 import keypath
from .project64 import project, project_backward


@dataclass
class Settings:
    z_near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)
    tile_w: int = 16
    tile_h: int = 16


def _set_slice(scene, views, k):
    s = int(views.view_set[k])
    return int(scene.set_offsets[s]), int(scene.set_offsets[s + 1])


def setup_view(scene, views, k, st: Settings):
    """Key path, FP64 projection of the kept Gaussians, and the splat table."""
    g0, g1 = _set_slice(scene, views, k)
    kp = keypath(scene.means[g0:g1], scene.log_scales[g0:g1], scene.quats[g0:g1],
                 scene.opacity_logits[g0:g1], views.viewmats[k], views.intrinsics[k],
                 views.width, views.height, st.tile_w, st.tile_h, st.z_near)
    vis = np.nonzero(kp["visible"])[0]
    sl = g0 + vis
    pr = project(scene.means[sl], scene.log_scales[sl], scene.quats[sl],
                 scene.opacity_logits[sl], scene.colors[sl], scene.sh_degree,
                 views.viewmats[k], views.intrinsics[k], views.width, views.height)
    rec = dict(u=pr["u"], v=pr["v"], A=pr["conic"][:, 0], B=pr["conic"][:, 1],
               C=pr["conic"][:, 2], sigma=pr["sigma"], z=pr["z"], color=pr["color"])
    local = np.full(g1 - g0, -1, np.int64)
    local[vis] = np.arange(vis.shape[0])
    return dict(g0=g0, g1=g1, kp=kp, vis=vis, pr=pr, rec=rec, local=local)


def bin_view(setup, k, st: Settings, width, height):
    """Sorted (key, value) list and tile ranges of view k (tile ids global
    over views: view k owns ids [k*TX*TY, (k+1)*TX*TY))."""
    kp = setup["kp"]
    TX, TY = kp["TX"], kp["TY"]
    off = k * TX * TY
    gidx = setup["g0"] + np.arange(setup["g1"] - setup["g0"])
    keys, vals = duplicate(kp, gidx, off)
    keys, vals = sort_keys(keys, vals)
    rng = tile_ranges(keys - np.uint64(off << 32) if keys.size else keys, TX * TY)
    return keys, vals, rng


def render_view(scene, views, k, st: Settings = Settings(), mode="tiled",
                keep=False, tiles=None):
    """Render view k.  mode 'tiled' walks per-tile sorted lists; 'brute'
    walks all kept Gaussians in (depth bits, index) order per pixel.
    `tiles` (tiled mode) restricts compositing to those tile indices; the
    other pixels are left at colour 0, alpha 0, T 1."""
    W, H = views.width, views.height
    su = setup_view(scene, views, k, st)
    rec, bg = su["rec"], np.asarray(st.bg, float)
    color = np.zeros((3, H, W))
    depth = np.zeros((H, W))
    alpha = np.zeros((H, W))
    T_final = np.ones((H, W))
    last = np.zeros((H, W), np.int64)
    n_eval = np.zeros((H, W), np.int64)
    amb = np.zeros((H, W), bool)
    tiles_kept = []
    out = dict(setup=su)
    if mode == "tiled":
        keys, vals, rng = bin_view(su, k, st, W, H)
        out.update(keys=keys, vals=vals, ranges=rng)
        TX, TY = su["kp"]["TX"], su["kp"]["TY"]
        for t in (range(TX * TY) if tiles is None else tiles):
            tx, ty = t % TX, t // TX
            x0, y0 = tx * st.tile_w, ty * st.tile_h
            xx, yy, sx, sy = pixel_grid(x0, y0, min(x0 + st.tile_w, W),
                                        min(y0 + st.tile_h, H))
            lo, hi = rng[t]
            order = su["local"][vals[lo:hi] - su["g0"]]
            r = composite(sx, sy, rec, order, bg, keep=keep)
            _scatter(r, xx, yy, color, depth, alpha, T_final, last, n_eval, amb)
            if keep:
                tiles_kept.append((xx, yy, r))
    elif mode == "brute":
        vis = su["vis"]
        zb = su["kp"]["zbits"][vis]
        order = np.lexsort((vis, zb))
        for y in range(H):
            xx, yy, sx, sy = pixel_grid(0, y, W, y + 1)
            r = composite(sx, sy, rec, order, bg, keep=keep)
            _scatter(r, xx, yy, color, depth, alpha, T_final, last, n_eval, amb)
            if keep:
                tiles_kept.append((xx, yy, r))
    else:
        raise ValueError(mode)
    out.update(color=color, depth=depth, alpha=alpha, T_final=T_final, last=last,
               n_eval=n_eval, ambiguous=amb, pieces=tiles_kept)
    return out


def _scatter(r, xx, yy, color, depth, alpha, T_final, last, n_eval, amb):
    color[:, yy, xx] = r["color"].T
    depth[yy, xx] = r["depth"]
    alpha[yy, xx] = r["alpha"]
    T_final[yy, xx] = r["T_final"]
    last[yy, xx] = r["last"]
    n_eval[yy, xx] = r["n_eval"]
    amb[yy, xx] = r["ambiguous"]


def render_pixels(scene, views, k, pix_x, pix_y, st: Settings = Settings()):
    """Brute-force render of selected pixels of view k (for sampled checks
    at sizes where a whole-image oracle render is too slow)."""
    su = setup_view(scene, views, k, st)
    vis = su["vis"]
    order = np.lexsort((vis, su["kp"]["zbits"][vis]))
    px = np.asarray(pix_x) + 0.5
    py = np.asarray(pix_y) + 0.5
    outs = []
    for i in range(0, px.shape[0], 64):
        outs.append(composite(px[i:i + 64], py[i:i + 64], su["rec"], order,
                              np.asarray(st.bg, float)))
    cat = {key: np.concatenate([o[key] for o in outs]) for key in outs[0]}
    return cat


def splat_grads(r, gC, gD, gA):
    """Screen-space splat gradients from one composited piece.

    r is the keep=True output of composite() for P pixels; gC [P,3], gD [P],
    gA [P] are dL/dcolour, dL/ddepth, dL/dalpha at those pixels.  Returns
    per-entry arrays (over r['order']) of dL/d(u, v, A, B, C, sigma, colour,
    z).  Uses the stored forward transmittance T_before (no division)."""
    w = r["w"]
    if w.shape[1] == 0:
        z0 = np.zeros(0)
        return dict(u=z0, v=z0, A=z0, B=z0, C=z0, sigma=z0, color=np.zeros((0, 3)), z=z0)
    bl = r["blended"]
    a, Tb, col, z = r["alpha_e"], r["T_before"], r["col"], r["z"]
    Tf = r["T_final"]
    bg_term = r["color"] - np.stack([np.cumsum(w * col[None, :, c], 1)[:, -1]
                                     for c in range(3)], 1)  # T_final*bg
    wc = w[:, :, None] * col[None, :, :]
    cumc = np.cumsum(wc, axis=1)
    SC = cumc[:, -1:, :] - cumc + bg_term[:, None, :]
    wz = w * z[None, :]
    cumz = np.cumsum(wz, axis=1)
    SD = cumz[:, -1:] - cumz
    one_m = 1.0 - a
    dLda = np.einsum("pc,plc->pl", gC, col[None, :, :] * Tb[:, :, None]
                     - SC / one_m[:, :, None])
    dLda += gD[:, None] * (z[None, :] * Tb - SD / one_m)
    dLda += gA[:, None] * Tf[:, None] / one_m
    dLda = np.where(bl, dLda, 0.0)
    free = bl & ~r["clamped"]
    g_sig = np.where(free, r["G"] * dLda, 0.0)
    g_pow = np.where(free, a * dLda, 0.0)
    dx, dy = r["dx"], r["dy"]
    A, B, C = r["A"][None, :], r["B"][None, :], r["C"][None, :]
    return dict(u=np.sum(g_pow * -(A * dx + B * dy), 0),
                v=np.sum(g_pow * -(B * dx + C * dy), 0),
                A=np.sum(g_pow * (-0.5 * dx * dx), 0),
                B=np.sum(g_pow * (-dx * dy), 0),
                C=np.sum(g_pow * (-0.5 * dy * dy), 0),
                sigma=g_sig.sum(0),
                color=np.einsum("pl,pc->lc", w, gC),
                z=np.sum(w * gD[:, None], 0))


def render_backward(scene, views, grad_color, grad_depth, grad_alpha,
                    st: Settings = Settings(), view_ids=None):
    """Exact FP64 gradient of sum(grad_color*color + grad_depth*depth +
    grad_alpha*alpha) over the given views.  grad_* are [V,...] arrays (any
    may be None).  Returns dict of parameter gradients (scene-sized) and
    d_pose [V,6]."""
    N = scene.n
    out = dict(d_means=np.zeros((N, 3)), d_log_scales=np.zeros((N, 3)),
               d_quats=np.zeros((N, 4)), d_opacity=np.zeros(N),
               d_colors=np.zeros(scene.colors.shape), d_pose=np.zeros((views.n, 6)))
    W, H = views.width, views.height
    view_ids = range(views.n) if view_ids is None else view_ids
    for k in view_ids:
        gC = np.zeros((3, H, W)) if grad_color is None else np.asarray(grad_color[k], float)
        gD = np.zeros((H, W)) if grad_depth is None else np.asarray(grad_depth[k], float)
        gA = np.zeros((H, W)) if grad_alpha is None else np.asarray(grad_alpha[k], float)
        # tiles whose pixels all have zero upstream gradient contribute nothing
        live = np.abs(gC).sum(0) + np.abs(gD) + np.abs(gA) > 0
        TX, TY = -(-W // st.tile_w), -(-H // st.tile_h)
        tiles = [t for t in range(TX * TY)
                 if live[(t // TX) * st.tile_h:(t // TX + 1) * st.tile_h,
                         (t % TX) * st.tile_w:(t % TX + 1) * st.tile_w].any()]
        rv = render_view(scene, views, k, st, mode="tiled", keep=True, tiles=tiles)
        su = rv["setup"]
        nv = su["vis"].shape[0]
        acc = dict(u=np.zeros(nv), v=np.zeros(nv), A=np.zeros(nv), B=np.zeros(nv),
                   C=np.zeros(nv), sigma=np.zeros(nv), color=np.zeros((nv, 3)),
                   z=np.zeros(nv))
        for xx, yy, r in rv["pieces"]:
            g = splat_grads(r, gC[:, yy, xx].T, gD[yy, xx], gA[yy, xx])
            for key in acc:
                np.add.at(acc[key], r["order"], g[key])
        if nv == 0:
            continue
        conic_g = np.stack([acc["A"], acc["B"], acc["C"]], 1)
        sl = su["g0"] + su["vis"]
        pb = project_backward(su["pr"], acc["u"], acc["v"], conic_g, acc["sigma"],
                              acc["color"], acc["z"], scene.colors[sl], scene.sh_degree)
        np.add.at(out["d_means"], sl, pb["d_means"])
        np.add.at(out["d_log_scales"], sl, pb["d_log_scales"])
        np.add.at(out["d_quats"], sl, pb["d_quats"])
        np.add.at(out["d_opacity"], sl, pb["d_opacity"])
        np.add.at(out["d_colors"], sl, pb["d_colors"])
        out["d_pose"][k] = pb["d_pose"]
    return out
