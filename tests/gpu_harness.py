"""Helpers for the GPU parity tests: run the HIP path through the C ABI on
synthetic scenes and bring its outputs back as numpy."""
from __future__ import annotations

import sys

import numpy as np


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


def make_rasterizer(scene, views, tile=(16, 16), max_instances=None, chunk=0):
    from paper_2605_10760_amd import Rasterizer
    so = scene.set_offsets
    P = int(sum(so[s + 1] - so[s] for s in views.view_set))
    return Rasterizer(views.width, views.height, max(P, 1), views.n,
                      max_instances=max_instances, tile=tile, chunk=chunk), P


def gpu_forward(scene, views, tile=(16, 16), z_near=0.2, bg=(0.0, 0.0, 0.0), export=True,
                rast=None, chunk=0):
    """Forward on the GPU; returns dict of numpy outputs (+ binning export)."""
    import torch
    st_, vt = to_gpu(scene, views)
    if rast is None:
        rast, P = make_rasterizer(scene, views, tile, chunk=chunk)
    else:
        P = int(sum(scene.set_offsets[s + 1] - scene.set_offsets[s] for s in views.view_set))
    c, d, a, state, ne = rast.forward(st_, vt, z_near=z_near, bg=bg, n_eval=True)
    counts = rast.poll(state)
    out = dict(color=c.cpu().numpy(), depth=d.cpu().numpy(), alpha=a.cpu().numpy(),
               n_eval=ne.cpu().numpy(), counts=counts, state=state, rast=rast, scene_t=st_,
               views_t=vt, P=P)
    if export:
        out["dbg"] = rast.debug_export(state, views.n, P, int(counts["instances"]))
    torch.cuda.synchronize()
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
