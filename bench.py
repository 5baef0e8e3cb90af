#!/usr/bin/env python
"""Throughput of the differentiable Gaussian-splatting rasterizer on one GPU.

Default workload: agents' submaps of uneven sizes (50k, 120k, 200k, 300k,
400k, 600k Gaussians) x 8 keyframes each at 640x480, one fwd+bwd
optimisation step per iteration: forward render of all 48 views, the L1
colour + depth loss gradient of the mapping loss (weights 0.95 / 0.25,
Sec. III-A Eq. (map_loss)), the backward to every Gaussian parameter and
every keyframe pose, and an Adam update.

  batched : all sets x views in one launch sequence, captured once as a
            HIP graph (torch.cuda.CUDAGraph) and replayed
  plain   : a per-view loop, each view with its own projection, sort and
            backward, run eagerly

Prints ONE JSON line.  `value` is batched fwd+bwd views/s; the line also
carries Gaussian-pixel evaluations/s, the plain loop's rates, per-stage
times, the roofline of the dominant kernel and the CPU oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3        # packed / dual-issue FP32
FP32_NONPACKED_PEAK_TFLOPS = 78.6      # one FMA per lane per cycle
# VALU instruction issue of the whole chip at one wave64 instruction per SIMD
# per 4 cycles: 256 CUs x 4 SIMDs x 2.4 GHz / 4
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4

# Floating-point operations per unit of compositing work, counted from the
# definition (one per +, -, *, /, min, compare, exp).
# Forward, per list entry examined by a pixel: offsets (2), the quadratic
# form -(A dx^2 + C dy^2)/2 - B dx dy (9), exp (1), sigma G (1), clamp (1),
# the two skip tests (2), T (1 - alpha) (2), the stop test (1).
OPS_FWD_EXAMINED = 19
# Forward, per blended entry: weight alpha T (1), colour and depth
# accumulation (8).
OPS_FWD_BLENDED = 9
# Backward, per entry walked back from the pixel's last contributor: alpha
# recomputed up to the skip tests (16), T_j = T_(j+1) / (1 - alpha) (2).
OPS_BWD_WALKED = 18
# Backward, per blended entry: c . dL/dC + z dL/dD (7), dL/dalpha (3), the
# running sum with its weight (3), colour and depth gradients (8), sigma
# gradient (2), dL/dpower (1), conic gradients (9), mean gradients (10).
OPS_BWD_BLENDED = 43

WORKLOADS = ("multi-agent", "room", "room-1m", "fused", "small")
LR_SCALE = 1e-3

# kernel that makes up each library stage (stages of one kernel only)
STAGE_KERNEL = {"project": "k_project", "render_fwd": "k_render_fwd",
                "render_bwd": "k_render_bwd_w", "project_bwd": "k_project_bwd"}


def _code_only(text):
    """C/C++ source without its comments and whitespace (string and character
    literals kept as they are), so that editing a comment keeps the digest."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_digest():
    """SHA-256 over the code of the library's kernel sources and the ABI
    header (comments and whitespace left out): a recorded counter figure
    holds only for the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for d in (os.path.join(ROOT, "paper_2605_10760_amd", "csrc"), os.path.join(ROOT, "include")):
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".h")):
                h.update(f.encode())
                with open(os.path.join(d, f), encoding="utf-8") as fh:
                    h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def recorded(tag, kernel, workload, tile):
    """A record from a committed rocprofv3 counter summary under profiles/
    (a line `<tag>-json: {...}`) for this kernel, workload, tile shape and
    source digest, or None.  Tags: `traffic` (FETCH_SIZE and WRITE_SIZE per
    dispatch, each scaled by what the counter reads for a plain copy of known
    size) and `valu` (VALU instructions, busy and dual-issue quad-cycles)."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    want = source_digest()
    for f in sorted(os.listdir(d)):
        if not f.endswith((".txt", ".md")):
            continue
        with open(os.path.join(d, f)) as fh:
            for ln in fh:
                if not ln.startswith(f"{tag}-json:"):
                    continue
                try:
                    r = json.loads(ln.split(":", 1)[1])
                except ValueError:
                    continue
                if (r.get("kernel") == kernel and r.get("workload") == workload
                        and r.get("tile") == tile and r.get("source_digest") == want):
                    return r
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=WORKLOADS, default="multi-agent")
    ap.add_argument("--tile", default="16x16", help="tile shape when not autotuning")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip gsr_autotune and use --tile with the default compositing options")
    ap.add_argument("--persistent", type=int, choices=(0, 1), default=None,
                    help="force the persistent tile queue off/on (after autotuning)")
    ap.add_argument("--bwd-cols", type=int, choices=(1, 2), default=None,
                    help="force the tiles per backward wave (after autotuning)")
    ap.add_argument("--no-graph", action="store_true", help="time the batched step eagerly")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the kernels beyond the rasterizer step (profiling runs)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads (small, room, room-1m autograd, fused map)")
    ap.add_argument("--config-steps", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle budget per run (one core, then every core)")
    ap.add_argument("--digest", action="store_true",
                    help="print the kernel-source digest that counter records are keyed on")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counters)")
    return ap.parse_args()


def make_workload(name):
    from synth import scenes
    if name == "multi-agent":
        return scenes.multi_agent()
    if name == "room":
        return scenes.room_plain()
    if name == "room-1m":
        return scenes.room_plain(seed=20, n=1_000_000)
    if name == "fused":
        # 16 forward-only novel views + 32 fwd+bwd keyframes in one batch
        return scenes.fused_map()
    return scenes.small_plain(0)


def plan_options(tuned):
    """Rasterizer keyword arguments of an autotune result (or defaults)."""
    if tuned is None:
        return dict(chunk=0, fwd_batch=1, bwd_batch=1, persistent=False, bwd_cols=1)
    return dict(chunk=tuned["chunk"], fwd_batch=tuned["fwd_batch"],
                bwd_batch=tuned["bwd_batch"], persistent=tuned["persistent"],
                bwd_cols=tuned["bwd_cols"])


class Step:
    """One optimisation step on preallocated buffers (capture-safe)."""

    def __init__(self, torch, rast, sc, vw, tc, td, lr_scale=1.0):
        self.t = torch
        self.rast, self.sc, self.vw, self.tc, self.td = rast, sc, vw, tc, td
        V, H, W = vw.n, vw.height, vw.width
        dev = sc.means.device
        self.state = rast.new_state()
        self.out = (torch.empty((V, 3, H, W), device=dev), torch.empty((V, H, W), device=dev),
                    torch.empty((V, H, W), device=dev))
        self.gc = torch.empty((V, 3, H, W), device=dev)
        self.gd = torch.empty((V, H, W), device=dev)
        self.lg = dict(d_color=self.gc, d_depth=self.gd, d_exposure=None)
        from paper_2605_10760_amd import l1_loss_grad
        self.l1 = l1_loss_grad
        params = [sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.colors]
        self.grads = dict(d_means=torch.zeros_like(sc.means), d_log_scales=torch.zeros_like(sc.log_scales),
                          d_quats=torch.zeros_like(sc.quats),
                          d_opacity_logits=torch.zeros_like(sc.opacity_logits),
                          d_colors=torch.zeros_like(sc.colors),
                          d_pose=torch.zeros((V, 6), device=dev))
        for p, k in zip(params, ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors")):
            p.grad = self.grads[k]
        lrs = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3)
        # the library's Adam: one launch over the five parameter arrays
        # (graph-capturable, device step count)
        from paper_2605_10760_amd import Adam
        self.opt = Adam([(p, lr * lr_scale) for p, lr in zip(params, lrs)], eps=1e-15)

    def __call__(self):
        t = self.t
        c, d, a, _ = self.rast.forward(self.sc, self.vw, state=self.state, out=self.out)
        # L1 mapping loss gradient (Eq. (map_loss) weights), one fused pass
        self.l1(c, self.tc, d, self.td, None, 0.95, 0.25, out=self.lg)
        self.rast.backward(self.sc, self.vw, self.state, self.gc, self.gd, None, out=self.grads)
        self.opt.step()


_CPU = {}


def _cpu_tiles(tiles):
    """Compositing forward + backward of some tiles of the CPU baseline's
    keyframe (a worker of the all-core run; the keyframe's set-up is
    inherited from the parent process)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.composite import composite, pixel_grid
    from oracle.render import splat_grads
    su, vals, rng_t, TX, W, H = (_CPU[k] for k in ("su", "vals", "rng_t", "TX", "W", "H"))
    nv = su["vis"].shape[0]
    acc = {key: np.zeros(nv) for key in ("u", "v", "A", "B", "C", "sigma", "z")}
    acc["color"] = np.zeros((nv, 3))
    if len(tiles) == 0:
        return acc
    rng = np.random.default_rng(int(tiles[0]))
    with threadpool_limits(limits=1):
        for t in tiles:
            ty, tx = divmod(int(t), TX)
            xx, yy, sx, sy = pixel_grid(tx * 16, ty * 16, min(tx * 16 + 16, W), min(ty * 16 + 16, H))
            lo, hi = rng_t[t]
            lst = su["local"][vals[lo:hi] - su["g0"]]
            r = composite(sx, sy, su["rec"], lst, np.zeros(3), keep=True)
            g = splat_grads(r, rng.normal(size=(sx.shape[0], 3)), rng.normal(size=sx.shape[0]),
                            np.zeros(sx.shape[0]))
            for key in acc:
                np.add.at(acc[key], r["order"], g[key])
    return acc


def time_cpu_baseline(wl, seconds):
    """The CPU oracle (FP64 NumPy) on a bounded sample of the same workload:
    one keyframe of the largest submap with its full projection, binning,
    sort and projection backward, and compositing forward+backward on an
    evenly spread sample of its tiles, extrapolated to all tiles.  Timed on
    one core, then with the compositing spread over every host core (a
    process pool over tiles; set-up and projection backward stay on one
    core)."""
    import multiprocessing as mp
    import platform

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle.project64 import project_backward
    from oracle.render import Settings, bin_view, setup_view
    sc, vw = wl.scene, wl.views
    sizes = np.diff(sc.set_offsets)
    k = int(np.nonzero(vw.view_set == int(np.argmax(sizes)))[0][0])
    one = vw.select([k])
    H, W = one.height, one.width
    st = Settings()
    TX, TY = -(-W // 16), -(-H // 16)
    order = np.argsort((np.arange(TX * TY) * 0.6180339887) % 1.0)
    t_start = time.perf_counter()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        su = setup_view(sc, one, 0, st)
        keys, vals, rng_t = bin_view(su, 0, st, W, H)
        t_setup = time.perf_counter() - t0
    _CPU.update(su=su, vals=vals, rng_t=rng_t, TX=TX, W=W, H=H)
    _cpu_tiles(order[:0])  # imports outside the timed region
    # one core: tiles one by one until the budget is spent
    budget = max(2.0, seconds - 1.5 * t_setup)
    n_done, t_tiles, acc = 0, 0.0, None
    while n_done < TX * TY and t_tiles < budget:
        t1 = time.perf_counter()
        a = _cpu_tiles(order[n_done:n_done + 4])
        t_tiles += time.perf_counter() - t1
        n_done += len(order[n_done:n_done + 4])
        acc = a if acc is None else {key: acc[key] + a[key] for key in acc}
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sl = su["g0"] + su["vis"]
        project_backward(su["pr"], acc["u"], acc["v"], np.stack([acc["A"], acc["B"], acc["C"]], 1),
                         acc["sigma"], acc["color"], acc["z"], sc.colors[sl], sc.sh_degree)
        t_pb = time.perf_counter() - t0
    per_view_1 = t_setup + t_pb + t_tiles / n_done * TX * TY
    # every core: the same per-tile work over a process pool
    # worker processes: the host cores, at most 16 (the CPU share of one GPU)
    ncpu = max(1, min(16, os.cpu_count() or 1))
    n_all = min(TX * TY, max(n_done, 1) * ncpu)
    chunks = [order[i:n_all:ncpu * 4] for i in range(0, ncpu * 4)]
    chunks = [c for c in chunks if len(c)]
    ctx = mp.get_context("fork")
    with ctx.Pool(ncpu) as pool:
        t1 = time.perf_counter()
        parts = pool.map(_cpu_tiles, chunks)
        t_pool = time.perf_counter() - t1
    del parts
    per_view_n = t_setup + t_pb + t_pool / n_all * TX * TY
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        model = platform.processor()
    desc = (f"one {W}x{H} keyframe of the {int(sizes.max())}-Gaussian submap: projection, "
            f"binning, sort and projection backward in full, compositing fwd+bwd on a sample "
            f"of its {TX * TY} tiles extrapolated to the whole view; FP64 NumPy")
    return dict(value=round(1.0 / per_view_1, 6), unit="views/s", cores=1, kind="oracle",
                sample=f"{desc}; {n_done} tiles on 1 core",
                all_cores=dict(value=round(1.0 / per_view_n, 6), unit="views/s", cores=ncpu,
                               sample=f"{n_all} tiles over a pool of {ncpu} processes "
                                      f"(set-up and projection backward on one core)"),
                cpu_model=model, host_cpus=ncpu,
                seconds=round(time.perf_counter() - t_start, 1))


def work_counts(np, rast, sc, vw, V, H, W, tile):
    """Measured work of one untimed forward: pairs, instances, entries
    examined (forward) and walked (backward) per pixel, blended entries, and
    the per-tile maxima that bound the compositing list reads."""
    c, d, a, state, ne = rast.forward(sc, vw, n_eval=True)
    counts = rast.poll(state)
    P = int(sum(int(sc.set_offsets[s + 1] - sc.set_offsets[s]) for s in vw.view_set))
    dbg = rast.debug_export(state, V, P, 0, n_blend=True)
    n_eval = ne.cpu().numpy().astype(np.int64)
    last = dbg["last"].astype(np.int64)
    TX, TY = dbg["TX"], dbg["TY"]

    def tile_max(x):
        pad = np.zeros((V, TY * tile[1], TX * tile[0]), np.int64)
        pad[:, :H, :W] = x
        return pad.reshape(V, TY, tile[1], TX, tile[0]).max(axis=(2, 4))

    out = dict(pairs=P, visible_pairs=int(counts["visible_pairs"]),
               instances=int(counts["instances"]), row_entries=int(counts["row_entries"]),
               examined=int(n_eval.sum()),
               walked=int(last.sum()), blended=int(dbg["n_blend"].astype(np.int64).sum()),
               E_fwd=int(tile_max(n_eval).sum()), E_bwd=int(tile_max(last).sum()))
    del state, c, d, a, ne
    return out


def algorithmic(cnt, sc_np, V, H, W, sh_stride, fwd_only_views=0):
    """Algorithmic bytes per stage (the minimum each stage must move, from
    the measured counts) and operations of the compositing kernels."""
    P, Pv = cnt["pairs"], cnt["visible_pairs"]
    rgb = sc_np.sh_degree == 0
    par = 56 if rgb else 4 * (3 + 3 + 4 + 1 + 3 * sh_stride)
    npx = V * H * W
    byt = {
        # key pass: the key path's parameters (means, log-scales, quaternion,
        # opacity: 44 B) once per Gaussian, a depth key per pair
        "project": 44 * sc_np.n + 4 * P,
        # read the keys, write each pair's visible position and each visible
        # pair's key
        "compact": 4 * P + 4 * P + 4 * Pv,
        # record pass: every parameter once per Gaussian, the visible position
        # per pair, rect + record per visible pair
        "record": par * sc_np.n + 4 * P + (48 + 8) * Pv,
        # four 8-bit passes over the visible keys: the histogram reads the
        # keys, the scatter reads keys (and values, from the second pass on)
        # and writes values (and keys, except in the last pass)
        "depth_sort": (4 + 4 + 8) * Pv + 2 * (4 + 8 + 8) * Pv + (4 + 8 + 4) * Pv,
        # rects and depth order read by the counting and scatter passes, the
        # (pair, tile row) entries written; the tile lists are filtered from
        # them by the compositing kernels
        "binning": 2 * 12 * Pv + 8 * cnt["row_entries"],
        "render_fwd": 52 * cnt["E_fwd"] + 28 * npx,
        "render_bwd": 52 * cnt["E_bwd"] + 80 * cnt["E_bwd"] + 28 * npx,
        # parameters read and gradients written once per Gaussian, the visible
        # position per pair, each visible pair's gradient row read and cleared
        "project_bwd": 2 * par * sc_np.n + 4 * P + 80 * Pv,
    }
    ops = {
        "render_fwd": OPS_FWD_EXAMINED * cnt["examined"] + OPS_FWD_BLENDED * cnt["blended"],
        "render_bwd": OPS_BWD_WALKED * cnt["walked"] + OPS_BWD_BLENDED * cnt["blended"],
    }
    return byt, ops


def time_steps(torch, run, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def run_plain(torch, np, wl, sc, vw, tc, td, step, tile, opts, steps):
    """The per-view loop: each view with its own projection, sort,
    compositing and backward, eagerly; gradients summed, then Adam."""
    from paper_2605_10760_amd import Rasterizer, l1_loss_grad
    sc_np, vw_np = wl.scene, wl.views
    V, H, W = vw_np.n, vw_np.height, vw_np.width
    so = sc_np.set_offsets
    per_view = [vw.select([k]) for k in range(V)]
    max_set = int(max(so[s_ + 1] - so[s_] for s_ in vw_np.view_set))
    r1 = Rasterizer(W, H, max_set, 1, tile=tile, max_instances=1 << 20, **opts)
    for k in range(V):
        r1.fit_capacity(sc, per_view[k])
    st1 = r1.new_state()
    o1 = (torch.empty((1, 3, H, W), device="cuda"), torch.empty((1, H, W), device="cuda"),
          torch.empty((1, H, W), device="cuda"))
    g1 = {k_: torch.empty_like(v_) for k_, v_ in step.grads.items()}
    g1["d_pose"] = torch.empty((1, 6), device="cuda")
    gcv = torch.empty((1, 3, H, W), device="cuda")
    gdv = torch.empty((1, H, W), device="cuda")
    lgv = dict(d_color=gcv, d_depth=gdv, d_exposure=None)
    tot = step.grads

    def plain_step():
        for g_ in tot.values():
            g_.zero_()
        for k in range(V):
            c1, d1, _, _ = r1.forward(sc, per_view[k], state=st1, out=o1)
            if vw_np.needs_grad is not None and not vw_np.needs_grad[k]:
                continue
            # the batch's loss is a mean over all V views: scale by 1/V
            l1_loss_grad(c1, tc[k:k + 1], d1, td[k:k + 1], None, 0.95 / V, 0.25 / V, out=lgv)
            r1.backward(sc, per_view[k], st1, gcv, gdv, None, out=g1)
            for key in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_colors"):
                tot[key].add_(g1[key])
            tot["d_pose"][k].copy_(g1["d_pose"][0])
        step.opt.step()

    plain_step()
    return time_steps(torch, plain_step, steps)


def run_workload(torch, np, wl, args, steps, warmup, tuned=None, tile=(16, 16), stages=True,
                 plain_steps=2, ab_steps=0):
    """Batched step (graph replay) and plain loop on one workload: rates,
    measured work, per-stage times and algorithmic bytes/ops."""
    from paper_2605_10760_amd import Rasterizer, SceneTensors, ViewTensors
    sc_np, vw_np = wl.scene, wl.views
    V, H, W = vw_np.n, vw_np.height, vw_np.width
    sc = SceneTensors.from_numpy(sc_np)
    vw = ViewTensors.from_numpy(vw_np)
    tc = torch.from_numpy(wl.target_color).cuda()
    td = torch.from_numpy(wl.target_depth if wl.target_depth is not None
                          else np.zeros((V, H, W), np.float32)).cuda()
    so = sc_np.set_offsets
    P = int(sum(so[s + 1] - so[s] for s in vw_np.view_set))
    if tuned is not None:
        tile = tuned["tile"]
    opts = plan_options(tuned)
    if args.persistent is not None:
        opts["persistent"] = bool(args.persistent)
    if getattr(args, "bwd_cols", None) is not None:
        opts["bwd_cols"] = int(args.bwd_cols)
    rast = Rasterizer(W, H, P, V, tile=tile, **opts)
    rast.fit_capacity(sc, vw)
    cnt = work_counts(np, rast, sc, vw, V, H, W, tile)

    # The Adam update runs in full every step, with the learning rates
    # scaled by LR_SCALE: against random targets the full rates move every
    # opacity logit by ~0.05 per step, so the scene (and the work per step)
    # would drift away from the one the counts were taken on.
    step = Step(torch, rast, sc, vw, tc, td, lr_scale=LR_SCALE)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(1, warmup)):
            step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(2):
            graph.replay()
    dt = time_steps(torch, graph.replay if graph is not None else step, steps)
    post = rast.poll(step.state, raise_on_overflow=False)
    if post["overflow"]:
        raise RuntimeError(f"{wl.name}: instance capacity overflow during the timed steps")

    stage_acc = {}
    if stages:
        # per-stage times: eager steps with HIP events on the launching stream
        rast.profile(True)
        n_prof = max(3, min(steps, 10))
        for _ in range(n_prof):
            step()
            for k_, v_ in rast.stage_ms().items():
                stage_acc[k_] = stage_acc.get(k_, 0.0) + v_ / n_prof
        rast.profile(False)
        torch.cuda.synchronize()

    ab = None
    if ab_steps:
        # A/B of the compositing options on this workload: eager steps with
        # one option changed from the plan in use (same state buffer)
        base = dict(fwd_batch=rast.desc.fwd_batch or 1, bwd_batch=rast.desc.bwd_batch or 1,
                    persistent=rast.desc.persistent, bwd_cols=rast.desc.bwd_cols or 1)
        variants = [("plan", {})]
        variants.append(("persistent" if not base["persistent"] else "grid",
                         dict(persistent=1 - base["persistent"])))
        variants.append((f"fwd_batch={3 - base['fwd_batch']}", dict(fwd_batch=3 - base["fwd_batch"])))
        for bb in (1, 2, 4):
            if bb != base["bwd_batch"]:
                variants.append((f"bwd_batch={bb}", dict(bwd_batch=bb)))
        if rast.desc.tile_w <= 16 and 2 * rast.desc.tile_w * rast.desc.tile_h <= 512:
            variants.append((f"bwd_cols={3 - base['bwd_cols']}",
                             dict(bwd_cols=3 - base["bwd_cols"])))
        ab = {}
        for name, change in variants:
            rast.replan(**{**base, **change})
            step()
            ab[name] = round(time_steps(torch, step, ab_steps) * 1e3, 4)
        rast.replan(**base)
        torch.cuda.synchronize()

    n_bwd = int(np.sum(vw_np.needs_grad)) if vw_np.needs_grad is not None else V
    plain = None
    if plain_steps:
        pdt = run_plain(torch, np, wl, sc, vw, tc, td, step, tile, opts, plain_steps)
        plain = dict(views_per_s=round(n_bwd / pdt, 2),
                     evals_per_s=round((cnt["examined"] + cnt["walked"]) / pdt, 1),
                     ms_per_step=round(pdt * 1e3, 3), steps=plain_steps)
    byt, ops = algorithmic(cnt, sc_np, V, H, W, sc.sh_stride)
    res = dict(name=wl.name, V=V, H=H, W=W, n_bwd=n_bwd, dt=dt, cnt=cnt, bytes=byt, ops=ops,
               stage_ms=stage_acc, plain=plain, tile=tile, opts=opts, rast=rast, step=step, ab=ab,
               sc=sc, vw=vw, tc=tc, td=td, graph=graph is not None,
               step_bytes=sum(byt.values()))
    return res


def summary(res):
    """Compact record of a workload's batched rate, plain rate and work."""
    dt, cnt = res["dt"], res["cnt"]
    return dict(workload=res["name"], fwd_bwd_views=res["n_bwd"], views=res["V"],
                views_per_s=round(res["n_bwd"] / dt, 2), ms_per_step=round(dt * 1e3, 4),
                evals_per_s=round((cnt["examined"] + cnt["walked"]) / dt, 1),
                evals={"forward": cnt["examined"], "backward": cnt["walked"],
                       "blended": cnt["blended"]},
                counts={k: cnt[k] for k in ("pairs", "visible_pairs", "instances", "row_entries")},
                step_algorithmic_GB=round(res["step_bytes"] / 1e9, 3),
                step_hbm_roofline_frac=round(res["step_bytes"] / (dt * HBM_PEAK_GBS * 1e9), 4),
                tile=f"{res['tile'][0]}x{res['tile'][1]}", options=res["opts"],
                option_ab_ms_per_step=res.get("ab"),
                form="batched, hip graph replay" if res["graph"] else "batched, eager",
                plain=res["plain"])


def run_autograd(torch, np, wl, steps, warmup):
    """The autograd form: rasterize() as a torch.autograd.Function with a
    pose delta, the mapping loss in torch, loss.backward(), Adam (eager)."""
    from paper_2605_10760_amd import Rasterizer, rasterize
    sc_np, vw_np = wl.scene, wl.views
    V, H, W = vw_np.n, vw_np.height, vw_np.width
    P = int(sum(sc_np.set_offsets[s + 1] - sc_np.set_offsets[s] for s in vw_np.view_set))
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda().requires_grad_(True)
    params = [f(sc_np.means), f(sc_np.log_scales), f(sc_np.quats), f(sc_np.opacity_logits),
              f(sc_np.colors)]
    pose = torch.zeros((V, 6), device="cuda", requires_grad=True)
    vm = torch.from_numpy(vw_np.viewmats).cuda()
    intr = torch.from_numpy(vw_np.intrinsics).cuda()
    tc = torch.from_numpy(wl.target_color).cuda()
    td = torch.from_numpy(wl.target_depth).cuda()
    rast = Rasterizer(W, H, P, V)
    lrs = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1e-3)
    from paper_2605_10760_amd import Adam
    opt = Adam([(p, lr * LR_SCALE) for p, lr in zip(params + [pose], lrs)], eps=1e-15)

    def one():
        for p in params + [pose]:
            if p.grad is not None:
                p.grad.zero_()
        c, d, _ = rasterize(rast, *params, vm, intr, sc_np.set_offsets, vw_np.view_set, W, H,
                            pose_delta=pose, sh_degree=int(sc_np.sh_degree))
        loss = 0.95 * (c - tc).abs().mean() + 0.25 * (d - td).abs().mean()
        loss.backward()
        opt.step()

    for _ in range(max(1, warmup)):
        one()
    dt = time_steps(torch, one, steps)
    return dict(workload=wl.name + "-autograd", views=V, fwd_bwd_views=V,
                views_per_s=round(V / dt, 2), ms_per_step=round(dt * 1e3, 4),
                form="torch.autograd.Function, eager, with pose delta")


def measure_extras(torch, sc, vw, out_color, out_depth, tc, td, rast=None, reps=10):
    """HBM-bound kernels beyond the rasterizer (Sim(3) correction, pose lift,
    refinement loss gradients, pruning) on the same batch: average time per
    call from torch events on the stream they launch on, algorithmic bytes,
    and the fraction of the 8 TB/s HBM peak."""
    import numpy as np
    from paper_2605_10760_amd import (iso_grad, l1_loss_grad, normal_loss_grad, prune, seed,
                                      sim3_gaussians, sim3_views, ssim_grad)
    V, _, H, W = out_color.shape
    N = sc.n
    rng = np.random.default_rng(0)
    sims = []
    for _ in range(len(sc.set_offsets) - 1):
        q = rng.normal(size=4)
        sims.append(np.concatenate([[1.1], q / np.linalg.norm(q), rng.normal(0, 0.1, 3)]))
    sims = torch.from_numpy(np.array(sims, np.float32)).cuda()
    expo = torch.zeros((V, 2), device="cuda")
    gs = (torch.empty_like(sc.means), torch.empty_like(sc.log_scales), torch.empty_like(sc.quats))
    vmo = torch.empty_like(vw.viewmats)
    gl = dict(d_color=torch.empty_like(out_color), d_depth=torch.empty_like(out_depth),
              d_exposure=torch.empty((V, 2), device="cuda"))
    ws = ssim_grad(out_color, tc, gl["d_color"], expo, gl["d_exposure"])
    px = V * H * W
    prior = torch.zeros_like(out_color)
    prior[:, 2] = -1.0
    g_ls = torch.zeros_like(sc.log_scales)
    calls = {
        # 40 B read + 40 B written per Gaussian
        "sim3_gaussians": (lambda: sim3_gaussians(sc.means, sc.log_scales, sc.quats,
                                                  sc.set_offsets, sims, out=gs), 80 * N),
        "sim3_views": (lambda: sim3_views(vw.viewmats, sims, vw.view_set, out=vmo), 96 * V),
        # colour: read I^, I, write dI^ (3 channels); depth: read 2, write 1
        "l1_loss_grad": (lambda: l1_loss_grad(out_color, tc, out_depth, td, expo, 1.75, 0.25,
                                              out=gl), 48 * px),
        # per pixel and channel: read I^ and I, read-modify-write dI^
        "ssim_grad": (lambda: ssim_grad(out_color, tc, gl["d_color"], expo, gl["d_exposure"],
                                        workspace=ws), 16 * 3 * px),
        # read the log-scales, read-modify-write their gradient
        "iso_grad": (lambda: iso_grad(sc.log_scales, g_ls, 10.0), 36 * N),
        # read depth and the 3-channel prior, read-modify-write dD
        "normal_loss_grad": (lambda: normal_loss_grad(out_depth, prior, vw.intrinsics,
                                                      gl["d_depth"], 1e-2), 24 * px),
    }
    res = {}
    for name, (fn, nbytes) in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = dict(ms=round(ms, 4), algorithmic_GBps=round(gbs, 1),
                         hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
    # deduplication: the target is the largest submap's Gaussians in the part
    # of the room with x < 0.5 m, with that submap's keyframe depths; the
    # borrowed set is the next largest submap (uniform in the room), so the
    # borrowed Gaussians beyond the target's coverage survive (synchronises)
    from paper_2605_10760_amd import dedup
    so = sc.set_offsets
    tgt, src = len(so) - 2, len(so) - 3
    kfs = [k for k in range(V) if vw.view_set[k] == tgt]
    ta, tb = int(so[tgt]), int(so[tgt + 1])
    sa, sb = int(so[src]), int(so[src + 1])
    part = sc.means[ta:tb, 0] < 0.5
    t_means = sc.means[ta:tb][part].contiguous()
    t_ls = sc.log_scales[ta:tb][part].contiguous()
    dep = out_depth[kfs].contiguous()
    vm_k, in_k = vw.viewmats[kfs].contiguous(), vw.intrinsics[kfs].contiguous()
    dedup(sc.means[sa:sb], t_means, t_ls, dep, vm_k, in_k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keep, nvox = dedup(sc.means[sa:sb], t_means, t_ls, dep, vm_k, in_k)
    ms = (time.perf_counter() - t0) * 1e3
    res["dedup"] = dict(ms=round(ms, 3), target=int(t_means.shape[0]), borrowed=sb - sa,
                        kept=int(keep.sum().item()), rays=len(kfs) * H * W, voxels=nvox,
                        note="voxel 0.05, k 1; target: the largest submap's Gaussians with "
                             "x < 0.5 m; includes the host synchronisation")
    # seeding one keyframe synchronises (host count): wall time of one call
    seed(out_depth[0], out_color[0], vw.viewmats[0], vw.intrinsics[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sd = seed(out_depth[0], out_color[0], vw.viewmats[0], vw.intrinsics[0])
    ms = (time.perf_counter() - t0) * 1e3
    res["seed"] = dict(ms=round(ms, 4), seeded=int(sd["means"].shape[0]), pixels=H * W,
                       note="one keyframe, stride 1; includes the host synchronisation")
    # pruning synchronises (host offsets): wall time of one call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = prune(sc, 0.005)
    ms = (time.perf_counter() - t0) * 1e3
    kept = pr.n
    row = 56 if sc.colors.dim() == 2 else 4 * (3 + 3 + 4 + 1 + 3 * sc.sh_stride)
    nbytes = 4 * N + 2 * row * kept
    res["prune"] = dict(ms=round(ms, 4), kept=kept, of=N,
                        algorithmic_GBps=round(nbytes / (ms * 1e-3) / 1e9, 1),
                        note="includes the host synchronisation for the pruned set offsets")
    if rast is not None:
        # one iteration of the joint refinement (Eq. (refine_loss)) of every
        # view: forward, L1 + SSIM + normal gradients on the exposure-
        # compensated render, backward, Adam over Gaussians, pose deltas and
        # exposure (eager; it moves the scene, so it runs last)
        from paper_2605_10760_amd import REFINE_WEIGHTS, Optimizer, Rates
        opt = Optimizer(rast, sc, vw, tc, td, prior, REFINE_WEIGHTS, Rates().scaled(0.5),
                        pose=True, exposure=True)
        opt.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            opt.step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res["refine_step"] = dict(ms=round(ms, 3), views=V, views_per_s=round(V / (ms * 1e-3), 1),
                                  note="eager, one refinement iteration of all views")
    return res


def tile_key(tile, opts):
    """Tile shape as the counter summaries record it: WxH, with -bwd2 when
    the backward takes two tiles of a tile row per wave."""
    return f"{tile[0]}x{tile[1]}" + ("-bwd2" if int(opts.get("bwd_cols", 1)) == 2 else "")


def roofline_of(res, kernel_stage, workload_name):
    """Roofline record of one compositing (VALU-bound) or HBM-bound stage:
    algorithmic rate over the measured average launch time, with the HBM
    traffic and VALU issue figures of the committed counter summaries when
    they were taken on these sources."""
    ms = res["stage_ms"].get(kernel_stage, 0.0)
    if ms <= 0:
        return None
    kern = STAGE_KERNEL.get(kernel_stage, kernel_stage)
    tile = tile_key(res["tile"], res["opts"])
    byt = res["bytes"].get(kernel_stage, 0)
    hbm = byt / (ms * 1e-3) / 1e9
    tr = recorded("traffic", kern, workload_name, tile)
    va = recorded("valu", kern, workload_name, tile)
    if kernel_stage in res["ops"]:
        ach = res["ops"][kernel_stage] / (ms * 1e-3) / 1e12
        r = dict(bound="alu", kernel=kern, achieved=round(ach, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                 unit="TFLOP/s", frac=round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                 frac_of_nonpacked=round(ach / FP32_NONPACKED_PEAK_TFLOPS, 4))
    else:
        r = dict(bound="hbm", kernel=kern, achieved=round(hbm, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                 frac=round(hbm / HBM_PEAK_GBS, 4))
    r["traffic"] = None if tr is None else int(tr["fetch_bytes"] + tr["write_bytes"])
    if tr is not None:
        r["traffic_unit"] = "bytes per launch"
    r["algorithmic_bytes"] = int(byt)
    r["hbm_algorithmic_GBps"] = round(hbm, 1)
    r["hbm_frac"] = round(hbm / HBM_PEAK_GBS, 4)
    if va is not None:
        # counter-based: VALU instructions over the issue capacity at one
        # wave64 instruction per SIMD per 4 cycles (2.4 GHz), and the share
        # of quad-cycles with a VALU instruction issued
        r["valu_issue_frac"] = round(va["valu_insts"] / (ms * 1e-3 * VALU_ISSUE_PEAK), 4)
        r["valu_busy_frac"] = va.get("valu_busy_frac")
        r["valu_dual_issue_frac"] = va.get("valu_dual_frac")
        r["clock_GHz"] = va.get("clock_GHz")
    r["ms"] = round(ms, 4)
    return r


def main():
    args = parse()
    if args.digest:
        print(source_digest())
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the rasterizer's multi-GPU form (views or "
              "submaps sharded over GPUs with an all-reduce of Gaussian gradients) is not "
              "built; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    wl = make_workload(args.workload)
    # the CPU oracle first: its process pool forks before anything touches the GPU
    cpu = None
    if not args.no_cpu:
        cpu = time_cpu_baseline(wl, args.cpu_seconds)
        print(f"[bench] cpu baseline: {cpu['value']:.4g} views/s on 1 core, "
              f"{cpu['all_cores']['value']:.4g} on {cpu['all_cores']['cores']}",
              file=sys.stderr, flush=True)

    import torch

    from paper_2605_10760_amd import SceneTensors, ViewTensors
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain elementwise copy kernel of known size: 1 GiB read + 1 GiB
        # written per launch (the reference for the HBM byte counters)
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
        # a gather of 48-byte rows in random order (the record reads of the
        # compositing kernels): 1 GiB gathered + 1 GiB written per launch
        rows = torch.empty((1 << 30) // 48, 12, dtype=torch.float32, device="cuda").fill_(1.0)
        perm = torch.randperm(rows.shape[0], device="cuda", dtype=torch.int64)
        gat = torch.empty_like(rows)
        for _ in range(3):
            torch.index_select(rows, 0, perm, out=gat)
        torch.cuda.synchronize()
        del rows, perm, gat

    tuned = None
    tile = tuple(int(x) for x in args.tile.split("x"))
    if not args.no_autotune:
        from paper_2605_10760_amd import autotune
        t0 = time.perf_counter()
        tuned = autotune(SceneTensors.from_numpy(wl.scene), ViewTensors.from_numpy(wl.views))
        tuned["seconds"] = round(time.perf_counter() - t0, 1)
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    ps = args.plain_steps if args.plain_steps is not None else max(2, args.steps // 4)
    res = run_workload(torch, np, wl, args, args.steps, args.warmup, tuned=tuned, tile=tile,
                       plain_steps=0 if args.no_plain else ps,
                       ab_steps=0 if args.no_extras else 5)
    print(f"[bench] {wl.name}: {res['dt'] * 1e3:.3f} ms per step", file=sys.stderr, flush=True)

    stages = {}
    for name, ms in res["stage_ms"].items():
        if ms <= 0:
            continue
        e = dict(ms=round(ms, 4))
        if name in res["bytes"]:
            e["algorithmic_GBps"] = round(res["bytes"][name] / (ms * 1e-3) / 1e9, 1)
        if name in res["ops"]:
            e["algorithmic_TFLOPs"] = round(res["ops"][name] / (ms * 1e-3) / 1e12, 2)
        stages[name] = e
    dom = max(res["stage_ms"], key=lambda k_: res["stage_ms"][k_])
    roof = roofline_of(res, dom, wl.name)
    roof_fwd = roofline_of(res, "render_fwd", wl.name) if dom != "render_fwd" else None

    extras = None
    if not args.no_extras:
        extras = measure_extras(torch, res["sc"], res["vw"], res["step"].out[0],
                                res["step"].out[1], res["tc"], res["td"], rast=res["rast"])
    main_sum = summary(res)
    for k_ in ("rast", "step", "sc", "vw", "tc", "td"):
        res.pop(k_, None)
    torch.cuda.empty_cache()

    configs = None
    if not args.no_configs:
        # the other workloads at their own sizes: small plain, room 300k plain,
        # room 1M through the autograd form, the fused SH3 map (batched vs
        # plain, its own roofline)
        configs = {}
        cs = max(2, args.config_steps)
        for name in ("small", "room", "fused"):
            w2 = make_workload(name)
            tuned2 = None
            if name == "fused" and not args.no_autotune:
                # the fused map's batch of uneven views: tile shape, batches
                # and the persistent queue tuned for it
                from paper_2605_10760_amd import autotune
                t0 = time.perf_counter()
                tuned2 = autotune(SceneTensors.from_numpy(w2.scene), ViewTensors.from_numpy(w2.views))
                tuned2["seconds"] = round(time.perf_counter() - t0, 1)
                torch.cuda.empty_cache()
            r2 = run_workload(torch, np, w2, args, cs, 2, tuned=tuned2, tile=(16, 16),
                              plain_steps=2 if name != "small" else cs,
                              ab_steps=3 if name == "fused" else 0)
            d2 = summary(r2)
            d2["roofline"] = roofline_of(r2, max(r2["stage_ms"], key=lambda k_: r2["stage_ms"][k_]),
                                         w2.name)
            d2["stages_ms"] = {k_: round(v_, 4) for k_, v_ in r2["stage_ms"].items() if v_ > 0}
            d2["autotune"] = tuned2
            configs[name] = d2
            print(f"[bench] {w2.name}: {r2['dt'] * 1e3:.3f} ms per step", file=sys.stderr,
                  flush=True)
            del r2, w2
            torch.cuda.empty_cache()
        configs["room-1m-autograd"] = run_autograd(torch, np, make_workload("room-1m"), cs, 2)
        torch.cuda.empty_cache()

    line = {
        "metric": "fwd+bwd views/sec and Gaussian-pixel evals/sec, batched vs plain, 1 MI355X",
        "value": main_sum["views_per_s"],
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_sum["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "views": res["V"], "fwd_bwd_views": res["n_bwd"],
                   "width": res["W"], "height": res["H"], "gaussians": int(wl.scene.n),
                   "sets": int(wl.scene.n_sets), "sh_degree": int(wl.scene.sh_degree),
                   "tile": main_sum["tile"], "binning_chunk": int(res["opts"]["chunk"]),
                   "fwd_batch": int(res["opts"]["fwd_batch"]),
                   "bwd_batch": int(res["opts"]["bwd_batch"]),
                   "persistent": bool(res["opts"]["persistent"]),
                   "bwd_cols": int(res["opts"].get("bwd_cols", 1)),
                   "autotuned": tuned is not None, "form": main_sum["form"]},
        "evals_per_s": main_sum["evals_per_s"],
        "evals": main_sum["evals"],
        "counts": main_sum["counts"],
        "step_algorithmic_GB": main_sum["step_algorithmic_GB"],
        "step_hbm_roofline_frac": main_sum["step_hbm_roofline_frac"],
        "plain": main_sum["plain"],
        "option_ab_ms_per_step": main_sum["option_ab_ms_per_step"],
        "stages_ms": stages,
        "roofline": roof,
        "roofline_render_fwd": roof_fwd,
        "autotune": tuned,
        "configs": configs,
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
