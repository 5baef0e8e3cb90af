"""Python front end of libgsr: device memory and streams come from PyTorch,
every computation runs in the library's HIP kernels.

    rast = Rasterizer(width, height, max_pairs, max_views)
    color, depth, alpha, state = rast.forward(scene, views)
    grads = rast.backward(scene, views, state, grad_color, grad_depth, grad_alpha)

`scene` is a SceneTensors (FP32 CUDA tensors, host set offsets), `views` a
ViewTensors (CUDA view matrices and intrinsics, host view->set map).
`rasterize()` wraps both in a torch.autograd.Function that also returns the
gradient of each view's SE(3) pose delta.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L


@dataclass
class SceneTensors:
    means: torch.Tensor          # [N,3]
    log_scales: torch.Tensor     # [N,3]
    quats: torch.Tensor          # [N,4] (w,x,y,z)
    opacity_logits: torch.Tensor # [N]
    colors: torch.Tensor         # [N,3] or [N,K,3]
    set_offsets: np.ndarray      # int64 [S+1] (host)
    sh_degree: int = 0

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def sh_stride(self) -> int:
        return 1 if self.colors.dim() == 2 else int(self.colors.shape[1])

    @staticmethod
    def from_numpy(sc, device="cuda") -> "SceneTensors":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return SceneTensors(t(sc.means), t(sc.log_scales), t(sc.quats), t(sc.opacity_logits),
                            t(sc.colors), np.asarray(sc.set_offsets, np.int64), int(sc.sh_degree))


@dataclass
class ViewTensors:
    viewmats: torch.Tensor       # [V,3,4] world->camera
    intrinsics: torch.Tensor     # [V,4]
    view_set: np.ndarray         # int32 [V] (host)
    width: int
    height: int
    needs_grad: np.ndarray = field(default=None)  # uint8 [V] (host) or None

    @property
    def n(self) -> int:
        return int(self.viewmats.shape[0])

    @staticmethod
    def from_numpy(vw, device="cuda") -> "ViewTensors":
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return ViewTensors(t(vw.viewmats), t(vw.intrinsics), np.asarray(vw.view_set, np.int32),
                           int(vw.width), int(vw.height),
                           np.asarray(vw.needs_grad, np.uint8) if vw.needs_grad is not None else None)

    def select(self, idx) -> "ViewTensors":
        idx = np.atleast_1d(np.asarray(idx))
        ti = torch.as_tensor(idx, device=self.viewmats.device)
        return ViewTensors(self.viewmats[ti].contiguous(), self.intrinsics[ti].contiguous(),
                           self.view_set[idx].copy(), self.width, self.height,
                           None if self.needs_grad is None else self.needs_grad[idx].copy())


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda or t.dtype not in (torch.float32, torch.int32, torch.uint8) or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA float32/int32/uint8 tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def pairs_of(scene: SceneTensors, views: ViewTensors) -> int:
    so = scene.set_offsets
    return int(sum(so[s + 1] - so[s] for s in views.view_set))


class Rasterizer:
    """A libgsr context with one plan (image size, tile shape, capacities)."""

    def __init__(self, width: int, height: int, max_pairs: int, max_views: int = 1,
                 max_instances: int | None = None, tile=(16, 16), device: int | None = None,
                 chunk: int = 0, fwd_batch: int = 1, bwd_batch: int = 1, persistent: bool = False,
                 bwd_cols: int = 1):
        self.lib = L.load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        st = self.lib.gsr_create(C.byref(h), self.device)
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_create failed (no gfx950 device?)")
        self.ctx = h
        if max_instances is None:
            # (pair, tile row) entries: a few per visible pair; fit_capacity
            # and gsr_poll's overflow report give the measured need
            max_instances = min(0xFFFFFFFE, max(1 << 20, 8 * int(max_pairs)))
        self.desc = L.PlanDesc(int(max_pairs), int(max_instances), int(max_views), int(width),
                               int(height), int(tile[0]), int(tile[1]), int(chunk),
                               int(fwd_batch), int(bwd_batch), int(bool(persistent)),
                               int(bwd_cols))
        self._plan()

    def _plan(self):
        self._check(self.lib.gsr_plan(self.ctx, C.byref(self.desc)))
        n = C.c_size_t()
        self._check(self.lib.gsr_state_bytes(C.byref(self.desc), C.byref(n)))
        self.state_bytes = int(n.value)

    def replan(self, **kw):
        for k, v in kw.items():
            setattr(self.desc, k, int(v))
        self._plan()

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.gsr_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def _check(self, st: int):
        if st != L.GSR_OK:
            raise L.GsrError(st, self.lib.gsr_last_error(self.ctx).decode())

    @property
    def tile(self):
        return (self.desc.tile_w, self.desc.tile_h)

    def new_state(self) -> torch.Tensor:
        # torch's caching allocator returns 512-byte aligned blocks
        return torch.empty(self.state_bytes, dtype=torch.uint8, device=f"cuda:{self.device}")

    # ------------------------------------------------------------- marshalling
    @staticmethod
    def _scene(scene: SceneTensors):
        so = np.ascontiguousarray(scene.set_offsets, np.int64)
        s = L.Scene(_ptr(scene.means), _ptr(scene.log_scales), _ptr(scene.quats),
                    _ptr(scene.opacity_logits), _ptr(scene.colors),
                    so.ctypes.data_as(C.POINTER(C.c_int64)), int(so.shape[0] - 1),
                    int(scene.sh_degree), int(scene.sh_stride), 0)
        return s, so

    @staticmethod
    def _views(views: ViewTensors):
        vs = np.ascontiguousarray(views.view_set, np.int32)
        ng = None if views.needs_grad is None else np.ascontiguousarray(views.needs_grad, np.uint8)
        v = L.Views(_ptr(views.viewmats), _ptr(views.intrinsics),
                    vs.ctypes.data_as(C.POINTER(C.c_int32)),
                    ng.ctypes.data_as(C.POINTER(C.c_uint8)) if ng is not None else None,
                    views.n, int(views.width), int(views.height), 0)
        return v, (vs, ng)

    @staticmethod
    def _settings(z_near=0.2, bg=(0.0, 0.0, 0.0)):
        return L.Settings(float(z_near), (C.c_float * 3)(*[float(b) for b in bg]))

    # ------------------------------------------------------------------ calls
    def forward(self, scene: SceneTensors, views: ViewTensors, z_near=0.2, bg=(0.0, 0.0, 0.0),
                state: torch.Tensor | None = None, out=None, n_eval=False, stream=None):
        """Render all views.  Returns (color [V,3,H,W], depth [V,H,W],
        alpha [V,H,W], state) (+ n_eval [V,H,W] int32 if n_eval)."""
        dev = scene.means.device
        V, H, W = views.n, views.height, views.width
        if out is None:
            out = (torch.empty((V, 3, H, W), dtype=torch.float32, device=dev),
                   torch.empty((V, H, W), dtype=torch.float32, device=dev),
                   torch.empty((V, H, W), dtype=torch.float32, device=dev))
        ne = torch.empty((V, H, W), dtype=torch.int32, device=dev) if n_eval else None
        if state is None:
            state = self.new_state()
        sc, keep1 = self._scene(scene)
        vw, keep2 = self._views(views)
        st = self._settings(z_near, bg)
        img = L.Images(_ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(ne))
        self._check(self.lib.gsr_forward(self.ctx, C.byref(sc), C.byref(vw), C.byref(st),
                                         C.c_void_p(state.data_ptr()), C.byref(img),
                                         _stream(stream)))
        if n_eval:
            return out[0], out[1], out[2], state, ne
        return out[0], out[1], out[2], state

    def backward(self, scene: SceneTensors, views: ViewTensors, state: torch.Tensor,
                 grad_color=None, grad_depth=None, grad_alpha=None, z_near=0.2,
                 bg=(0.0, 0.0, 0.0), out=None, stream=None):
        """Gradients of sum(g_c*color + g_d*depth + g_a*alpha) for the forward
        that wrote `state`.  Returns a dict of tensors."""
        dev = scene.means.device
        if out is None:
            out = dict(d_means=torch.empty_like(scene.means),
                       d_log_scales=torch.empty_like(scene.log_scales),
                       d_quats=torch.empty_like(scene.quats),
                       d_opacity_logits=torch.empty_like(scene.opacity_logits),
                       d_colors=torch.empty_like(scene.colors),
                       d_pose=torch.empty((views.n, 6), dtype=torch.float32, device=dev))
        sc, keep1 = self._scene(scene)
        vw, keep2 = self._views(views)
        st = self._settings(z_near, bg)
        gi = L.GradImages(_ptr(grad_color), _ptr(grad_depth), _ptr(grad_alpha))
        g = L.Grads(_ptr(out["d_means"]), _ptr(out["d_log_scales"]), _ptr(out["d_quats"]),
                    _ptr(out["d_opacity_logits"]), _ptr(out["d_colors"]), _ptr(out["d_pose"]))
        self._check(self.lib.gsr_backward(self.ctx, C.byref(sc), C.byref(vw), C.byref(st),
                                          C.c_void_p(state.data_ptr()), C.byref(gi), C.byref(g),
                                          _stream(stream)))
        return out

    def poll(self, state: torch.Tensor, raise_on_overflow=True, stream=None) -> dict:
        c = L.Counts()
        st = self.lib.gsr_poll(self.ctx, C.c_void_p(state.data_ptr()), C.byref(c), _stream(stream))
        if st not in (L.GSR_OK, L.GSR_E_OVERFLOW) or (st == L.GSR_E_OVERFLOW and raise_on_overflow):
            self._check(st)
        return dict(visible_pairs=c.visible_pairs, instances=c.instances,
                    row_entries=c.row_entries, capacity=c.capacity, overflow=bool(c.overflow))

    def fit_capacity(self, scene: SceneTensors, views: ViewTensors, z_near=0.2, margin=1.25):
        """Run one forward, and re-plan the binning's entry capacity to the
        measured need times `margin` if it overflowed or is more than four
        times too large (synchronises; for set-up, not for captured steps)."""
        _, _, _, state = self.forward(scene, views, z_near=z_near)
        c = self.poll(state, raise_on_overflow=False)
        if c["overflow"] or c["row_entries"] * margin * 4 < self.desc.max_instances:
            self.replan(max_instances=min(0xFFFFFFFE,
                                          max(1 << 20, int(c["row_entries"] * margin))))
        return c

    def profile(self, enable: bool = True):
        """Record per-stage HIP events in later forward/backward calls."""
        self._check(self.lib.gsr_profile_enable(self.ctx, int(enable)))

    def stage_ms(self) -> dict:
        """Milliseconds per stage of the most recent calls (synchronises)."""
        n = len(L.STAGES)
        buf = (C.c_float * n)()
        self._check(self.lib.gsr_profile_read(self.ctx, buf, n))
        return {name: float(buf[i]) for i, name in enumerate(L.STAGES)}

    def debug_export(self, state: torch.Tensor, n_views: int, n_pairs: int, n_inst: int,
                     stream=None, n_blend: bool = False) -> dict:
        TX = -(-self.desc.width // self.desc.tile_w)
        TY = -(-self.desc.height // self.desc.tile_h)
        H, W = self.desc.height, self.desc.width
        z = np.zeros(n_pairs, np.uint32)
        rects = np.zeros((n_pairs, 4), np.uint16)
        order = np.zeros(n_pairs, np.uint32)
        vis_off = np.zeros(n_views + 1, np.int64)
        inst = np.zeros(max(1, n_inst), np.uint32)
        ranges = np.zeros((n_views * TX * TY, 2), np.uint32)
        tf = np.zeros((n_views, H, W), np.float32)
        last = np.zeros((n_views, H, W), np.uint32)
        vp = lambda a: C.c_void_p(a.ctypes.data)
        nb = np.zeros((n_views, H, W), np.int32) if n_blend else None
        d = L.Debug(vp(z), vp(rects), vp(order), vp(vis_off), vp(inst), vp(ranges), vp(tf),
                    vp(last), vp(nb) if n_blend else None, int(n_pairs), int(n_inst))
        self._check(self.lib.gsr_debug_export(self.ctx, C.c_void_p(state.data_ptr()),
                                              int(n_views), C.byref(d), _stream(stream)))
        out = dict(zkeys=z, rects=rects, order=order[:int(vis_off[-1])], vis_off=vis_off,
                   inst=inst[:n_inst], ranges=ranges, t_final=tf, last=last, TX=TX, TY=TY)
        if n_blend:
            out["n_blend"] = nb
        return out


def autotune(scene: SceneTensors, views: ViewTensors, max_pairs: int | None = None,
             max_instances: int | None = None, z_near=0.2, device: int | None = None,
             stream=None):
    """Native coordinate search (gsr_autotune) over the tile shape, binning
    chunk, forward and backward entries per lane, tiles per backward wave
    and the persistent tile queue for this call.  Returns a dict: tile
    (tile_w, tile_h), ms (its forward+backward time), chunk, fwd_batch,
    bwd_batch, persistent, bwd_cols — the keyword arguments of Rasterizer
    besides the sizes."""
    lib = L.load()
    dev = torch.cuda.current_device() if device is None else int(device)
    P = pairs_of(scene, views) if max_pairs is None else int(max_pairs)
    base = L.PlanDesc(P, int(max_instances or min(0xFFFFFFFE, max(1 << 20, 8 * P))), views.n,
                      views.width, views.height, 16, 16, 0, 1, 1, 0, 1)
    sc, keep1 = Rasterizer._scene(scene)
    vw, keep2 = Rasterizer._views(views)
    st = Rasterizer._settings(z_near)
    best = L.PlanDesc()
    ms = C.c_float()
    status = lib.gsr_autotune(dev, C.byref(base), C.byref(sc), C.byref(vw), C.byref(st),
                              C.byref(best), C.byref(ms), _stream(stream))
    if status != L.GSR_OK:
        raise L.GsrError(status, "gsr_autotune failed")
    return dict(tile=(best.tile_w, best.tile_h), ms=float(ms.value), chunk=int(best.chunk),
                fwd_batch=int(best.fwd_batch) or 1, bwd_batch=int(best.bwd_batch) or 1,
                persistent=bool(best.persistent), bwd_cols=int(best.bwd_cols) or 1)


def apply_pose_delta(viewmats: torch.Tensor, delta: torch.Tensor, out: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """Exp(delta[v]) @ viewmats[v] on the device (left SE(3) update)."""
    lib = L.load()
    if out is None:
        out = torch.empty_like(viewmats)
    st = lib.gsr_apply_pose_delta(_ptr(viewmats.contiguous()), _ptr(delta.contiguous()),
                                  _ptr(out), int(viewmats.shape[0]), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_apply_pose_delta failed")
    return out


def sim3_gaussians(means: torch.Tensor, log_scales: torch.Tensor, quats: torch.Tensor,
                   set_offsets, sims: torch.Tensor, out=None, stream=None):
    """Sim(3) correction of every Gaussian set on the device (set k moved by
    sims[k] = (s, qw, qx, qy, qz, tx, ty, tz)); returns (means, log_scales,
    quats), written to `out` (a 3-tuple, may alias the inputs) if given."""
    lib = L.load()
    offs = np.ascontiguousarray(np.asarray(set_offsets, np.int64))
    if out is None:
        out = (torch.empty_like(means), torch.empty_like(log_scales), torch.empty_like(quats))
    st = lib.gsr_sim3_gaussians(_ptr(means.contiguous()), _ptr(log_scales.contiguous()),
                                _ptr(quats.contiguous()),
                                offs.ctypes.data_as(C.POINTER(C.c_int64)), int(offs.shape[0] - 1),
                                _ptr(sims.contiguous()), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]),
                                _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_sim3_gaussians failed")
    return out


def sim3_views(viewmats: torch.Tensor, sims: torch.Tensor, view_set, out=None, stream=None):
    """Lift of keyframe poses into the global frame by their sets'
    similarities (rigid form: the camera's length unit scaled by s)."""
    lib = L.load()
    vs = np.ascontiguousarray(np.asarray(view_set, np.int32))
    if out is None:
        out = torch.empty_like(viewmats)
    st = lib.gsr_sim3_views(_ptr(viewmats.contiguous()), _ptr(sims.contiguous()),
                            vs.ctypes.data_as(C.POINTER(C.c_int32)), int(vs.shape[0]),
                            int(sims.shape[0]), _ptr(out), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_sim3_views failed")
    return out


def l1_loss_grad(color: torch.Tensor, target_color: torch.Tensor, depth: torch.Tensor | None = None,
                 target_depth: torch.Tensor | None = None, exposure: torch.Tensor | None = None,
                 w_color: float = 0.95, w_depth: float = 0.25, out: dict | None = None,
                 stream=None) -> dict:
    """Gradient of w_color mean|exp(a) I^ + b - I| + w_depth mean|D^ - D| on
    the device (exposure [V,2] = (a, b) per view, or None for a = b = 0).
    Returns dict d_color, d_depth (None without depth), d_exposure (None
    without exposure)."""
    lib = L.load()
    V, _, H, W = color.shape
    if out is None:
        out = dict(d_color=torch.empty_like(color),
                   d_depth=torch.empty_like(depth) if depth is not None else None,
                   d_exposure=torch.empty((V, 2), device=color.device)
                   if exposure is not None else None)
    c = lambda t: None if t is None else t.contiguous()
    st = lib.gsr_l1_loss_grad(_ptr(c(color)), _ptr(c(depth)), _ptr(c(target_color)),
                              _ptr(c(target_depth)), _ptr(c(exposure)), int(V), int(W), int(H),
                              float(w_color), float(w_depth), _ptr(out["d_color"]),
                              _ptr(out["d_depth"]), _ptr(out["d_exposure"]), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_l1_loss_grad failed")
    return out


def ssim_grad(color: torch.Tensor, target_color: torch.Tensor, d_color: torch.Tensor,
              exposure: torch.Tensor | None = None, d_exposure: torch.Tensor | None = None,
              weight: float = 0.2, workspace: torch.Tensor | None = None,
              ssim_out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Adds the gradient of weight (1 - SSIM(exp(a) I^ + b, I)) into d_color
    (and d_exposure if given) on the device; returns the workspace (reuse it
    across calls to avoid allocations, e.g. under graph capture)."""
    lib = L.load()
    V, _, H, W = color.shape
    if workspace is None:
        nb = C.c_size_t()
        st = lib.gsr_ssim_workspace_bytes(int(V), int(W), int(H), C.byref(nb))
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_ssim_workspace_bytes failed")
        workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=color.device)
    c = lambda t: None if t is None else t.contiguous()
    st = lib.gsr_ssim_grad(_ptr(c(color)), _ptr(c(target_color)), _ptr(c(exposure)), int(V),
                           int(W), int(H), float(weight), _ptr(workspace), _ptr(d_color),
                           _ptr(d_exposure), _ptr(ssim_out), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_ssim_grad failed")
    return workspace


def dedup(src_means: torch.Tensor, tgt_means: torch.Tensor, tgt_log_scales: torch.Tensor,
          depth: torch.Tensor | None, viewmats: torch.Tensor | None,
          intrinsics: torch.Tensor | None, voxel: float = 0.05, k_env: float = 1.0,
          table_slots: int | None = None, stream=None):
    """Occupancy-aware deduplication on the device: returns (keep uint8
    [n_src], distinct voxels).  depth [K,H,W] (camera depth of the target's
    keyframes) may be None (no free-space carving).  With table_slots None
    the hash set starts at twice the number of boxes and rays (rays of one
    keyframe share most of their voxels) and grows fourfold when it
    overflows.  Synchronises."""
    lib = L.load()
    n_tgt, n_src = int(tgt_means.shape[0]), int(src_means.shape[0])
    K = 0 if depth is None else int(depth.shape[0])
    H = 0 if depth is None else int(depth.shape[1])
    W = 0 if depth is None else int(depth.shape[2])
    grow = table_slots is None
    if grow:
        est = 2 * (n_tgt + K * H * W) + 1024
        table_slots = 1 << max(10, int(est - 1).bit_length())
    keep = torch.empty(n_src, dtype=torch.uint8, device=src_means.device)
    nvox = C.c_int64()
    c = lambda t: None if t is None else t.contiguous()
    while True:
        nb = C.c_size_t()
        st = lib.gsr_dedup_workspace_bytes(int(table_slots), C.byref(nb))
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_dedup_workspace_bytes failed")
        ws = torch.empty(int(nb.value), dtype=torch.uint8, device=src_means.device)
        prm = L.DedupParams(float(voxel), float(k_env), int(table_slots))
        st = lib.gsr_dedup(C.byref(prm), _ptr(c(tgt_means)), _ptr(c(tgt_log_scales)), n_tgt,
                           _ptr(c(depth)), _ptr(c(viewmats)), _ptr(c(intrinsics)), K, W, H,
                           _ptr(c(src_means)), n_src, _ptr(keep), _ptr(ws), C.byref(nvox),
                           _stream(stream))
        if st == L.GSR_E_OVERFLOW and grow and table_slots < (1 << 30):
            del ws
            table_slots *= 4
            continue
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_dedup failed")
        return keep, int(nvox.value)


def prune(scene: SceneTensors, min_opacity: float = 0.005, stream=None) -> SceneTensors:
    """Opacity pruning on the device: a new SceneTensors with the Gaussians
    whose sigmoid(opacity) >= min_opacity, in order, and the pruned set
    offsets (synchronises)."""
    lib = L.load()
    s, so = Rasterizer._scene(scene)
    new = [torch.empty_like(x) for x in (scene.means, scene.log_scales, scene.quats,
                                         scene.opacity_logits, scene.colors)]
    offs = np.zeros(so.shape[0], np.int64)
    st = lib.gsr_prune(C.byref(s), float(min_opacity), *(_ptr(x) for x in new),
                       offs.ctypes.data_as(C.POINTER(C.c_int64)), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_prune failed")
    n = int(offs[-1])
    return SceneTensors(*(x[:n] for x in new), offs, scene.sh_degree)


def iso_grad(log_scales: torch.Tensor, d_log_scales: torch.Tensor, weight: float = 10.0,
             stream=None) -> torch.Tensor:
    """Adds weight * d/d log_scales of sum_i sum_c |s_ic - mean_c s_ic|
    (s = exp(log_scales) [n,3]) into d_log_scales on the device."""
    lib = L.load()
    st = lib.gsr_iso_grad(_ptr(log_scales.contiguous()), int(log_scales.shape[0]), float(weight),
                          _ptr(d_log_scales), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_iso_grad failed")
    return d_log_scales


def normal_loss_grad(depth: torch.Tensor, normal_prior: torch.Tensor, intrinsics: torch.Tensor,
                     d_depth: torch.Tensor, weight: float = 1e-2, stream=None) -> torch.Tensor:
    """Adds weight * dL_normal/dD into d_depth [V,H,W] on the device;
    L_normal is the mean over interior pixels of 1 - N(D) . prior with the
    depth-induced normal N (prior [V,3,H,W])."""
    lib = L.load()
    V, H, W = depth.shape
    st = lib.gsr_normal_loss_grad(_ptr(depth.contiguous()), _ptr(normal_prior.contiguous()),
                                  _ptr(intrinsics.contiguous()), int(V), int(W), int(H),
                                  float(weight), _ptr(d_depth), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_normal_loss_grad failed")
    return d_depth


def seed(depth: torch.Tensor, color: torch.Tensor, viewmat: torch.Tensor,
         intrinsics: torch.Tensor, stride: int = 1, opacity_logit: float = 0.0,
         stream=None) -> dict:
    """Gaussians seeded from one keyframe (depth [H,W], color [3,H,W],
    viewmat [3,4], intrinsics [4]) on the device: dict of means, log_scales,
    quats, opacity_logits, colors (synchronises)."""
    lib = L.load()
    H, W = depth.shape
    cap = ((W + stride - 1) // stride) * ((H + stride - 1) // stride)
    dev = depth.device
    out = dict(means=torch.empty((cap, 3), device=dev), log_scales=torch.empty((cap, 3), device=dev),
               quats=torch.empty((cap, 4), device=dev), opacity_logits=torch.empty(cap, device=dev),
               colors=torch.empty((cap, 3), device=dev))
    n = C.c_int64()
    st = lib.gsr_seed(_ptr(depth.contiguous()), _ptr(color.contiguous()),
                      _ptr(viewmat.contiguous()), _ptr(intrinsics.contiguous()), int(W), int(H),
                      int(stride), float(opacity_logit), int(cap), _ptr(out["means"]),
                      _ptr(out["log_scales"]), _ptr(out["quats"]), _ptr(out["opacity_logits"]),
                      _ptr(out["colors"]), C.byref(n), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_seed failed")
    return {k: v[:int(n.value)] for k, v in out.items()}


def seed_noalloc(depth: torch.Tensor, color: torch.Tensor, viewmat: torch.Tensor,
                 intrinsics: torch.Tensor, out: dict, n_out: torch.Tensor, stride: int = 1,
                 opacity_logit: float = 0.0, stream=None) -> None:
    """gsr_seed_noalloc: seeding into caller-allocated rows `out` (means,
    log_scales, quats, opacity_logits, colors, capacity = their row count)
    with the seeded count written to the device int64 tensor `n_out` [1];
    the library allocates nothing and does not synchronise."""
    lib = L.load()
    H, W = depth.shape
    cap = int(out["means"].shape[0])
    if not (n_out.dtype == torch.int64 and n_out.numel() == 1 and n_out.is_cuda):
        raise ValueError("n_out must be a one-element int64 CUDA tensor")
    st = lib.gsr_seed_noalloc(_ptr(depth), _ptr(color), _ptr(viewmat), _ptr(intrinsics),
                              int(W), int(H), int(stride), float(opacity_logit), cap,
                              _ptr(out["means"]), _ptr(out["log_scales"]), _ptr(out["quats"]),
                              _ptr(out["opacity_logits"]), _ptr(out["colors"]),
                              C.c_void_p(n_out.data_ptr()), _stream(stream))
    if st != L.GSR_OK:
        raise L.GsrError(st, "gsr_seed_noalloc failed")


class Adam:
    """Adam over a list of (parameter, learning rate) on the device: one
    gsr_adam launch per step updates every parameter from its `.grad` (the
    tensor itself is read at each step, so gradients may be written in place
    between steps).  Moments and the step count are device buffers, so
    `step()` allocates nothing and can be captured in a graph."""

    def __init__(self, params_lrs, betas=(0.9, 0.999), eps=1e-15):
        self.lib = L.load()
        self.params = [p for p, _ in params_lrs]
        self.lrs = [float(lr) for _, lr in params_lrs]
        if not 1 <= len(self.params) <= L.GSR_ADAM_MAX_GROUPS:
            raise ValueError(f"1..{L.GSR_ADAM_MAX_GROUPS} parameter arrays")
        for p in self.params:
            if not (p.is_cuda and p.dtype == torch.float32 and p.is_contiguous()):
                raise ValueError("parameters must be contiguous CUDA float32 tensors")
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = torch.zeros(1, dtype=torch.int32, device=self.params[0].device)
        self.betas, self.eps = (float(betas[0]), float(betas[1])), float(eps)

    def step(self, stream=None):
        groups = (L.AdamGroup * len(self.params))()
        for k, p in enumerate(self.params):
            if p.grad is None or not p.grad.is_contiguous():
                raise ValueError("every parameter needs a contiguous .grad")
            groups[k] = L.AdamGroup(p.data_ptr(), p.grad.data_ptr(), self.m[k].data_ptr(),
                                    self.v[k].data_ptr(), p.numel(), self.lrs[k], 0)
        st = self.lib.gsr_adam(groups, len(self.params), self.betas[0], self.betas[1], self.eps,
                               _ptr(self.t), _stream(stream))
        if st != L.GSR_OK:
            raise L.GsrError(st, "gsr_adam failed")


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, colors, pose_delta, viewmats,
                intrinsics, meta):
        rast, set_offsets, view_set, needs_grad, sh_degree, z_near, bg, W, H = meta
        vm = apply_pose_delta(viewmats, pose_delta) if pose_delta is not None else viewmats
        scene = SceneTensors(means.contiguous(), log_scales.contiguous(), quats.contiguous(),
                             opacity_logits.contiguous(), colors.contiguous(), set_offsets,
                             sh_degree)
        views = ViewTensors(vm.contiguous(), intrinsics.contiguous(), view_set, W, H, needs_grad)
        color, depth, alpha, state = rast.forward(scene, views, z_near=z_near, bg=bg)
        ctx.meta = meta
        ctx.scene = scene
        ctx.views = views
        ctx.state = state
        ctx.has_pose = pose_delta is not None
        return color, depth, alpha

    @staticmethod
    def backward(ctx, gc, gd, ga):
        rast, _, _, _, _, z_near, bg, _, _ = ctx.meta
        c = lambda t: None if t is None else t.contiguous()
        g = rast.backward(ctx.scene, ctx.views, ctx.state, c(gc), c(gd), c(ga), z_near=z_near,
                          bg=bg)
        return (g["d_means"], g["d_log_scales"], g["d_quats"], g["d_opacity_logits"],
                g["d_colors"], g["d_pose"] if ctx.has_pose else None, None, None, None)


def rasterize(rast: Rasterizer, means, log_scales, quats, opacity_logits, colors, viewmats,
              intrinsics, set_offsets, view_set, width, height, pose_delta=None, sh_degree=0,
              needs_grad=None, z_near=0.2, bg=(0.0, 0.0, 0.0)):
    """Differentiable render of V views.  Returns (color [V,3,H,W], depth
    [V,H,W], alpha [V,H,W]).  If `pose_delta` [V,6] is given (normally zeros
    with requires_grad), each view is rendered at Exp(pose_delta) @ viewmat
    and pose_delta.grad is the left-perturbation pose gradient there."""
    meta = (rast, np.asarray(set_offsets, np.int64), np.asarray(view_set, np.int32),
            None if needs_grad is None else np.asarray(needs_grad, np.uint8), int(sh_degree),
            float(z_near), tuple(float(b) for b in bg), int(width), int(height))
    return _RasterizeFn.apply(means, log_scales, quats, opacity_logits, colors, pose_delta,
                              viewmats, intrinsics, meta)
