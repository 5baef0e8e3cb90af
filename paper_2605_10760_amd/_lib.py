"""ctypes binding of libgsr.so (include/gsr.h).  Argument marshalling only:
every step of the rasterizer runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

GSR_MAX_VIEWS = 64
GSR_MAX_SETS = 64
GSR_SEED_NOALLOC_MAX_POINTS = 1 << 24
GSR_ADAM_MAX_GROUPS = 8

STATUS = {0: "GSR_OK", 1: "GSR_E_INVALID_ARG", 2: "GSR_E_NOT_PLANNED", 3: "GSR_E_CAPACITY",
          4: "GSR_E_OVERFLOW", 5: "GSR_E_DEVICE", 6: "GSR_E_OOM", 7: "GSR_E_UNIMPLEMENTED"}
GSR_OK, GSR_E_INVALID_ARG, GSR_E_NOT_PLANNED, GSR_E_CAPACITY = 0, 1, 2, 3
GSR_E_OVERFLOW, GSR_E_DEVICE, GSR_E_OOM, GSR_E_UNIMPLEMENTED = 4, 5, 6, 7

EXPORTED = ("gsr_create", "gsr_destroy", "gsr_plan", "gsr_state_bytes", "gsr_forward",
            "gsr_backward", "gsr_poll", "gsr_debug_export", "gsr_apply_pose_delta",
            "gsr_autotune", "gsr_profile_enable", "gsr_profile_read", "gsr_status_string",
            "gsr_last_error", "gsr_sim3_gaussians", "gsr_sim3_views", "gsr_l1_loss_grad",
            "gsr_prune", "gsr_ssim_workspace_bytes", "gsr_ssim_grad",
            "gsr_dedup_workspace_bytes", "gsr_dedup", "gsr_iso_grad", "gsr_normal_loss_grad",
            "gsr_seed", "gsr_seed_noalloc", "gsr_adam")

STAGES = ("project", "compact", "depth_sort", "binning", "render_fwd", "zero", "render_bwd",
          "project_bwd", "record")


class PlanDesc(C.Structure):
    _fields_ = [("max_pairs", C.c_int64), ("max_instances", C.c_int64),
                ("max_views", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("chunk", C.c_int32),
                ("fwd_batch", C.c_int32), ("bwd_batch", C.c_int32), ("persistent", C.c_int32),
                ("bwd_cols", C.c_int32)]


class Scene(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("colors", C.c_void_p),
                ("set_offsets", C.POINTER(C.c_int64)), ("n_sets", C.c_int32),
                ("sh_degree", C.c_int32), ("sh_stride", C.c_int32), ("reserved", C.c_int32)]


class Views(C.Structure):
    _fields_ = [("viewmats", C.c_void_p), ("intrinsics", C.c_void_p),
                ("view_set", C.POINTER(C.c_int32)), ("needs_grad", C.POINTER(C.c_uint8)),
                ("n_views", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("reserved", C.c_int32)]


class Settings(C.Structure):
    _fields_ = [("z_near", C.c_float), ("bg", C.c_float * 3)]


class Images(C.Structure):
    _fields_ = [("color", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p),
                ("n_eval", C.c_void_p)]


class GradImages(C.Structure):
    _fields_ = [("color", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_log_scales", C.c_void_p), ("d_quats", C.c_void_p),
                ("d_opacity_logits", C.c_void_p), ("d_colors", C.c_void_p),
                ("d_pose", C.c_void_p)]


class Counts(C.Structure):
    _fields_ = [("visible_pairs", C.c_int64), ("instances", C.c_int64),
                ("row_entries", C.c_int64), ("capacity", C.c_int64),
                ("overflow", C.c_int32), ("n_views", C.c_int32)]


class DedupParams(C.Structure):
    _fields_ = [("voxel", C.c_double), ("k_env", C.c_double), ("table_slots", C.c_int64)]


class AdamGroup(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("exp_avg", C.c_void_p),
                ("exp_avg_sq", C.c_void_p), ("n", C.c_int64), ("lr", C.c_float),
                ("reserved", C.c_int32)]


class Debug(C.Structure):
    _fields_ = [("zkeys", C.c_void_p), ("rects", C.c_void_p), ("order", C.c_void_p),
                ("vis_off", C.c_void_p), ("inst", C.c_void_p), ("ranges", C.c_void_p),
                ("t_final", C.c_void_p), ("last", C.c_void_p), ("n_blend", C.c_void_p),
                ("n_pairs", C.c_int64),
                ("n_inst", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libgsr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2605_10760_amd.build`")
    lib = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    lib.gsr_create.argtypes = [P(vp), C.c_int]
    lib.gsr_create.restype = C.c_int
    lib.gsr_destroy.argtypes = [vp]
    lib.gsr_destroy.restype = None
    lib.gsr_plan.argtypes = [vp, P(PlanDesc)]
    lib.gsr_plan.restype = C.c_int
    lib.gsr_state_bytes.argtypes = [P(PlanDesc), P(C.c_size_t)]
    lib.gsr_state_bytes.restype = C.c_int
    lib.gsr_forward.argtypes = [vp, P(Scene), P(Views), P(Settings), vp, P(Images), vp]
    lib.gsr_forward.restype = C.c_int
    lib.gsr_backward.argtypes = [vp, P(Scene), P(Views), P(Settings), vp, P(GradImages),
                                 P(Grads), vp]
    lib.gsr_backward.restype = C.c_int
    lib.gsr_poll.argtypes = [vp, vp, P(Counts), vp]
    lib.gsr_poll.restype = C.c_int
    lib.gsr_debug_export.argtypes = [vp, vp, C.c_int32, P(Debug), vp]
    lib.gsr_debug_export.restype = C.c_int
    lib.gsr_apply_pose_delta.argtypes = [vp, vp, vp, C.c_int32, vp]
    lib.gsr_apply_pose_delta.restype = C.c_int
    lib.gsr_autotune.argtypes = [C.c_int, P(PlanDesc), P(Scene), P(Views), P(Settings),
                                 P(PlanDesc), P(C.c_float), vp]
    lib.gsr_autotune.restype = C.c_int
    lib.gsr_profile_enable.argtypes = [vp, C.c_int]
    lib.gsr_profile_enable.restype = C.c_int
    lib.gsr_profile_read.argtypes = [vp, P(C.c_float), C.c_int32]
    lib.gsr_profile_read.restype = C.c_int
    lib.gsr_sim3_gaussians.argtypes = [vp, vp, vp, P(C.c_int64), C.c_int32, vp, vp, vp, vp, vp]
    lib.gsr_sim3_gaussians.restype = C.c_int
    lib.gsr_sim3_views.argtypes = [vp, vp, P(C.c_int32), C.c_int32, C.c_int32, vp, vp]
    lib.gsr_sim3_views.restype = C.c_int
    lib.gsr_l1_loss_grad.argtypes = [vp, vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_float, C.c_float, vp, vp, vp, vp]
    lib.gsr_l1_loss_grad.restype = C.c_int
    lib.gsr_ssim_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, P(C.c_size_t)]
    lib.gsr_ssim_workspace_bytes.restype = C.c_int
    lib.gsr_ssim_grad.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float, vp, vp,
                                  vp, vp, vp]
    lib.gsr_ssim_grad.restype = C.c_int
    lib.gsr_dedup_workspace_bytes.argtypes = [C.c_int64, P(C.c_size_t)]
    lib.gsr_dedup_workspace_bytes.restype = C.c_int
    lib.gsr_dedup.argtypes = [P(DedupParams), vp, vp, C.c_int64, vp, vp, vp, C.c_int32, C.c_int32,
                              C.c_int32, vp, C.c_int64, vp, vp, P(C.c_int64), vp]
    lib.gsr_dedup.restype = C.c_int
    lib.gsr_prune.argtypes = [P(Scene), C.c_float, vp, vp, vp, vp, vp, P(C.c_int64), vp]
    lib.gsr_prune.restype = C.c_int
    lib.gsr_iso_grad.argtypes = [vp, C.c_int64, C.c_float, vp, vp]
    lib.gsr_iso_grad.restype = C.c_int
    lib.gsr_normal_loss_grad.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                         vp, vp]
    lib.gsr_normal_loss_grad.restype = C.c_int
    lib.gsr_seed.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                             C.c_int64, vp, vp, vp, vp, vp, P(C.c_int64), vp]
    lib.gsr_seed.restype = C.c_int
    lib.gsr_seed_noalloc.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                     C.c_int64, vp, vp, vp, vp, vp, vp, vp]
    lib.gsr_seed_noalloc.restype = C.c_int
    lib.gsr_adam.argtypes = [P(AdamGroup), C.c_int32, C.c_double, C.c_double, C.c_double, vp, vp]
    lib.gsr_adam.restype = C.c_int
    lib.gsr_status_string.argtypes = [C.c_int]
    lib.gsr_status_string.restype = C.c_char_p
    lib.gsr_last_error.argtypes = [vp]
    lib.gsr_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class GsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
