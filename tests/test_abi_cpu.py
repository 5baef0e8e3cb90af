"""The C ABI library loads, exports every symbol include/gsr.h declares, and
its host-only entry points and error paths behave (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_bound_entry_points():
    from paper_2605_10760_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_create_without_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    h = C.c_void_p(123)
    assert lib.gsr_create(C.byref(h), 0) == _lib.GSR_E_DEVICE
    assert not h.value
    assert lib.gsr_status_string(_lib.GSR_E_DEVICE) == b"device error"


def _desc(**kw):
    from paper_2605_10760_amd import _lib
    d = dict(max_pairs=1000, max_instances=10000, max_views=2, width=128, height=96,
             tile_w=16, tile_h=16, chunk=0, fwd_batch=0, bwd_batch=0, persistent=0, bwd_cols=0)
    d.update(kw)
    return _lib.PlanDesc(*[d[k] for k in ("max_pairs", "max_instances", "max_views", "width",
                                          "height", "tile_w", "tile_h", "chunk", "fwd_batch",
                                          "bwd_batch", "persistent", "bwd_cols")])


def test_state_bytes_host_only_and_validation():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    n = C.c_size_t()
    assert lib.gsr_state_bytes(C.byref(_desc()), C.byref(n)) == _lib.GSR_OK
    # header + per pair (depth key, visible position, rect, record, order) + row ranges
    # (2 views x 6 rows) + row entries (8 B each) + tile order + 2 per-pixel planes
    assert n.value >= (512 + 1000 * (4 + 4 + 8 + 48 + 4) + 2 * 6 * 8 + 10000 * 8
                       + 2 * 48 * 4 + 2 * 2 * 128 * 96 * 4)
    assert n.value % 256 == 0
    for bad in (dict(max_pairs=0), dict(max_views=65), dict(tile_w=12), dict(tile_w=32, tile_h=32),
                dict(width=0), dict(max_instances=0), dict(chunk=-1), dict(fwd_batch=3),
                dict(bwd_batch=3), dict(bwd_batch=8), dict(persistent=2), dict(bwd_cols=3),
                dict(bwd_cols=2, tile_w=32, tile_h=8), dict(bwd_cols=2, tile_w=16, tile_h=32)):
        assert lib.gsr_state_bytes(C.byref(_desc(**bad)), C.byref(n)) == _lib.GSR_E_INVALID_ARG, bad
    for good in (dict(bwd_cols=2), dict(bwd_cols=2, tile_w=8, tile_h=16),
                 dict(bwd_cols=1, tile_w=32, tile_h=16)):
        assert lib.gsr_state_bytes(C.byref(_desc(**good)), C.byref(n)) == _lib.GSR_OK, good
    assert lib.gsr_state_bytes(None, C.byref(n)) == _lib.GSR_E_INVALID_ARG


def test_null_context_paths():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    assert lib.gsr_plan(None, C.byref(_desc())) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_forward(None, None, None, None, None, None, None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_backward(None, None, None, None, None, None, None, None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_poll(None, None, None, None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_apply_pose_delta(None, None, None, 1, None) == _lib.GSR_E_INVALID_ARG
    assert lib.gsr_last_error(None) == b"no context"
    lib.gsr_destroy(None)


def test_sim3_argument_validation():
    """Host-side checks of the Sim(3) entry points (no kernel is launched)."""
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    E = _lib.GSR_E_INVALID_ARG
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    offs = (C.c_int64 * 3)(0, 5, 3)  # decreasing
    assert lib.gsr_sim3_gaussians(None, fake, fake, offs, 2, fake, fake, fake, fake, None) == E
    assert lib.gsr_sim3_gaussians(fake, fake, fake, offs, 2, fake, fake, fake, fake, None) == E
    offs0 = (C.c_int64 * 2)(1, 5)  # does not start at 0
    assert lib.gsr_sim3_gaussians(fake, fake, fake, offs0, 1, fake, fake, fake, fake, None) == E
    assert lib.gsr_sim3_gaussians(fake, fake, fake, offs, 0, fake, fake, fake, fake, None) == E
    vs = (C.c_int32 * 2)(0, 3)  # set 3 of 2
    assert lib.gsr_sim3_views(fake, fake, vs, 2, 2, fake, None) == E
    assert lib.gsr_sim3_views(fake, fake, vs, 0, 2, fake, None) == E
    assert lib.gsr_sim3_views(None, fake, vs, 2, 4, fake, None) == E


def test_refine_argument_validation():
    """Host-side checks of the loss-gradient and pruning entry points."""
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    E = _lib.GSR_E_INVALID_ARG
    f = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.gsr_l1_loss_grad(None, None, f, None, None, 1, 4, 4, 1.0, 0.0, f, None, None, None) == E
    assert lib.gsr_l1_loss_grad(f, None, f, None, None, 0, 4, 4, 1.0, 0.0, f, None, None, None) == E
    # a depth gradient needs both depth inputs
    assert lib.gsr_l1_loss_grad(f, None, f, f, None, 1, 4, 4, 1.0, 1.0, f, f, None, None) == E
    assert lib.gsr_prune(None, 0.005, f, f, f, f, f, None, None) == E
    offs = (C.c_int64 * 2)(0, 10)
    sc = _lib.Scene(f, f, f, f, f, C.cast(offs, C.POINTER(C.c_int64)), 1, 0, 1, 0)
    out = (C.c_int64 * 2)()
    assert lib.gsr_prune(C.byref(sc), 1.5, f, f, f, f, f, out, None) == E
    assert lib.gsr_prune(C.byref(sc), 0.005, f, f, f, f, None, out, None) == E


def test_ssim_argument_validation():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    E = _lib.GSR_E_INVALID_ARG
    nb = C.c_size_t()
    assert lib.gsr_ssim_workspace_bytes(2, 64, 48, C.byref(nb)) == _lib.GSR_OK
    # per 32 x 32 tile and channel: a partial SSIM sum and two exposure
    # partials; per view one float
    tiles = 2 * 2 * 3 * 2
    assert nb.value >= tiles * 4 + tiles * 8 + 2 * 4
    assert lib.gsr_ssim_workspace_bytes(0, 64, 48, C.byref(nb)) == E
    f = C.c_void_p(0x1000)
    assert lib.gsr_ssim_grad(None, f, None, 1, 8, 8, 0.2, f, f, None, None, None) == E
    # misaligned workspace
    assert lib.gsr_ssim_grad(f, f, None, 1, 8, 8, 0.2, C.c_void_p(0x1004), f, None, None, None) == E


def test_dedup_argument_validation():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    E = _lib.GSR_E_INVALID_ARG
    nb = C.c_size_t()
    assert lib.gsr_dedup_workspace_bytes(1 << 10, C.byref(nb)) == _lib.GSR_OK
    assert nb.value >= 12 * 1024
    assert lib.gsr_dedup_workspace_bytes(1000, C.byref(nb)) == E  # not a power of two
    f = C.c_void_p(0x1000)
    n = C.c_int64()
    bad = [_lib.DedupParams(0.0, 1.0, 1 << 10), _lib.DedupParams(0.05, -1.0, 1 << 10),
           _lib.DedupParams(0.05, 1.0, 1000)]
    for prm in bad:
        assert lib.gsr_dedup(C.byref(prm), f, f, 10, None, None, None, 0, 0, 0, f, 10, f, f,
                             C.byref(n), None) == E
    ok = _lib.DedupParams(0.05, 1.0, 1 << 10)
    # keyframes without depth arrays
    assert lib.gsr_dedup(C.byref(ok), f, f, 10, None, None, None, 2, 8, 8, f, 10, f, f,
                         C.byref(n), None) == E
    # misaligned workspace
    assert lib.gsr_dedup(C.byref(ok), f, f, 10, None, None, None, 0, 0, 0, f, 10, f,
                         C.c_void_p(0x1008), C.byref(n), None) == E


def test_mapping_argument_validation():
    from paper_2605_10760_amd import _lib
    lib = _lib.load()
    E = _lib.GSR_E_INVALID_ARG
    f = C.c_void_p(0x1000)
    assert lib.gsr_iso_grad(f, -1, 10.0, f, None) == E
    assert lib.gsr_iso_grad(None, 5, 10.0, f, None) == E
    assert lib.gsr_iso_grad(f, 5, 10.0, None, None) == E
    assert lib.gsr_normal_loss_grad(None, f, f, 1, 8, 8, 1.0, f, None) == E
    assert lib.gsr_normal_loss_grad(f, f, f, 0, 8, 8, 1.0, f, None) == E
    # no interior pixel: nothing to do, no device work
    assert lib.gsr_normal_loss_grad(f, f, f, 1, 2, 8, 1.0, f, None) == _lib.GSR_OK
    n = C.c_int64()
    args = [f, f, f, f, 8, 8, 1, 0.0, 64, f, f, f, f, f, C.byref(n), None]
    for k, bad in ((6, 0), (8, -1), (9, None), (14, None), (4, 0)):
        a = list(args)
        a[k] = bad
        assert lib.gsr_seed(*a) == E, k
