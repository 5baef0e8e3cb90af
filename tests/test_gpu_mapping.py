"""GPU parity of the mapping-loss extras (Sec. III-A, Eq. (map_loss)):
isotropy gradient, depth-normal loss gradient and back-projection seeding,
through the C ABI, against the oracle."""
import numpy as np
import pytest

from gpu_harness import announce
from oracle.mapping import iso_loss_grad, normal_loss_grad, seed
from synth.scenes import look_at, slanted_depth

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_iso_grad_matches_oracle():
    announce("mapping iso grad")
    import torch
    from paper_2605_10760_amd import iso_grad
    rng = np.random.default_rng(31)
    n = 100_003  # ragged against the 256-thread blocks
    ls = rng.normal(-3.0, 0.5, (n, 3)).astype(np.float32)
    ls[:50] = ls[:50, :1]            # isotropic: zero gradient
    ls[50:100, 1] = ls[50:100, 0]    # two equal components
    base = rng.normal(0, 1e-3, (n, 3)).astype(np.float32)
    g = _t(base)
    iso_grad(_t(ls), g, weight=10.0)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64) - base
    ref = 10.0 * iso_loss_grad(ls)
    s = np.exp(ls.astype(np.float64))
    # components within FP32 rounding of their Gaussian's mean scale may take
    # either sign of the subgradient; compare the Gaussians without such a tie
    rel = np.abs(s - s.mean(1, keepdims=True)) / s.mean(1, keepdims=True)
    tie = np.any((rel < 1e-5) & (rel > 0), axis=1)
    assert tie.sum() < n // 1000
    np.testing.assert_allclose(got[~tie], ref[~tie], rtol=1e-4, atol=2e-6)
    assert np.all(got[:50] == 0.0)
    # empty input is a no-op
    iso_grad(torch.empty((0, 3), device="cuda"), torch.empty((0, 3), device="cuda"))


@pytest.mark.parametrize("V,H,W", [(2, 37, 53), (1, 3, 3), (1, 16, 16), (3, 33, 17)])
def test_normal_loss_grad_matches_oracle(V, H, W):
    announce(f"mapping normal grad {V}x{H}x{W}")
    import torch
    from paper_2605_10760_amd import normal_loss_grad as gpu_grad
    rng = np.random.default_rng(40 + H)
    depth, prior, intr = slanted_depth(rng, V, W, H, f=0.8 * W, hole_frac=0.03)
    base = rng.normal(0, 1e-3, depth.shape).astype(np.float32)
    g = _t(base)
    gpu_grad(_t(depth), _t(prior), _t(intr), g, weight=0.5)
    torch.cuda.synchronize()
    got = g.cpu().numpy().astype(np.float64) - base
    ref = 0.5 * normal_loss_grad(depth, np.moveaxis(prior, 1, -1), intr)
    scale = np.abs(ref).max()
    assert scale > 0
    np.testing.assert_allclose(got, ref, rtol=1e-3, atol=1e-4 * scale)


def test_normal_loss_grad_full_size_sampled():
    """48 views at 640 x 480 in one launch; views 0, 17 and 47 against the
    oracle (views are independent; the oracle's mean runs over its own
    views, hence the factor)."""
    announce("mapping normal grad 48x480x640")
    import torch
    from paper_2605_10760_amd import normal_loss_grad as gpu_grad
    rng = np.random.default_rng(45)
    V, H, W = 48, 480, 640
    depth, prior, intr = slanted_depth(rng, V, W, H, f=320.0)
    g = torch.zeros(depth.shape, device="cuda")
    gpu_grad(_t(depth), _t(prior), _t(intr), g, weight=1.0)
    torch.cuda.synchronize()
    for v in (0, 17, 47):
        ref = normal_loss_grad(depth[v:v + 1], np.moveaxis(prior[v:v + 1], 1, -1),
                               intr[v:v + 1]) / V
        got = g[v].cpu().numpy().astype(np.float64)
        np.testing.assert_allclose(got, ref[0], rtol=1e-3, atol=1e-4 * np.abs(ref).max())


@pytest.mark.parametrize("stride", [1, 3])
def test_seed_matches_oracle(stride):
    announce(f"mapping seed stride {stride}")
    from paper_2605_10760_amd import seed as gpu_seed
    rng = np.random.default_rng(50 + stride)
    H, W = 37, 53
    depth, _, intr = slanted_depth(rng, 1, W, H, f=40.0, hole_frac=0.05)
    depth = depth[0]
    depth[:4, :6] = 0.0      # a block of holes: some seeds lose every neighbour
    depth[10, 10] = -1.0     # negative depth is not seeded
    col = rng.random((3, H, W)).astype(np.float32)
    vm = look_at(np.array([0.3, -0.2, -1.0]), (0.0, 0.0, 1.0), 0.2).astype(np.float32)
    got = gpu_seed(_t(depth), _t(col), _t(vm), _t(intr[0]), stride=stride, opacity_logit=-1.5)
    ref = seed(depth, col, vm, intr[0], stride=stride, opacity_logit=np.float32(-1.5))
    assert got["means"].shape[0] == ref["means"].shape[0]
    g = {k: v.cpu().numpy() for k, v in got.items()}
    np.testing.assert_array_equal(g["colors"], ref["colors"].astype(np.float32))
    np.testing.assert_array_equal(g["opacity_logits"], np.float32(-1.5))
    np.testing.assert_array_equal(g["quats"], ref["quats"].astype(np.float32))
    np.testing.assert_allclose(g["means"], ref["means"], rtol=0, atol=2e-6 * np.abs(ref["means"]).max())
    np.testing.assert_allclose(g["log_scales"], ref["log_scales"], rtol=0, atol=2e-5)


def test_seed_full_size_sampled():
    """One 1200 x 680 keyframe (the paper's frame size), stride 1: the count
    against the valid pixels and sampled rows against the oracle on 3 x 3
    crops around their pixels (a seed reads only its four neighbours)."""
    announce("mapping seed 680x1200")
    from paper_2605_10760_amd import seed as gpu_seed
    rng = np.random.default_rng(60)
    H, W = 680, 1200
    depth, _, intr = slanted_depth(rng, 1, W, H, f=600.0, hole_frac=0.02)
    depth = depth[0]
    col = rng.random((3, H, W)).astype(np.float32)
    vm = look_at(np.array([1.0, 0.2, -2.0]), (0.0, 0.0, 0.5), 0.1).astype(np.float32)
    got = gpu_seed(_t(depth), _t(col), _t(vm), _t(intr[0]), stride=1, opacity_logit=0.0)
    valid = (depth > 0).ravel()
    assert got["means"].shape[0] == int(valid.sum())
    rows = np.cumsum(valid) - 1
    g = {k: v.cpu().numpy() for k, v in got.items()}
    for p in rng.choice(np.nonzero(valid)[0], 40, replace=False):
        j, i = divmod(int(p), W)
        j0, i0 = max(j - 1, 0), max(i - 1, 0)
        crop = depth[j0:j + 2, i0:i + 2]
        ci = intr[0].astype(np.float64).copy()
        ci[2] -= i0
        ci[3] -= j0
        r = seed(crop, col[:, j0:j + 2, i0:i + 2], vm, ci, stride=1)
        k = int(np.count_nonzero(crop.ravel()[:(j - j0) * crop.shape[1] + (i - i0)] > 0))
        q = rows[p]
        np.testing.assert_allclose(g["means"][q], r["means"][k], rtol=0, atol=1e-5)
        np.testing.assert_allclose(g["log_scales"][q], r["log_scales"][k], rtol=0, atol=2e-5)
        np.testing.assert_array_equal(g["colors"][q], col[:, j, i])


def test_seed_degenerate_inputs():
    """No valid depth seeds nothing; a stride beyond the image keeps only
    pixel (0, 0); a capacity below the count reports an overflow."""
    announce("mapping seed degenerate")
    import ctypes as C
    import torch
    from paper_2605_10760_amd import _lib, seed as gpu_seed
    H, W = 9, 11
    col = np.zeros((3, H, W), np.float32)
    vm = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(np.float32)
    intr = np.array([10.0, 10.0, 5.5, 4.5], np.float32)
    got = gpu_seed(_t(np.zeros((H, W), np.float32)), _t(col), _t(vm), _t(intr))
    assert got["means"].shape[0] == 0
    d = np.full((H, W), 2.0, np.float32)
    got = gpu_seed(_t(d), _t(col), _t(vm), _t(intr), stride=50)
    ref = seed(d, col, vm, intr, stride=50)
    assert got["means"].shape[0] == ref["means"].shape[0] == 1
    np.testing.assert_allclose(got["log_scales"].cpu().numpy(), ref["log_scales"], atol=2e-6)
    lib = _lib.load()
    dt, ct, vt, it = _t(d), _t(col), _t(vm), _t(intr)
    out = [torch.empty((4, k), device="cuda") for k in (3, 3, 4)]
    op, cl = torch.empty(4, device="cuda"), torch.empty((4, 3), device="cuda")
    n = C.c_int64()
    st = lib.gsr_seed(dt.data_ptr(), ct.data_ptr(), vt.data_ptr(), it.data_ptr(), W, H, 1, 0.0, 4,
                      out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), op.data_ptr(),
                      cl.data_ptr(), C.byref(n), None)
    torch.cuda.synchronize()
    assert st == _lib.GSR_E_OVERFLOW and n.value == H * W
    # the first four rows are still written
    ref = seed(d, col, vm, intr)
    np.testing.assert_allclose(out[0].cpu().numpy(), ref["means"][:4], atol=1e-6)
