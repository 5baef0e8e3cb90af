"""GPU checks of the optimisation drivers (Sec. III-A Eq. (map_loss),
Sec. III-C Eq. (refine_loss)): one step's gradients against the oracle's
chain (render, loss-term gradients, render backward), and convergence of the
exposure and pose parameters on targets rendered at known values."""
import numpy as np
import pytest

from gpu_harness import announce
from synth.scenes import F32, Views, look_at, tiny_scene

pytestmark = pytest.mark.gpu


def _two_views(seed):
    sc, vw = tiny_scene(seed, n=40, width=48, height=32)
    vm2 = look_at(np.array([0.15, -0.1, 0.0]), (0.05, 0.0, 3.0), 0.0).astype(F32)
    views = Views(np.stack([vw.viewmats[0], vm2]), np.repeat(vw.intrinsics, 2, 0),
                  np.zeros(2, np.int32), 48, 32)
    return sc, views


def _close(got, ref, name):
    """Per tensor: max and 2-norm of the error within 1e-3 of the reference's."""
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max() + 1e-12, name
    assert np.linalg.norm(got - ref) <= 1e-3 * np.linalg.norm(ref) + 1e-12, name


@pytest.mark.parametrize("mode", ["refine", "map"])
def test_step_gradients_match_oracle_chain(mode):
    announce(f"optim gradients {mode}")
    import torch
    from oracle.mapping import iso_loss_grad, normal_loss_grad
    from oracle.refine import l1_loss_grad
    from oracle.render import Settings, render_backward, render_view
    from oracle.ssim import ssim_term_grad
    from paper_2605_10760_amd import (MAP_WEIGHTS, REFINE_WEIGHTS, Optimizer, Rasterizer,
                                      SceneTensors, ViewTensors)
    sc, views = _two_views(22)
    rng = np.random.default_rng(5)
    V, H, W = 2, 32, 48
    tc = rng.random((V, 3, H, W)).astype(F32)
    td = (1.5 + 2 * rng.random((V, H, W))).astype(F32)
    pr = np.stack([rng.normal(0, 0.3, (V, H, W)), rng.normal(0, 0.3, (V, H, W)),
                   -np.ones((V, H, W))], 1)
    pr = (pr / np.linalg.norm(pr, axis=1, keepdims=True)).astype(F32)
    w = REFINE_WEIGHTS if mode == "refine" else MAP_WEIGHTS
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st, vt = SceneTensors.from_numpy(sc), ViewTensors.from_numpy(views)
    rast = Rasterizer(W, H, 2 * sc.n, 2)
    opt = Optimizer(rast, st, vt, t(tc), t(td), t(pr), w, pose=True, exposure=mode == "refine")
    g = {k: (None if v is None else v.cpu().numpy()) for k, v in opt.gradients().items()}
    # the oracle's chain at a = b = 0
    color = np.zeros((V, 3, H, W))
    depth = np.zeros((V, H, W))
    for k in range(V):
        rv = render_view(sc, views, k, Settings())
        assert not rv["ambiguous"].any()
        color[k], depth[k] = rv["color"], rv["depth"]
    zero = np.zeros(V)
    lg = l1_loss_grad(color, depth, tc, td, zero, zero, w.color, w.depth)
    d_color, d_depth = lg["d_color"], lg["d_depth"]
    d_a, d_b = lg["d_a"], lg["d_b"]
    if w.ssim:
        sg = ssim_term_grad(color, tc, zero, zero, w.ssim)
        d_color = d_color + sg["d_color"]
        d_a, d_b = d_a + sg["d_a"], d_b + sg["d_b"]
    d_depth = d_depth + w.normal * normal_loss_grad(depth, np.moveaxis(pr, 1, -1),
                                                    views.intrinsics)
    ref = render_backward(sc, views, d_color, d_depth, None)
    if w.iso:
        ref["d_log_scales"] = ref["d_log_scales"] + w.iso * iso_loss_grad(sc.log_scales)
    for k_gpu, k_ref in [("d_means", "d_means"), ("d_log_scales", "d_log_scales"),
                         ("d_quats", "d_quats"), ("d_opacity_logits", "d_opacity"),
                         ("d_colors", "d_colors"), ("d_pose", "d_pose")]:
        _close(g[k_gpu], ref[k_ref], k_gpu)
    if mode == "refine":
        _close(g["d_exposure"][:, 0], d_a, "d_a")
        _close(g["d_exposure"][:, 1], d_b, "d_b")


def test_exposure_recovered():
    """Targets rendered from the scene itself, then exp(a*) I + b*; with the
    Gaussians held still (zero rates) the refinement loss is minimised at
    (a*, b*)."""
    announce("optim exposure recovery")
    import torch
    from paper_2605_10760_amd import (REFINE_WEIGHTS, Optimizer, Rasterizer, Rates,
                                      SceneTensors, ViewTensors)
    sc, views = _two_views(22)
    st, vt = SceneTensors.from_numpy(sc), ViewTensors.from_numpy(views)
    rast = Rasterizer(48, 32, 2 * sc.n, 2)
    c, d, _, _ = rast.forward(st, vt)
    a_true = torch.tensor([0.2, -0.15], device="cuda")
    b_true = torch.tensor([-0.05, 0.03], device="cuda")
    tc = torch.exp(a_true)[:, None, None, None] * c + b_true[:, None, None, None]
    rates = Rates(0.0, 0.0, 0.0, 0.0, 0.0, pose=0.0, exposure=1e-2)
    opt = Optimizer(rast, st, vt, tc.contiguous(), d.clone(), None, REFINE_WEIGHTS, rates,
                    exposure=True)
    for _ in range(400):
        opt.step()
    torch.cuda.synchronize()
    e = opt.exposure.cpu().numpy()
    np.testing.assert_allclose(e[:, 0], a_true.cpu().numpy(), atol=0.03)
    np.testing.assert_allclose(e[:, 1], b_true.cpu().numpy(), atol=0.02)


def test_pose_refinement_reduces_loss():
    """Targets rendered at slightly moved cameras; refining the pose deltas
    alone brings the render back toward them."""
    announce("optim pose refinement")
    import torch
    from paper_2605_10760_amd import (REFINE_WEIGHTS, Optimizer, Rasterizer, Rates,
                                      SceneTensors, ViewTensors, apply_pose_delta)
    sc, views = _two_views(22)
    st, vt = SceneTensors.from_numpy(sc), ViewTensors.from_numpy(views)
    rast = Rasterizer(48, 32, 2 * sc.n, 2)
    xi = torch.tensor([[0.01, -0.008, 0.012, 0.006, -0.004, 0.005],
                       [-0.009, 0.007, -0.01, -0.005, 0.006, -0.004]], device="cuda")
    vt_true = ViewTensors(apply_pose_delta(vt.viewmats, xi), vt.intrinsics, vt.view_set, 48, 32)
    tc, td, _, _ = rast.forward(st, vt_true)
    tc, td = tc.clone(), td.clone()
    rates = Rates(0.0, 0.0, 0.0, 0.0, 0.0, pose=2e-3, exposure=0.0)
    opt = Optimizer(rast, st, vt, tc, td, None, REFINE_WEIGHTS, rates, pose=True)

    def l1():
        c, d, _, _ = rast.forward(st, opt.views)
        return float((c - tc).abs().mean() + (d - td).abs().mean())

    before = l1()
    for _ in range(150):
        opt.step()
    after = l1()
    assert after < 0.5 * before, (before, after)


def test_refine_driver_prunes():
    announce("optim refine driver")
    import torch
    from paper_2605_10760_amd import Rasterizer, SceneTensors, ViewTensors, refine
    sc, views = _two_views(22)
    o = sc.opacity_logits.copy()
    o[:5] = -8.0  # opacity 3e-4: pruned after refinement
    sc.opacity_logits = o
    st, vt = SceneTensors.from_numpy(sc), ViewTensors.from_numpy(views)
    rast = Rasterizer(48, 32, 2 * sc.n, 2)
    c, d, _, _ = rast.forward(st, vt)
    pruned, vm, ex = refine(rast, st, vt, c.clone(), d.clone(), iters=10)
    torch.cuda.synchronize()
    assert pruned.n <= sc.n - 5 and vm.shape == (2, 3, 4) and ex.shape == (2, 2)
    assert torch.isfinite(pruned.means).all() and torch.isfinite(vm).all()
