"""GPU parity of the refinement extras (Sec. III-C, Eq. (refine_loss)):
exposure-compensated L1 gradient and opacity pruning, through the C ABI,
against the oracle."""
import numpy as np
import pytest

from gpu_harness import announce
from oracle.refine import exposure, l1_loss_grad, prune
from synth.scenes import multi_agent

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("H,W", [(37, 53), (40, 52)])
def test_l1_loss_grad_matches_oracle(H, W):
    """37 x 53: ragged, one pixel at a time; 40 x 52: four pixels per load."""
    announce(f"refine l1 grad {H}x{W}")
    import torch
    from paper_2605_10760_amd import l1_loss_grad as gpu_grad
    rng = np.random.default_rng(7)
    V = 3
    c = rng.random((V, 3, H, W)).astype(np.float32)
    d = (0.5 + 3 * rng.random((V, H, W))).astype(np.float32)
    tc = rng.random((V, 3, H, W)).astype(np.float32)
    td = (0.5 + 3 * rng.random((V, H, W))).astype(np.float32)
    tc[0, 0, :2] = c[0, 0, :2]  # exact zeros of the residual: subgradient 0
    ex = np.stack([rng.normal(0, 0.3, V), rng.normal(0, 0.1, V)], 1).astype(np.float32)
    t = lambda a: torch.from_numpy(a).cuda()
    for expo in (None, ex):
        a = np.zeros(V) if expo is None else expo[:, 0]
        b = np.zeros(V) if expo is None else expo[:, 1]
        got = gpu_grad(t(c), t(tc), t(d), t(td), None if expo is None else t(expo), 1.75, 0.25)
        torch.cuda.synchronize()
        ref = l1_loss_grad(c, d, tc, td, a, b, 1.75, 0.25)
        # residuals the FP32 and FP64 evaluations could sign differently
        resid = exposure(c, a, b) - tc
        amb = (np.abs(resid) < 1e-5) & (resid != 0)
        gc = got["d_color"].cpu().numpy()
        np.testing.assert_allclose(gc[~amb], ref["d_color"][~amb], rtol=1e-6, atol=0)
        np.testing.assert_allclose(got["d_depth"].cpu().numpy(), ref["d_depth"], rtol=1e-6, atol=0)
        if expo is not None:
            ge = got["d_exposure"].cpu().numpy()
            scale = np.abs(ref["d_color"]).max() * c[0].size
            np.testing.assert_allclose(ge[:, 0], ref["d_a"], atol=1e-5 * scale)
            np.testing.assert_allclose(ge[:, 1], ref["d_b"], atol=1e-5 * scale)
            assert amb.sum() < 20


def test_prune_matches_oracle():
    announce("refine prune")
    import torch
    from paper_2605_10760_amd import SceneTensors, prune as gpu_prune
    wl = multi_agent(scale=0.01, keyframes=1)
    sc = wl.scene
    rng = np.random.default_rng(8)
    o = sc.opacity_logits.copy()
    o[rng.random(o.shape[0]) < 0.3] = -6.0  # sigmoid = 0.0025: pruned
    # logits at and next to logit(0.005) = -5.2933048...
    o[::97] = np.float32(-5.2933048)
    o[1::97] = np.nextafter(np.float32(-5.2933048), np.float32(0))
    o[2::97] = np.nextafter(np.float32(-5.2933048), np.float32(-10))
    sc.opacity_logits = o
    st_ = SceneTensors.from_numpy(sc)
    out = gpu_prune(st_, 0.005)
    idx, offs = prune(o, sc.set_offsets, 0.005)
    np.testing.assert_array_equal(out.set_offsets, offs)
    np.testing.assert_array_equal(out.means.cpu().numpy(), sc.means[idx])
    np.testing.assert_array_equal(out.log_scales.cpu().numpy(), sc.log_scales[idx])
    np.testing.assert_array_equal(out.quats.cpu().numpy(), sc.quats[idx])
    np.testing.assert_array_equal(out.opacity_logits.cpu().numpy(), o[idx])
    np.testing.assert_array_equal(out.colors.cpu().numpy(), sc.colors[idx])
    assert 0 < idx.shape[0] < o.shape[0]


@pytest.mark.parametrize("V,H,W", [(2, 37, 45), (2, 150, 70)])
def test_ssim_grad_matches_oracle(V, H, W):
    """Ragged tiles in both directions (16 x 64 output tiles, 5-pixel halo)."""
    announce(f"refine ssim {V}x{H}x{W}")
    import torch
    from oracle.ssim import ssim, ssim_term_grad
    from paper_2605_10760_amd import ssim_grad
    rng = np.random.default_rng(9)
    c = rng.random((V, 3, H, W)).astype(np.float32)
    tgt = np.clip(c + 0.1 * rng.normal(size=c.shape), 0, 1).astype(np.float32)
    ex = np.array([[0.15, 0.02], [-0.1, -0.03]], np.float32)
    t = lambda a: torch.from_numpy(a).cuda()
    # accumulated onto: small enough that the FP32 sum keeps the gradient digits
    base = (1e-4 * rng.normal(size=c.shape)).astype(np.float32)
    d_color = t(base.copy())
    d_exp = t(np.array([[1.0, 2.0], [3.0, 4.0]], np.float32))
    out = torch.zeros(1, device="cuda")
    ssim_grad(t(c), t(tgt), d_color, t(ex), d_exp, 0.2, ssim_out=out)
    torch.cuda.synchronize()
    ref = ssim_term_grad(c, tgt, ex[:, 0], ex[:, 1], 0.2)
    xt = np.exp(ex[:, 0])[:, None, None, None] * c + ex[:, 1][:, None, None, None]
    assert abs(out.item() - ssim(xt, tgt)) <= 2e-5
    got = d_color.cpu().numpy() - base
    scale = np.abs(ref["d_color"]).max()
    assert np.abs(got - ref["d_color"]).max() <= 1e-3 * scale
    ge = d_exp.cpu().numpy() - np.array([[1.0, 2.0], [3.0, 4.0]])
    sa = np.abs(ref["d_a"]).max()
    np.testing.assert_allclose(ge[:, 0], ref["d_a"], atol=1e-3 * sa)
    np.testing.assert_allclose(ge[:, 1], ref["d_b"], atol=1e-3 * np.abs(ref["d_b"]).max())


def test_ssim_grad_full_size_sampled():
    """The refinement batch's size, 48 views x 3 x 480 x 640: the gradient and
    exposure gradients of three sampled views against the oracle (the window
    stays inside a view, so a view's gradient is the one-view oracle's scaled
    by 1/48), and the batch's mean SSIM against the mean of the 48 one-view
    means the kernel reports."""
    V, H, W = 48, 480, 640
    announce(f"refine ssim full size {V}x3x{H}x{W}")
    import torch
    from oracle.ssim import ssim, ssim_term_grad
    from paper_2605_10760_amd import ssim_grad
    rng = np.random.default_rng(12)
    c = rng.random((V, 3, H, W), dtype=np.float32)
    tgt = np.clip(c + 0.08 * rng.standard_normal(c.shape, dtype=np.float32), 0, 1)
    ex = np.stack([rng.normal(0, 0.1, V), rng.normal(0, 0.02, V)], 1).astype(np.float32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    d_color = torch.zeros((V, 3, H, W), device="cuda")
    d_exp = torch.zeros((V, 2), device="cuda")
    out = torch.zeros(1, device="cuda")
    ct, tt, et = t(c), t(tgt), t(ex)
    ssim_grad(ct, tt, d_color, et, d_exp, 0.2, ssim_out=out)
    torch.cuda.synchronize()
    per_view = []
    one = torch.zeros(1, device="cuda")
    for v in range(V):
        ssim_grad(ct[v:v + 1], tt[v:v + 1], torch.zeros((1, 3, H, W), device="cuda"), et[v:v + 1],
                  None, 0.2, ssim_out=one)
        per_view.append(one.item())
    assert abs(out.item() - float(np.mean(per_view))) <= 1e-5
    g = d_color.cpu().numpy()
    ge = d_exp.cpu().numpy()
    for v in (0, 23, 47):
        ref = ssim_term_grad(c[v:v + 1], tgt[v:v + 1], ex[v:v + 1, 0], ex[v:v + 1, 1], 0.2)
        xt = np.exp(ex[v, 0]) * c[v:v + 1].astype(np.float64) + ex[v, 1]
        assert abs(per_view[v] - ssim(xt, tgt[v:v + 1])) <= 2e-5
        want = ref["d_color"][0] / V
        assert np.abs(g[v] - want).max() <= 1e-3 * np.abs(want).max(), v
        np.testing.assert_allclose(ge[v, 0], ref["d_a"][0] / V, rtol=1e-3,
                                   atol=1e-4 * abs(ref["d_a"][0] / V))
        np.testing.assert_allclose(ge[v, 1], ref["d_b"][0] / V, rtol=1e-3,
                                   atol=1e-4 * abs(ref["d_b"][0] / V))
