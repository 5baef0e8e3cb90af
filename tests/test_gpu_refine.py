"""GPU parity of the refinement extras (Sec. III-C, Eq. (refine_loss)):
exposure-compensated L1 gradient and opacity pruning, through the C ABI,
against the oracle."""
import numpy as np
import pytest

from gpu_harness import announce
from oracle.refine import exposure, l1_loss_grad, prune
from synth.scenes import multi_agent

pytestmark = pytest.mark.gpu


def test_l1_loss_grad_matches_oracle():
    announce("refine l1 grad")
    import torch
    from paper_2605_10760_amd import l1_loss_grad as gpu_grad
    rng = np.random.default_rng(7)
    V, H, W = 3, 37, 53  # ragged: not a multiple of the 256-pixel blocks
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
