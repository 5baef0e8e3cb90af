"""Pins of the oracle's Adam update (the optimiser reading of the mapping
and refinement steps, Kingma & Ba 2015 Algorithm 1)."""
import numpy as np

from oracle.adam import adam_step


def test_adam_matches_torch_reference():
    """Several steps against torch.optim.Adam (an independent implementation)
    in float64 on the CPU, with changing gradients."""
    import torch
    rng = np.random.default_rng(0)
    n = 257
    p0 = rng.normal(size=n)
    p = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.8, 0.95), eps=1e-6)
    q, m, v = p0.copy(), np.zeros(n), np.zeros(n)
    for t in range(1, 8):
        g = rng.normal(size=n) * (0.1 + t)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        q, m, v = adam_step(q, g, m, v, t, 3e-3, 0.8, 0.95, 1e-6)
        np.testing.assert_allclose(q, p.detach().numpy(), rtol=0, atol=1e-15)


def test_adam_constant_gradient_closed_form():
    """With the same gradient every step the bias-corrected moments equal g
    and g^2 exactly, so every step moves by lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    g = rng.normal(size=100)
    g[:5] = 0.0
    q, m, v = np.zeros(100), np.zeros(100), np.zeros(100)
    lr, eps = 0.01, 1e-8
    for t in range(1, 30):
        q_prev = q
        q, m, v = adam_step(q, g, m, v, t, lr, 0.9, 0.999, eps)
        np.testing.assert_allclose(q_prev - q, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)
    assert np.all(q[:5] == 0.0)


def test_adam_first_step_is_sign_step():
    """At t = 1 from zero moments the update is lr g / (|g| + eps): the sign
    of the gradient scaled by lr, whatever its magnitude."""
    g = np.array([1e-3, -5.0, 2e4, -1e-12])
    q, _, _ = adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.5, 0.9, 0.999, 1e-15)
    np.testing.assert_allclose(q, -0.5 * np.sign(g), rtol=1e-3)
