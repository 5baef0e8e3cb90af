"""Pins of the oracle's SSIM term (Eq. (refine_loss)): identity and symmetry,
an explicit per-pixel window sum, and central differences of the gradient."""
import math

import numpy as np

from oracle.ssim import C1, C2, ssim, ssim_grad, ssim_term_grad, window_1d


def test_window_is_normalised_gaussian():
    w = window_1d()
    assert w.shape == (11,) and abs(w.sum() - 1) < 1e-15
    assert abs(w[5] / w[4] - math.exp(1 / (2 * 1.5 ** 2))) < 1e-12


def test_identity_and_symmetry():
    rng = np.random.default_rng(0)
    x = rng.random((2, 3, 13, 17))
    y = rng.random((2, 3, 13, 17))
    assert abs(ssim(x, x) - 1.0) < 1e-12
    assert abs(ssim(x, y) - ssim(y, x)) < 1e-14
    assert ssim(x, y) < 0.5


def test_matches_explicit_window_sum():
    """Brute force: every pixel's statistics as a direct sum over its 11 x 11
    neighbourhood inside the image."""
    rng = np.random.default_rng(1)
    H, W = 9, 12
    x = rng.random((1, 1, H, W))
    y = rng.random((1, 1, H, W))
    w = window_1d()
    tot = 0.0
    for i in range(H):
        for j in range(W):
            m = np.zeros(5)
            for di in range(-5, 6):
                for dj in range(-5, 6):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < H and 0 <= jj < W:
                        k = w[di + 5] * w[dj + 5]
                        a, b = x[0, 0, ii, jj], y[0, 0, ii, jj]
                        m += k * np.array([a, b, a * a, b * b, a * b])
            mx, my = m[0], m[1]
            sxx, syy, sxy = m[2] - mx * mx, m[3] - my * my, m[4] - mx * my
            tot += ((2 * mx * my + C1) * (2 * sxy + C2)
                    / ((mx * mx + my * my + C1) * (sxx + syy + C2)))
    assert abs(ssim(x, y) - tot / (H * W)) < 1e-13


def test_gradient_central_differences():
    rng = np.random.default_rng(2)
    x = rng.random((2, 3, 10, 14))
    y = rng.random((2, 3, 10, 14))
    g = ssim_grad(x, y)
    h = 1e-6
    for _ in range(25):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (ssim(xp, y) - ssim(xm, y)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * np.abs(g).max(), idx


def test_term_grad_chain_through_exposure():
    rng = np.random.default_rng(3)
    c = rng.random((2, 3, 8, 11))
    t = rng.random((2, 3, 8, 11))
    a = np.array([0.2, -0.1])
    b = np.array([0.05, -0.02])
    g = ssim_term_grad(c, t, a, b, 0.2)
    f = lambda c_, a_, b_: 0.2 * (1 - ssim(np.exp(a_)[:, None, None, None] * c_
                                           + b_[:, None, None, None], t))
    h = 1e-6
    for k in range(2):
        for key, arr in (("d_a", a), ("d_b", b)):
            p, m = arr.copy(), arr.copy()
            p[k] += h
            m[k] -= h
            fd = ((f(c, p, b) - f(c, m, b)) if key == "d_a" else (f(c, a, p) - f(c, a, m))) / (2 * h)
            assert abs(fd - g[key][k]) <= 1e-6 * max(abs(fd), 1e-6), key
    idx = (1, 2, 3, 4)
    cp, cm = c.copy(), c.copy()
    cp[idx] += h
    cm[idx] -= h
    fd = (f(cp, a, b) - f(cm, a, b)) / (2 * h)
    assert abs(fd - g["d_color"][idx]) <= 1e-6 * np.abs(g["d_color"]).max()
