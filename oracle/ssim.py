"""Structural-similarity term of the refinement loss and its gradient (test
infrastructure only).

Sec. III-C, Eq. (refine_loss) adds lambda (1 - SSIM(I~, I)), lambda = 0.2, on
the exposure-compensated render I~ = exp(a_k) I^ + b_k.  The paper does not
spell SSIM out; the reading here is the usual one (Wang et al. 2004, as used
by 3DGS): per colour channel, local statistics under an 11 x 11 Gaussian
window with standard deviation 1.5 (normalised), zero outside the image
("same"-size output), C1 = 0.01^2 and C2 = 0.03^2 for a dynamic range of 1,

  S = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
  mx = w*x, sxx = w*(x x) - mx^2, sxy = w*(x y) - mx my,

and SSIM is the mean of S over every pixel, channel and view.

Gradient (symmetric window, so sum_p w(p - q) f(p) = (w*f)(q)):
  d mean(S) / dx(q) = (1/N) [ (w*f1)(q) + 2 x(q) (w*f2)(q) + y(q) (w*f3)(q) ]
  f1 = dS/dmx - 2 mx dS/dsxx - my dS/dsxy,  f2 = dS/dsxx,  f3 = dS/dsxy,
  dS/dmx = 2 my A2/(B1 B2) - 2 mx S/B1,  dS/dsxx = -S/B2,  dS/dsxy = 2 A1/(B1 B2)
with A1, A2, B1, B2 the four factors of S.  Everything is FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.signal import convolve2d

C1 = 0.01 ** 2
C2 = 0.03 ** 2
RADIUS = 5
SIGMA = 1.5


def window_1d() -> np.ndarray:
    g = np.array([math.exp(-(i * i) / (2 * SIGMA * SIGMA)) for i in range(-RADIUS, RADIUS + 1)])
    return g / g.sum()


def _blur(img):
    w = window_1d()
    return convolve2d(img, np.outer(w, w), mode="same", boundary="fill", fillvalue=0.0)


def _stats(x, y):
    mx, my = _blur(x), _blur(y)
    sxx = _blur(x * x) - mx * mx
    syy = _blur(y * y) - my * my
    sxy = _blur(x * y) - mx * my
    a1 = 2 * mx * my + C1
    a2 = 2 * sxy + C2
    b1 = mx * mx + my * my + C1
    b2 = sxx + syy + C2
    return mx, my, a1, a2, b1, b2


def ssim(x, y):
    """Mean SSIM of images x, y [V,C,H,W] (FP64)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    tot = 0.0
    for v in range(x.shape[0]):
        for c in range(x.shape[1]):
            _, _, a1, a2, b1, b2 = _stats(x[v, c], y[v, c])
            tot += np.sum(a1 * a2 / (b1 * b2))
    return tot / x.size


def ssim_grad(x, y):
    """d mean SSIM / dx, same shape as x."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    g = np.empty_like(x)
    for v in range(x.shape[0]):
        for c in range(x.shape[1]):
            xx, yy = x[v, c], y[v, c]
            mx, my, a1, a2, b1, b2 = _stats(xx, yy)
            s = a1 * a2 / (b1 * b2)
            d_mx = 2 * my * a2 / (b1 * b2) - 2 * mx * s / b1
            d_sxx = -s / b2
            d_sxy = 2 * a1 / (b1 * b2)
            f1 = d_mx - 2 * mx * d_sxx - my * d_sxy
            g[v, c] = _blur(f1) + 2 * xx * _blur(d_sxx) + yy * _blur(d_sxy)
    return g / x.size


def ssim_term_grad(color, target, a, b, weight=0.2):
    """Gradient of weight (1 - SSIM(exp(a) I^ + b, I)) with respect to I^
    [V,3,H,W] and to the per-view exposure (a, b): dict d_color, d_a, d_b."""
    c = np.asarray(color, np.float64)
    ea = np.exp(np.asarray(a, np.float64))
    xt = ea[:, None, None, None] * c + np.asarray(b, np.float64)[:, None, None, None]
    g_t = -weight * ssim_grad(xt, target)
    return dict(d_color=ea[:, None, None, None] * g_t,
                d_a=ea * np.sum(g_t * c, axis=(1, 2, 3)),
                d_b=np.sum(g_t, axis=(1, 2, 3)))
