"""Front-to-back alpha compositing of colour, depth and opacity (test
infrastructure only).

For one pixel with sample point x (pixel (i, j) is sampled at (i+0.5, j+0.5))
and an ordered list of splats (u, v, conic (A, B, C), opacity sigma, depth z,
colour c), walk the list front to back with transmittance T = 1:

  d = (u, v) - x;  power = -(A dx^2 + C dy^2)/2 - B dx dy
  skip the splat if power > 0
  alpha = min(0.99, sigma * exp(power));  skip it if alpha < 1/255
  T' = T (1 - alpha);  if T' < 1e-4 stop here, this splat not blended
  otherwise C += c alpha T,  D += z alpha T,  T = T',  last = position + 1

Outputs: colour C + T bg, depth D (not normalised by alpha), alpha 1 - T, and
the final T and last position.  The constants 0.99, 1/255 and 1e-4 are the
FP32 values of those decimals, used as exact numbers.  The number of list
entries examined, the stopping one included, is the evaluation count.

Two render modes share this per-pixel definition: `render_tiled` walks each
tile's sorted range; `render_brute` walks every visible Gaussian of the view
in (depth bits, index) order for every pixel.  The binning rule guarantees a
Gaussian left out of a tile has alpha < 1/255 on that tile's pixels, so the
two agree exactly in FP64 (the running products and sums are sequential, and
skipped splats multiply by exactly 1 and add exactly 0).
"""
from __future__ import annotations

import numpy as np

A_MAX = float(np.float32(0.99))
A_MIN = float(np.float32(1.0 / 255.0))
T_MIN = float(np.float32(1e-4))

# Decisions whose FP64 operand lies this close (relative) to its threshold
# are "ambiguous": an FP32 evaluation may legitimately take the other branch.
AMBIG_ALPHA = 2e-5
AMBIG_T = 2e-5


def composite(px, py, rec, order, bg, keep=False):
    """Composite pixels (sample points px, py [P]) against splats rec[order].

    rec: dict of FP64 arrays u, v, A, B, C, sigma, z, color[n,3].
    Returns dict color [P,3], depth, alpha, T_final, last, n_eval, ambiguous
    and, with keep=True, per-entry arrays for the backward pass.
    """
    px = np.asarray(px, np.float64)
    py = np.asarray(py, np.float64)
    P, L = px.shape[0], len(order)
    if L == 0:
        one = np.ones(P)
        out = dict(color=np.tile(np.asarray(bg, float), (P, 1)), depth=np.zeros(P),
                   alpha=np.zeros(P), T_final=one, last=np.zeros(P, np.int64),
                   n_eval=np.zeros(P, np.int64), ambiguous=np.zeros(P, bool))
        if keep:
            out.update(order=np.asarray(order, np.int64), w=np.zeros((P, 0)))
        return out
    order = np.asarray(order, np.int64)
    u, v = rec["u"][order], rec["v"][order]
    A, B, C = rec["A"][order], rec["B"][order], rec["C"][order]
    sig, z, col = rec["sigma"][order], rec["z"][order], rec["color"][order]
    dx = u[None, :] - px[:, None]
    dy = v[None, :] - py[:, None]
    power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
    G = np.exp(np.minimum(power, 0.0))
    raw = sig * G
    alpha = np.minimum(A_MAX, raw)
    skip = (power > 0) | (alpha < A_MIN)
    a_eff = np.where(skip, 0.0, alpha)
    T_after = np.cumprod(1.0 - a_eff, axis=1)
    T_before = np.concatenate([np.ones((P, 1)), T_after[:, :-1]], axis=1)
    stop_here = (~skip) & (T_after < T_MIN)
    has_stop = stop_here.any(axis=1)
    s = np.where(has_stop, np.argmax(stop_here, axis=1), L)
    pos = np.arange(L)[None, :]
    blended = (~skip) & (pos < s[:, None])
    w = np.where(blended, a_eff * T_before, 0.0)
    rows = np.arange(P)
    T_final = np.where(has_stop, T_before[rows, np.minimum(s, L - 1)], T_after[:, -1])
    Csum = np.stack([np.cumsum(w * col[None, :, k], axis=1)[:, -1] for k in range(3)], 1)
    Dsum = np.cumsum(w * z[None, :], axis=1)[:, -1]
    last = np.where(blended.any(axis=1), L - np.argmax(blended[:, ::-1], axis=1), 0)
    n_eval = np.where(has_stop, s + 1, L)
    examined = pos <= s[:, None]
    amb = examined & (np.abs(raw - A_MIN) <= AMBIG_ALPHA * A_MIN)
    amb |= examined & (power <= 0) & (np.abs(raw - A_MAX) <= AMBIG_ALPHA * A_MAX)
    amb |= examined & (~skip) & (np.abs(T_after - T_MIN) <= AMBIG_T * T_MIN)
    out = dict(color=Csum + T_final[:, None] * np.asarray(bg, float)[None, :],
               depth=Dsum, alpha=1.0 - T_final, T_final=T_final, last=last,
               n_eval=n_eval, ambiguous=amb.any(axis=1))
    if keep:
        clamped = raw > A_MAX
        out.update(order=order, w=w, blended=blended, alpha_e=a_eff,
                   T_before=T_before, G=G, clamped=clamped, dx=dx, dy=dy,
                   col=col, z=z, A=A, B=B, C=C, sig=sig)
    return out


def pixel_grid(x0, y0, x1, y1):
    """Pixel indices and sample points of the rectangle [x0,x1) x [y0,y1)."""
    yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    xx, yy = xx.ravel(), yy.ravel()
    return xx, yy, xx + 0.5, yy + 0.5


def composite_branches(x, y, rec, order, bg, band_alpha=AMBIG_ALPHA, band_t=AMBIG_T,
                       max_branches=64):
    """Every outcome of one pixel (sample point x, y) that an evaluation in
    another precision could legitimately reach.

    The walk is the one of composite(), entry by entry.  A decision whose FP64
    operand lies within the relative band of its threshold (the clamp at
    0.99, the skip at 1/255, the stop at 1e-4) is taken both ways, and each
    choice continues as its own branch.  Returns a list of dicts (color [3],
    depth, alpha, T_final, last, n_eval), one per branch; with no decision in
    a band it holds exactly composite()'s result for that pixel.
    """
    order = np.asarray(order, np.int64)
    bg = np.asarray(bg, float)
    L = order.shape[0]
    if L == 0:
        return [dict(color=bg.copy(), depth=0.0, alpha=0.0, T_final=1.0, last=0, n_eval=0)]
    # per-entry quantities with the same array expressions as composite()
    u, v = rec["u"][order], rec["v"][order]
    A, B, C = rec["A"][order], rec["B"][order], rec["C"][order]
    sig, z, col = rec["sigma"][order], rec["z"][order], rec["color"][order]
    dx = u[None, :] - np.array([[float(x)]])
    dy = v[None, :] - np.array([[float(y)]])
    power = (-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)[0]
    raw = (sig * np.exp(np.minimum(power, 0.0))[None, :])[0]
    out = []

    def finish(T, c, d, last, n_eval):
        out.append(dict(color=c + T * bg, depth=d, alpha=1.0 - T, T_final=T, last=last,
                        n_eval=n_eval))

    # explicit stack of partial walks: (position, T, colour, depth, last)
    stack = [(0, 1.0, np.zeros(3), 0.0, 0)]
    while stack:
        if len(out) + len(stack) > max_branches:
            raise RuntimeError("too many ambiguous decisions on one pixel")
        j, T, c, d, last = stack.pop()
        while True:
            if j == L:
                finish(T, c, d, last, L)
                break
            if power[j] > 0:
                j += 1
                continue
            # clamp: alpha = min(0.99, raw), both ways inside the band
            alphas = [min(A_MAX, raw[j])]
            if abs(raw[j] - A_MAX) <= band_alpha * A_MAX:
                alphas = [A_MAX, raw[j]]
            # skip: alpha < 1/255, both ways inside the band
            opts = []
            for a in alphas:
                if abs(raw[j] - A_MIN) <= band_alpha * A_MIN:
                    opts += [None, a]
                elif a < A_MIN:
                    opts.append(None)
                else:
                    opts.append(a)
            walks = []
            for a in opts:
                if a is None:
                    walks.append((j + 1, T, c, d, last, False))
                    continue
                Tn = T * (1.0 - a)
                stops = [Tn < T_MIN]
                if abs(Tn - T_MIN) <= band_t * T_MIN:
                    stops = [True, False]
                for s in stops:
                    if s:
                        walks.append((j, T, c, d, last, True))
                    else:
                        w = a * T
                        walks.append((j + 1, Tn, c + w * col[j], d + w * z[j], j + 1, False))
            # first option continues here, the others are pushed as branches
            for jj, TT, cc, dd, ll, stopped in walks[1:]:
                if stopped:
                    finish(TT, cc, dd, ll, jj + 1)
                else:
                    stack.append((jj, TT, cc, dd, ll))
            jj, TT, cc, dd, ll, stopped = walks[0]
            if stopped:
                finish(TT, cc, dd, ll, jj + 1)
                break
            j, T, c, d, last = jj, TT, cc, dd, ll
    return out
