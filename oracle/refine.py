"""Refinement extras of the fused map (test infrastructure only): the
exposure-compensated render, the gradient of the L1 terms of the refinement
loss, and opacity pruning.

Sec. III-C: every keyframe k carries a log-gain and a bias (a_k, b_k), and
the refinement compares the exposure-compensated render
I~ = exp(a_k) I^ + b_k (the same scalars on every colour channel) with the
image, Eq. (refine_loss):  alpha' L1(I~, I) + lambda (1 - SSIM(I~, I))
+ beta L1(D^, D) + lambda_n' L_normal, alpha' = 1.75, lambda = 0.2, beta from
Eq. (map_loss) (0.25).  The L1 terms are means over every pixel and channel
of every view in the batch; their subgradient at 0 is 0.  Here: the L1 terms
only (SSIM and the normal term are not part of this module).  With
a = b = 0 and alpha' = 0.95 the same function is the gradient of the L1
terms of the mapping loss Eq. (map_loss).

The refinement prunes Gaussians whose opacity sigmoid(o) is below 0.005;
pruning keeps the survivors in their order, set by set.

Everything is FP64.
"""
from __future__ import annotations

import numpy as np


def exposure(color, a, b):
    """I~ = exp(a_k) I^ + b_k for color [V,3,H,W], a, b [V]."""
    c = np.asarray(color, np.float64)
    a = np.asarray(a, np.float64)[:, None, None, None]
    b = np.asarray(b, np.float64)[:, None, None, None]
    return np.exp(a) * c + b


def l1_loss(color, depth, target_color, target_depth, a, b, w_color, w_depth):
    """w_color * mean|I~ - I| + w_depth * mean|D^ - D|."""
    ic = exposure(color, a, b)
    return (w_color * np.mean(np.abs(ic - np.asarray(target_color, np.float64)))
            + w_depth * np.mean(np.abs(np.asarray(depth, np.float64)
                                       - np.asarray(target_depth, np.float64))))


def l1_loss_grad(color, depth, target_color, target_depth, a, b, w_color, w_depth):
    """Gradient of l1_loss: dict with d_color [V,3,H,W], d_depth [V,H,W],
    d_a [V], d_b [V] (chain rule through I~ = exp(a) I^ + b)."""
    c = np.asarray(color, np.float64)
    d = np.asarray(depth, np.float64)
    n_c, n_d = c.size, d.size
    g_tilde = w_color * np.sign(exposure(c, a, b) - np.asarray(target_color, np.float64)) / n_c
    ea = np.exp(np.asarray(a, np.float64))
    return dict(d_color=ea[:, None, None, None] * g_tilde,
                d_depth=w_depth * np.sign(d - np.asarray(target_depth, np.float64)) / n_d,
                d_a=ea * np.sum(c * g_tilde, axis=(1, 2, 3)),
                d_b=np.sum(g_tilde, axis=(1, 2, 3)))


def prune(opacity_logits, set_offsets, min_opacity=0.005):
    """Indices of the Gaussians with sigmoid(o) >= min_opacity, in order, and
    the set offsets of the pruned scene.  sigmoid is increasing, so the test
    is o >= logit(min_opacity), evaluated on the FP32 logits."""
    o = np.asarray(opacity_logits, np.float64)
    keep = o >= np.log(min_opacity / (1.0 - min_opacity))
    idx = np.nonzero(keep)[0]
    offs = np.asarray(set_offsets, np.int64)
    new_offs = np.array([np.count_nonzero(keep[:e]) for e in offs], np.int64)
    return idx, new_offs
