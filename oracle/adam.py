"""Adam update of the optimisation drivers (test infrastructure only).

The paper minimises the mapping loss (Sec. III-A, Eq. (map_loss)) and the
refinement loss (Sec. III-C, Eq. (refine_loss)) by first-order steps with
per-parameter learning rates and gives no optimiser details; the reading is
Adam (Kingma & Ba 2015, Algorithm 1), the optimiser of 3DGS-style mapping:
with step t (counted from 1), gradient g and moments m, v (zero at t = 0),

  m <- beta1 m + (1 - beta1) g
  v <- beta2 v + (1 - beta2) g^2
  m^ = m / (1 - beta1^t),  v^ = v / (1 - beta2^t)
  p <- p - lr m^ / (sqrt(v^) + eps)

Everything is FP64.
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One update at step t; returns (p, m, v) as new FP64 arrays."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
