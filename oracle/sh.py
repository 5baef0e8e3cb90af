"""Real spherical harmonics up to degree 3 (test infrastructure only).

The fused map of Sec. III-C carries view-dependent colour; the colour model
used here is the 3DGS one: c = max(0, 0.5 + sum_lm Y_lm(d) k_lm) with d the
unit direction from the camera centre to the Gaussian mean.  Y_lm is the real
basis built from the complex harmonics *with* the Condon-Shortley phase:
Y_l0 = Y_l^0, Y_lm = sqrt(2) Re Y_l^m (m > 0), Y_lm = sqrt(2) Im Y_l^|m|
(m < 0); coefficient index l^2 + l + m.  Written out as polynomials of the
unit direction (x, y, z) with normalisation constants in closed form; the
test suite checks them against scipy's complex harmonics.
"""
from __future__ import annotations

import math

import numpy as np

PI = math.pi
K0 = 0.5 / math.sqrt(PI)
K1 = math.sqrt(3.0 / (4.0 * PI))
K2a = 0.5 * math.sqrt(15.0 / PI)
K2b = 0.25 * math.sqrt(5.0 / PI)
K2c = 0.25 * math.sqrt(15.0 / PI)
K3a = 0.25 * math.sqrt(35.0 / (2.0 * PI))
K3b = 0.5 * math.sqrt(105.0 / PI)
K3c = 0.25 * math.sqrt(21.0 / (2.0 * PI))
K3d = 0.25 * math.sqrt(7.0 / PI)
K3e = 0.25 * math.sqrt(105.0 / PI)


def sh_basis(d: np.ndarray, degree: int) -> np.ndarray:
    """Y[..., k] for k < (degree+1)^2 at unit directions d[..., 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [np.full_like(x, K0)]
    if degree >= 1:
        out += [-K1 * y, K1 * z, -K1 * x]
    if degree >= 2:
        out += [K2a * x * y, -K2a * y * z, K2b * (2 * z * z - x * x - y * y),
                -K2a * x * z, K2c * (x * x - y * y)]
    if degree >= 3:
        out += [-K3a * y * (3 * x * x - y * y), K3b * x * y * z,
                -K3c * y * (4 * z * z - x * x - y * y),
                K3d * z * (2 * z * z - 3 * x * x - 3 * y * y),
                -K3c * x * (4 * z * z - x * x - y * y),
                K3e * z * (x * x - y * y), -K3a * x * (x * x - 3 * y * y)]
    return np.stack(out, axis=-1)


def sh_basis_grad(d: np.ndarray, degree: int) -> np.ndarray:
    """dY[..., k, j] = partial Y_k / partial d_j of the polynomials above
    (treated as functions on R^3; callers project out the radial part)."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    zero = np.zeros_like(x)
    rows = [(zero, zero, zero)]
    if degree >= 1:
        rows += [(zero, -K1 + zero, zero), (zero, zero, K1 + zero),
                 (-K1 + zero, zero, zero)]
    if degree >= 2:
        rows += [(K2a * y, K2a * x, zero), (zero, -K2a * z, -K2a * y),
                 (-2 * K2b * x, -2 * K2b * y, 4 * K2b * z),
                 (-K2a * z, zero, -K2a * x), (2 * K2c * x, -2 * K2c * y, zero)]
    if degree >= 3:
        rows += [
            (-K3a * 6 * x * y, -K3a * (3 * x * x - 3 * y * y), zero),
            (K3b * y * z, K3b * x * z, K3b * x * y),
            (K3c * 2 * x * y, -K3c * (4 * z * z - x * x - 3 * y * y), -K3c * 8 * y * z),
            (-K3d * 6 * x * z, -K3d * 6 * y * z, K3d * (6 * z * z - 3 * x * x - 3 * y * y)),
            (-K3c * (4 * z * z - 3 * x * x - y * y), K3c * 2 * x * y, -K3c * 8 * x * z),
            (K3e * 2 * x * z, -K3e * 2 * y * z, K3e * (x * x - y * y)),
            (-K3a * (3 * x * x - 3 * y * y), K3a * 6 * x * y, zero),
        ]
    return np.stack([np.stack(r, axis=-1) for r in rows], axis=-2)
