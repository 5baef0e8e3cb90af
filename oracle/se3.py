"""SE(3) exponential and the left update of a world-to-camera pose (test
infrastructure only).

Sec. III-C refines per-keyframe pose deltas delta_xi_k jointly with the
Gaussians.  A delta xi = (rho, phi) (translation part first) acts on the
left: [R|t] <- Exp(xi) [R|t], where Exp(xi) = [[Exp_SO3(phi), V(phi) rho],
[0, 1]], Exp_SO3 is Rodrigues' formula and
V = I + (1 - cos th)/th^2 [phi]x + (th - sin th)/th^3 [phi]x^2, th = |phi|.
"""
from __future__ import annotations

import numpy as np


def _skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def exp_se3(xi: np.ndarray) -> np.ndarray:
    """4x4 matrix Exp(xi), xi = (rho, phi)."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    th = float(np.linalg.norm(phi))
    K = _skew(phi)
    if th < 1e-8:
        # second-order series; the FP64 error is far below 1e-16 here
        Rm = np.eye(3) + K + 0.5 * K @ K
        Vm = np.eye(3) + 0.5 * K + K @ K / 6.0
    else:
        Rm = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K
        Vm = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K
    T = np.eye(4)
    T[:3, :3] = Rm
    T[:3, 3] = Vm @ rho
    return T


def apply_left(xi: np.ndarray, viewmat: np.ndarray) -> np.ndarray:
    """Exp(xi) @ [viewmat; 0 0 0 1], returned as 3x4."""
    T = np.eye(4)
    T[:3, :] = np.asarray(viewmat, np.float64).reshape(3, 4)
    return (exp_se3(xi) @ T)[:3, :]
