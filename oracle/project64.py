"""FP64 projection of 3D Gaussians to screen-space splats, and its exact
derivative (test infrastructure only).

A Gaussian has mean mu, scale vector s and rotation R (Sec. III-C, Eq.
(gauss_update), lists mean, covariance, scale, opacity and colour), with
covariance Sigma = R diag(s)^2 R^T (the 3DGS factorisation).  A world-to-
camera pose [Rc | tc] (Sec. III-B) and pinhole intrinsics (Appendix A) map it
to the image by the EWA local-affine approximation: the camera-space mean
p = Rc mu + tc projects to (u, v) = (fx px/pz + cx, fy py/pz + cy), and the
covariance maps through the Jacobian J of the perspective division,
Sigma2 = J Rc Sigma Rc^T J^T + 0.3 I (a 0.3 px^2 low-pass dilation).  The
Jacobian's x/z and y/z ratios are clamped to 1.3 times the half field of view
(a guard band that keeps far-off-screen splats bounded).  Opacity is
sigmoid(o), colours are raw RGB (degree 0) or spherical harmonics evaluated at
the viewing direction.

Everything here is evaluated in FP64 from FP32 inputs, written in plain
matrix form; which Gaussians are kept is decided by the FP32 key path.
"""
from __future__ import annotations

import numpy as np

from .sh import sh_basis, sh_basis_grad

D = np.float64
BLUR = 0.3
GUARD = 1.3


def quat_to_rot(qhat: np.ndarray) -> np.ndarray:
    """Rotation matrices [n,3,3] of unit quaternions (w, x, y, z)."""
    w, x, y, z = qhat[:, 0], qhat[:, 1], qhat[:, 2], qhat[:, 3]
    R = np.empty((qhat.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def quat_rot_derivs(qhat: np.ndarray) -> np.ndarray:
    """dR/dq_c for c in (w,x,y,z): array [n,4,3,3] (linear in q)."""
    w, x, y, z = qhat[:, 0], qhat[:, 1], qhat[:, 2], qhat[:, 3]
    o = np.zeros_like(w)
    dw = np.stack([np.stack([o, -z, y], -1), np.stack([z, o, -x], -1),
                   np.stack([-y, x, o], -1)], -2)
    dx = np.stack([np.stack([o, y, z], -1), np.stack([y, -2 * x, -w], -1),
                   np.stack([z, w, -2 * x], -1)], -2)
    dy = np.stack([np.stack([-2 * y, x, w], -1), np.stack([x, o, z], -1),
                   np.stack([-w, z, -2 * y], -1)], -2)
    dz = np.stack([np.stack([-2 * z, -w, x], -1), np.stack([w, -2 * z, y], -1),
                   np.stack([x, y, o], -1)], -2)
    return 2.0 * np.stack([dw, dx, dy, dz], axis=1)


def skew(v: np.ndarray) -> np.ndarray:
    """[v]x for v [...,3]."""
    o = np.zeros_like(v[..., 0])
    return np.stack([np.stack([o, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], o, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], o], -1)], -2)


def project(means, log_scales, quats, opacity_logits, colors, sh_degree,
            viewmat, intrin, width, height):
    """Project the given Gaussians (already restricted to the visible ones)
    into one view.  Returns a dict of FP64 arrays."""
    m = np.asarray(means, D)
    vm = np.asarray(viewmat, D).reshape(3, 4)
    Rc, tc = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = np.asarray(intrin, D)
    p = m @ Rc.T + tc
    s = np.exp(np.asarray(log_scales, D))
    q = np.asarray(quats, D)
    qn = np.linalg.norm(q, axis=1)
    qhat = q / qn[:, None]
    R = quat_to_rot(qhat)
    M = R * s[:, None, :]
    S3 = M @ np.swapaxes(M, 1, 2)
    Scam = Rc @ S3 @ Rc.T
    rx = p[:, 0] / p[:, 2]
    ry = p[:, 1] / p[:, 2]
    limx = GUARD * (0.5 * width) / fx
    limy = GUARD * (0.5 * height) / fy
    rxc = np.clip(rx, -limx, limx)
    ryc = np.clip(ry, -limy, limy)
    z = p[:, 2]
    J = np.zeros((m.shape[0], 2, 3))
    J[:, 0, 0] = fx / z
    J[:, 0, 2] = -fx * rxc / z
    J[:, 1, 1] = fy / z
    J[:, 1, 2] = -fy * ryc / z
    S2 = J @ Scam @ np.swapaxes(J, 1, 2) + BLUR * np.eye(2)
    a, b, c = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = a * c - b * b
    conic = np.stack([c / det, -b / det, a / det], axis=1)
    u = fx * rx + cx
    v = fy * ry + cy
    sigma = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, D)))
    out = dict(p=p, s=s, qhat=qhat, qn=qn, R=R, M=M, S3=S3, Scam=Scam, J=J,
               S2=S2, conic=conic, u=u, v=v, z=z, sigma=sigma, Rc=Rc, tc=tc,
               fx=fx, fy=fy, rx=rx, ry=ry, limx=limx, limy=limy)
    k = np.asarray(colors, D)
    if sh_degree == 0:
        out["color"] = k.reshape(-1, 3)
    else:
        cam = -Rc.T @ tc
        dvec = m - cam
        r = np.linalg.norm(dvec, axis=1)
        dirs = dvec / r[:, None]
        nb = (sh_degree + 1) ** 2
        Y = sh_basis(dirs, sh_degree)                  # [n,nb]
        raw = 0.5 + np.einsum("nk,nkc->nc", Y, k[:, :nb, :])
        out.update(color=np.maximum(raw, 0.0), color_raw=raw, dirs=dirs,
                   dist=r, Y=Y)
    return out


def project_backward(pr, g_u, g_v, g_conic, g_sigma, g_color, g_z, colors,
                     sh_degree):
    """Chain rule from screen-space splat gradients to the Gaussian
    parameters of one view, plus that view's pose gradient.

    Inputs are per-Gaussian FP64 arrays (g_conic [n,3] = dL/d(A,B,C)).
    Returns dict with d_means, d_log_scales, d_quats, d_opacity, d_colors and
    d_pose (rho then phi, left perturbation of the world-to-camera pose).
    """
    n = pr["p"].shape[0]
    Q = np.stack([np.stack([pr["conic"][:, 0], pr["conic"][:, 1]], -1),
                  np.stack([pr["conic"][:, 1], pr["conic"][:, 2]], -1)], -2)
    GQ = np.stack([np.stack([g_conic[:, 0], 0.5 * g_conic[:, 1]], -1),
                   np.stack([0.5 * g_conic[:, 1], g_conic[:, 2]], -1)], -2)
    # conic = S2^{-1}:  dL/dS2 = -Q GQ Q
    GS2 = -Q @ GQ @ Q
    J, Scam, p = pr["J"], pr["Scam"], pr["p"]
    GScam = np.swapaxes(J, 1, 2) @ GS2 @ J
    GJ = 2.0 * GS2 @ J @ Scam                       # [n,2,3]
    fx, fy = pr["fx"], pr["fy"]
    px, py, z = p[:, 0], p[:, 1], p[:, 2]
    gp = np.zeros((n, 3))
    # (u, v) = (fx px/z + cx, fy py/z + cy)
    gp[:, 0] += g_u * fx / z
    gp[:, 1] += g_v * fy / z
    gp[:, 2] += -g_u * fx * px / z ** 2 - g_v * fy * py / z ** 2
    gp[:, 2] += g_z
    # J entries: J00 = fx/z, J11 = fy/z, J02 = -fx rxc/z, J12 = -fy ryc/z
    gp[:, 2] += -GJ[:, 0, 0] * fx / z ** 2 - GJ[:, 1, 1] * fy / z ** 2
    inx = np.abs(pr["rx"]) <= pr["limx"]
    iny = np.abs(pr["ry"]) <= pr["limy"]
    rxc = np.clip(pr["rx"], -pr["limx"], pr["limx"])
    ryc = np.clip(pr["ry"], -pr["limy"], pr["limy"])
    # d(rxc)/dpx = 1/z and d(rxc)/dz = -px/z^2 when not clamped, else 0
    gp[:, 0] += np.where(inx, GJ[:, 0, 2] * (-fx / z ** 2), 0.0)
    gp[:, 2] += GJ[:, 0, 2] * (fx * rxc / z ** 2)
    gp[:, 2] += np.where(inx, GJ[:, 0, 2] * (fx * px / z ** 3), 0.0)
    gp[:, 1] += np.where(iny, GJ[:, 1, 2] * (-fy / z ** 2), 0.0)
    gp[:, 2] += GJ[:, 1, 2] * (fy * ryc / z ** 2)
    gp[:, 2] += np.where(iny, GJ[:, 1, 2] * (fy * py / z ** 3), 0.0)

    Rc = pr["Rc"]
    g_means = gp @ Rc                                 # Rc^T gp, row-wise
    GS3 = Rc.T @ GScam @ Rc
    M, R, s = pr["M"], pr["R"], pr["s"]
    GM = 2.0 * GS3 @ M
    g_s = np.einsum("nik,nik->nk", GM, R)
    g_log_scales = g_s * s
    GR = GM * s[:, None, :]
    dR = quat_rot_derivs(pr["qhat"])
    g_qhat = np.einsum("nij,ncij->nc", GR, dR)
    qhat = pr["qhat"]
    g_quats = (g_qhat - qhat * np.sum(qhat * g_qhat, axis=1, keepdims=True)) \
        / pr["qn"][:, None]
    sig = pr["sigma"]
    g_opacity = g_sigma * sig * (1.0 - sig)

    g_mu_dir = np.zeros((n, 3))
    if sh_degree == 0:
        g_colors = g_color.copy()
    else:
        nb = (sh_degree + 1) ** 2
        k = np.asarray(colors, D)[:, :nb, :]
        gc = np.where(pr["color_raw"] > 0.0, g_color, 0.0)    # max(0, .) mask
        g_colors = np.zeros((n, np.asarray(colors).shape[1], 3))
        g_colors[:, :nb, :] = pr["Y"][:, :, None] * gc[:, None, :]
        dY = sh_basis_grad(pr["dirs"], sh_degree)             # [n,nb,3]
        g_dir = np.einsum("nc,nkc,nkj->nj", gc, k, dY)
        dirs = pr["dirs"]
        proj = np.eye(3)[None] - dirs[:, :, None] * dirs[:, None, :]
        g_mu_dir = np.einsum("nij,nj->ni", proj, g_dir) / pr["dist"][:, None]
        g_means = g_means + g_mu_dir

    # pose: left perturbation T <- Exp(xi) T, xi = (rho, phi) at 0.
    # p moves by rho + phi x p; the camera centre moves by -Rc^T rho;
    # Scam moves by [phi]x Scam - Scam [phi]x.
    g_rho = gp.sum(0) + (g_mu_dir @ Rc.T).sum(0)
    g_phi = np.cross(p, gp).sum(0)
    for k_ in range(3):
        e = np.zeros(3)
        e[k_] = 1.0
        E = skew(e)
        dS = E @ Scam - Scam @ E
        g_phi[k_] += np.sum(GScam * dS)
    return dict(d_means=g_means, d_log_scales=g_log_scales, d_quats=g_quats,
                d_opacity=g_opacity, d_colors=g_colors,
                d_pose=np.concatenate([g_rho, g_phi]))
