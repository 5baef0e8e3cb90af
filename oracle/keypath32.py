"""FP32 key path of the projection: the quantities that decide which tiles a
Gaussian is binned into and in which depth order it is sorted.

Test infrastructure only (see oracle/__init__.py).

The paper states that the map is rendered by differentiable 3D Gaussian
splatting (Sec. I and II-A cite 3DGS; Sec. III-A optimises the map by gradient
descent, Eq. (map_loss); Sec. III-C refines on differentiably rendered RGB and
depth).  It never spells out projection or binning, so the definition below
is the EWA projection of a 3D Gaussian (Zwicker et al. 2001, as used by 3DGS)
with an opacity-aware bounding box.  Every operation here is evaluated in IEEE
FP32 with round-to-nearest and no fused multiply-add, in a fixed left-to-right
order, so that a GPU implementation following the same order reproduces the
bits exactly.  The five transcendentals per Gaussian (three exp of the
log-scales, exp(-o) inside the sigmoid, log(255*sigma)) are evaluated in FP64
from the FP32 inputs and rounded once to FP32.

Order of operations (every name is an FP32 value):
  p_i  = ((Rc_i0*m0 + Rc_i1*m1) + Rc_i2*m2) + t_i
  cull unless p2 > z_near
  s_k  = f32(exp(f64(l_k)))
  qn   = sqrt(((w*w + x*x) + y*y) + z*z); cull unless qn > 0; q_hat = q/qn
  R    = unit-quaternion rotation matrix of q_hat (products xx, xy, ... first)
  M_ij = R_ij * s_j
  S_ij = (M_i0*M_j0 + M_i1*M_j1) + M_i2*M_j2           (i <= j, S symmetric)
  W_ik = (Rc_i0*S_0k + Rc_i1*S_1k) + Rc_i2*S_2k
  V_ij = (W_i0*Rc_j0 + W_i1*Rc_j1) + W_i2*Rc_j2         (i <= j, V symmetric)
  rx = p0/p2, ry = p1/p2, u = fx*rx + cx, v = fy*ry + cy
  limx = 1.3 * ((0.5*W)/fx); rxc = clamp(rx, -limx, limx)   (same for y)
  j00 = fx/p2, j02 = -(fx*rxc)/p2, j11 = fy/p2, j12 = -(fy*ryc)/p2
  T00 = j00*V00 + j02*V02, T01 = j00*V01 + j02*V12, T02 = j00*V02 + j02*V22
  T11 = j11*V11 + j12*V12, T12 = j11*V12 + j12*V22
  a = (T00*j00 + T02*j02) + 0.3,  b = T01*j11 + T02*j12,  c = (T11*j11 + T12*j12) + 0.3
  det = a*c - b*b; cull unless det > 0
  sigma = f32(1/(1 + exp(-f64(o)))); t = 255*f64(sigma); cull unless t > 1
  k2 = f32(2*log(t)); ex = sqrt(k2*a); ey = sqrt(k2*c)
  cull unless u, v, ex, ey are finite
  x0 = clampi(floor((u - ex)*(1/TW)), 0, TX); x1 = clampi(floor((u + ex)*(1/TW)) + 1, 0, TX)
  (same for y); cull if (x1-x0)*(y1-y0) == 0
  depth key = FP32 bit pattern of p2
Tile sizes are powers of two, so multiplying by 1/TW is exact.
"""
from __future__ import annotations

import numpy as np

F = np.float32
D = np.float64

BLUR = F(0.3)
GUARD = F(1.3)
HALF = F(0.5)


def _f32_of_f64(x64: np.ndarray):
    """Round an FP64 array to FP32 once; also flag values whose FP64 result
    lies within 4 FP64 ulps of an FP32 rounding midpoint (a different but
    equally accurate FP64 library could round those to the other FP32)."""
    r = x64.astype(F)
    up = np.nextafter(r, F(np.inf)).astype(D)
    dn = np.nextafter(r, F(-np.inf)).astype(D)
    rd = r.astype(D)
    mid_hi = 0.5 * (rd + up)
    mid_lo = 0.5 * (rd + dn)
    tol = 4.0 * np.spacing(np.abs(x64))
    with np.errstate(invalid="ignore"):
        flag = (np.abs(x64 - mid_hi) <= tol) | (np.abs(x64 - mid_lo) <= tol)
    return r, flag


def keypath(means, log_scales, quats, opacity_logits, viewmat, intrin, width,
            height, tile_w=16, tile_h=16, z_near=0.2):
    """Evaluate the FP32 key path for every Gaussian of one view.

    Returns a dict of per-Gaussian arrays: visible (bool), p (FP32 [N,3]),
    zbits (uint32), rect (int64 [N,4] = x0,y0,x1,y1 in tiles), tiles (int64),
    u, v, a, b, c (FP32) and straddle (bool: a transcendental result sat
    next to an FP32 rounding midpoint).
    """
    with np.errstate(all="ignore"):
        m = np.asarray(means, F)
        ls = np.asarray(log_scales, F)
        q = np.asarray(quats, F)
        o = np.asarray(opacity_logits, F)
        vm = np.asarray(viewmat, F).reshape(3, 4)
        Rc = vm[:, :3]
        tc = vm[:, 3]
        fx, fy, cx, cy = (F(x) for x in np.asarray(intrin, F))
        zn = F(z_near)

        m0, m1, m2 = m[:, 0], m[:, 1], m[:, 2]
        p = [((Rc[i, 0] * m0 + Rc[i, 1] * m1) + Rc[i, 2] * m2) + tc[i]
             for i in range(3)]
        p0, p1, p2 = p
        vis = p2 > zn

        s, st_s = _f32_of_f64(np.exp(ls.astype(D)))
        straddle = st_s.any(axis=1)
        qw, qx, qy, qz = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
        qn = np.sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz)
        vis &= qn > 0
        w, x, y, z = qw / qn, qx / qn, qy / qn, qz / qn
        xx, yy, zz = x * x, y * y, z * z
        xy, xz, yz = x * y, x * z, y * z
        wx, wy, wz = w * x, w * y, w * z
        one, two = F(1), F(2)
        R = [[one - two * (yy + zz), two * (xy - wz), two * (xz + wy)],
             [two * (xy + wz), one - two * (xx + zz), two * (yz - wx)],
             [two * (xz - wy), two * (yz + wx), one - two * (xx + yy)]]
        M = [[R[i][j] * s[:, j] for j in range(3)] for i in range(3)]
        S = [[None] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(i, 3):
                S[i][j] = (M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2]
                S[j][i] = S[i][j]
        Wm = [[(Rc[i, 0] * S[0][k] + Rc[i, 1] * S[1][k]) + Rc[i, 2] * S[2][k]
               for k in range(3)] for i in range(3)]
        V = [[None] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(i, 3):
                V[i][j] = (Wm[i][0] * Rc[j, 0] + Wm[i][1] * Rc[j, 1]) + Wm[i][2] * Rc[j, 2]
                V[j][i] = V[i][j]

        rx = p0 / p2
        ry = p1 / p2
        u = fx * rx + cx
        v = fy * ry + cy
        limx = GUARD * ((HALF * F(width)) / fx)
        limy = GUARD * ((HALF * F(height)) / fy)
        rxc = np.minimum(np.maximum(rx, -limx), limx)
        ryc = np.minimum(np.maximum(ry, -limy), limy)
        j00 = fx / p2
        j02 = -(fx * rxc) / p2
        j11 = fy / p2
        j12 = -(fy * ryc) / p2
        T00 = j00 * V[0][0] + j02 * V[0][2]
        T01 = j00 * V[0][1] + j02 * V[1][2]
        T02 = j00 * V[0][2] + j02 * V[2][2]
        T11 = j11 * V[1][1] + j12 * V[1][2]
        T12 = j11 * V[1][2] + j12 * V[2][2]
        a = (T00 * j00 + T02 * j02) + BLUR
        b = T01 * j11 + T02 * j12
        c = (T11 * j11 + T12 * j12) + BLUR
        det = a * c - b * b
        vis &= det > 0

        sig64 = 1.0 / (1.0 + np.exp(-o.astype(D)))
        sigma, st_o = _f32_of_f64(sig64)
        straddle |= st_o
        t = D(255.0) * sigma.astype(D)
        vis &= t > 1.0
        k2, st_k = _f32_of_f64(2.0 * np.log(np.where(t > 1.0, t, 2.0)))
        straddle |= st_k & (t > 1.0)
        ex = np.sqrt(k2 * a)
        ey = np.sqrt(k2 * c)
        vis &= np.isfinite(u) & np.isfinite(v) & np.isfinite(ex) & np.isfinite(ey)

        TX = -(-width // tile_w)
        TY = -(-height // tile_h)
        itw = F(1.0 / tile_w)
        ith = F(1.0 / tile_h)

        def clampi(f, hi):
            f = np.where(np.isfinite(f) | np.isinf(f), f, 0)  # NaN only on culled rows
            return np.clip(f, 0, hi).astype(np.int64)

        x0 = clampi(np.floor((u - ex) * itw), TX)
        x1 = clampi(np.floor((u + ex) * itw) + F(1), TX)
        y0 = clampi(np.floor((v - ey) * ith), TY)
        y1 = clampi(np.floor((v + ey) * ith) + F(1), TY)
        tiles = (x1 - x0) * (y1 - y0)
        vis &= tiles > 0
        rect = np.stack([x0, y0, x1, y1], axis=1)
        rect[~vis] = 0
        tiles = np.where(vis, tiles, 0)
        zbits = p2.view(np.uint32).copy()
    return dict(visible=vis, p=np.stack(p, 1), zbits=zbits, rect=rect,
                tiles=tiles, u=u, v=v, a=a, b=b, c=c, sigma=sigma,
                straddle=straddle & vis, TX=TX, TY=TY)
