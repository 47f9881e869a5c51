"""One-bounce screen-space indirect light (the paper's third effect).

Paper passages: Sec. 2.4 (SSGI after Ritschel et al. 2009 generalises SSAO
by adding indirect light from other surfaces visible on screen, computing
light transport between samples near a pixel from the G-buffer); Sec. 4 and
Table 1 (the half-resolution sub-image is not used for SSGI).

reading (estimator, not printed in the paper): the SSAO sampling and
occlusion test are run unchanged; every occluding sample instead adds the
directly lit colour of the texel it hit, as a small surface patch sending
light to the receiver:
  X_t = view position of the hit texel t, n_t its normal, C_t its colour;
  v = X_t - P, dd = dot(v, v), skip unless dd > 0;
  dist2 = max(dd, (0.1 r)(0.1 r)); v_hat = v (1 / sqrt(dd));
  g = (max(0, dot(n, v_hat)) max(0, -dot(n_t, v_hat))) / dist2;
  acc_c = acc_c + C_c g for each channel c;
  out_c = acc_c ((r r) / S).
dot(a, b) = ((a_x b_x) + (a_y b_y)) + (a_z b_z).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ssao import view_position, tangent_frame, camera


@dataclass
class SSGIParams:
    kernel: np.ndarray      # f32 [S][3]
    radius: float = 2.0
    bias_rel: float = 0.02


def _valid(z):
    return np.isfinite(z) & (z > 0)


def _dot(a, b):
    return ((a[0] * b[0]) + (a[1] * b[1])) + (a[2] * b[2])


def ssgi_texels(zi, ni, ci, focal, level, xs, ys, p: SSGIParams, dtype=np.float32):
    """Indirect RGB [3][n] at the listed texels of a level.

    zi [H_i][W_i], ni [3][H_i][W_i], ci [3][H_i][W_i] (colour, widened)."""
    Hi, Wi = zi.shape
    f, cx, cy = camera(Wi, Hi, focal, level, dtype)
    zl = zi.astype(dtype)
    nl = ni.astype(dtype)
    cl = ci.astype(dtype)
    z = zl[ys, xs]
    n = [nl[0][ys, xs], nl[1][ys, xs], nl[2][ys, xs]]
    K = p.kernel.astype(dtype)
    r = dtype(p.radius)
    b = dtype(p.bias_rel)
    S = K.shape[0]
    valid = _valid(z)
    zero = dtype(0.0)
    acc = np.zeros((3,) + z.shape, dtype)
    rmin = dtype(0.1) * r
    rmin2 = rmin * rmin
    with np.errstate(all="ignore"):
        Px, Py, Pz = view_position(xs, ys, z, f, cx, cy, dtype)
        T, B = tangent_frame(n[0], n[1], n[2], dtype)
        rT = [r * t for t in T]
        rB = [r * t for t in B]
        rN = [r * n[0], r * n[1], r * n[2]]
        Wf, Hf = dtype(Wi), dtype(Hi)
        for j in range(S):
            kx, ky, kz = K[j, 0], K[j, 1], K[j, 2]
            Qx = ((Px + kx * rT[0]) + ky * rB[0]) + kz * rN[0]
            Qy = ((Py + kx * rT[1]) + ky * rB[1]) + kz * rN[1]
            Qz = ((Pz + kx * rT[2]) + ky * rB[2]) + kz * rN[2]
            d = -Qz
            m = valid & (d > zero)
            inv = dtype(1.0) / d
            u = cx + (Qx * inv) * f
            v = cy - (Qy * inv) * f
            m &= (u >= zero) & (u < Wf) & (v >= zero) & (v < Hf)
            tx = np.where(m, np.floor(u), 0).astype(np.int64)
            ty = np.where(m, np.floor(v), 0).astype(np.int64)
            zs = zl[ty, tx]
            m &= _valid(zs)
            m &= (zs < d - (b * d)) & (np.abs(z - zs) < r)
            Xt = view_position(tx, ty, zs, f, cx, cy, dtype)
            vv = (Xt[0] - Px, Xt[1] - Py, Xt[2] - Pz)
            dd = _dot(vv, vv)
            m &= dd > zero
            dist2 = np.maximum(dd, rmin2)
            il = dtype(1.0) / np.sqrt(dd)
            vh = (vv[0] * il, vv[1] * il, vv[2] * il)
            nt = (nl[0][ty, tx], nl[1][ty, tx], nl[2][ty, tx])
            cr = np.maximum(zero, _dot(n, vh))
            ce = np.maximum(zero, -_dot(nt, vh))
            g = (cr * ce) / dist2
            for c in range(3):
                acc[c] = acc[c] + np.where(m, cl[c][ty, tx] * g, zero)
    scale = (r * r) / dtype(S)
    out = acc * scale
    return np.where(valid[None], out, zero).astype(dtype)


def ssgi_level(zi, ni, ci, focal, level, p: SSGIParams, stencil=None, dtype=np.float32,
               fill=np.nan):
    Hi, Wi = zi.shape
    if stencil is None:
        ys, xs = np.divmod(np.arange(Hi * Wi), Wi)
    else:
        ys, xs = np.nonzero(stencil)
    out = np.full((3, Hi, Wi), fill, dtype)
    if len(xs):
        out[:, ys, xs] = ssgi_texels(zi, ni, ci, focal, level, xs, ys, p, dtype)
    return out
