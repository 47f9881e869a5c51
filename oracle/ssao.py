"""Screen-space ambient occlusion evaluated per sub-image.

Paper passages: Sec. 2.4 names SSAO (Mittring 2007; Bavoil et al. 2008) but
prints no estimator; Sec. 3.2 / 4.1 evaluate the effect per sub-image only
where the level's stencil permits; Sec. 5 compares against naive rendering
at full resolution.

reading (estimator): normal-oriented hemisphere sampling with a fixed,
caller-supplied kernel K[S][3] (no per-pixel rotation), a hard range check
|z - z_s| < r, a relative depth bias, off-screen samples counted as
unoccluded, output = occluded fraction (0 = unoccluded).  The tangent frame
is the branch-free orthonormal basis of Duff et al., "Building an
Orthonormal Basis, Revisited", JCGT 6(1), 2017.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SSAOParams:
    kernel: np.ndarray      # f32 [S][3] hemisphere samples in the tangent frame
    radius: float = 1.0     # world-space sample radius r
    bias_rel: float = 0.02  # relative depth bias b


def _valid(z):
    return np.isfinite(z) & (z > 0)


def view_position(xs, ys, z, f, cx, cy, dtype):
    """Sub-image texel (x, y) with depth z -> view-space point
    P = (X z, Y z, -z), X = ((x + 0.5) - cx) / f, Y = (cy - (y + 0.5)) / f."""
    half = dtype(0.5)
    X = ((xs.astype(dtype) + half) - cx) / f
    Y = (cy - (ys.astype(dtype) + half)) / f
    return X * z, Y * z, -z


def tangent_frame(nx, ny, nz, dtype):
    """Duff et al. 2017: sg = copysign(1, nz), a = -1/(sg + nz), b = (nx ny) a,
    T = (1 + (sg (nx nx)) a, sg b, -(sg nx)), B = (b, sg + (ny ny) a, -ny)."""
    one = dtype(1.0)
    sg = np.copysign(one, nz).astype(dtype)
    a = -one / (sg + nz)
    b = (nx * ny) * a
    T = (one + ((sg * (nx * nx)) * a), sg * b, -(sg * nx))
    B = (b, sg + ((ny * ny) * a), -ny)
    return T, B


def camera(width_i, height_i, focal, level, dtype):
    """Sub-image camera: f_i = f / s_i, principal point (W_i / 2, H_i / 2)."""
    s = dtype(1 << (level - 1))
    f = dtype(focal) / s
    cx = dtype(0.5) * dtype(width_i)
    cy = dtype(0.5) * dtype(height_i)
    return f, cx, cy


def ssao_texels(zi, ni, focal, level, xs, ys, p: SSAOParams, dtype=np.float32):
    """Occlusion at the listed texels (xs, ys) of level `level`.

    zi: [H_i][W_i] level depth, ni: [3][H_i][W_i] level normals.
    Per sample j, with (kx, ky, kz) = K[j]:
      Q_c = ((P_c + kx rT_c) + ky rB_c) + kz rN_c      (rT = r T etc.)
      d = -Q_z; skip unless d > 0
      inv = 1 / d; u = cx + (Q_x inv) f; v = cy - (Q_y inv) f
      skip unless 0 <= u < W_i and 0 <= v < H_i
      z_s = z_i[floor v][floor u]; skip unless z_s is geometry
      occluded iff z_s < d - (b d) and |z - z_s| < r
    result = occluded count / S; background texels give 0."""
    Hi, Wi = zi.shape
    f, cx, cy = camera(Wi, Hi, focal, level, dtype)
    zl = zi.astype(dtype)
    z = zl[ys, xs]
    nx = ni[0][ys, xs].astype(dtype)
    ny = ni[1][ys, xs].astype(dtype)
    nz = ni[2][ys, xs].astype(dtype)
    K = p.kernel.astype(dtype)
    r = dtype(p.radius)
    b = dtype(p.bias_rel)
    S = K.shape[0]
    valid = _valid(z)
    occ = np.zeros(z.shape, np.int64)
    with np.errstate(all="ignore"):
        Px, Py, Pz = view_position(xs, ys, z, f, cx, cy, dtype)
        T, B = tangent_frame(nx, ny, nz, dtype)
        rT = [r * t for t in T]
        rB = [r * t for t in B]
        rN = [r * nx, r * ny, r * nz]
        Wf, Hf = dtype(Wi), dtype(Hi)
        zero = dtype(0.0)
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
            occ += m
    out = occ.astype(dtype) / dtype(S)
    return np.where(valid, out, dtype(0.0)).astype(dtype)


def ssao_level(zi, ni, focal, level, p: SSAOParams, stencil=None, dtype=np.float32,
               fill=np.nan):
    """Sub-image c_i: evaluated where the stencil is 1 (everywhere if None);
    other texels are undefined and set to `fill`."""
    Hi, Wi = zi.shape
    if stencil is None:
        ys, xs = np.divmod(np.arange(Hi * Wi), Wi)
    else:
        ys, xs = np.nonzero(stencil)
    out = np.full((Hi, Wi), fill, dtype)
    if len(xs):
        out[ys, xs] = ssao_texels(zi, ni, focal, level, xs, ys, p, dtype)
    return out


def ssao_plain(depth, normal, focal, p: SSAOParams, dtype=np.float32):
    """Naive full-resolution SSAO: the estimator at level 1 over every pixel."""
    return ssao_level(depth, normal, focal, 1, p, None, dtype)
