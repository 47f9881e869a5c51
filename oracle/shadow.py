"""Soft shadows from a shadow map (the paper's second effect).

Paper passages: Sec. 2.4 names shadow mapping (Williams 1978), percentage
closer filtering (Reeves et al. 1987) and the PCSS penumbra estimate
(Fernando 2005), sampling the map at several neighbouring positions.  Sec.
3.1: for soft shadows the mask also needs shadow edges, found from a fast
one-sample-per-pixel shadow test that is differentiated, and the geometry
edges are kept as well.

reading (estimator, not printed in the paper): Fernando's three steps.
  light coordinates: P_l = M P (3 x 4 affine, each row summed left to right),
    d_r = -P_l.z, su = c_L + (P_l.x / d_r) f_L, sv = c_L - (P_l.y / d_r) f_L
    with c_L = size / 2 (computed as inv = 1 / d_r, (P_l.x inv) f_L);
    outside the light frustum (d_r <= 0 or (su, sv) off the map) = lit.
  hard bit: SM[floor sv][floor su] < d_r - bias.
  blocker search: half-width R_s = (l (d_r - n_L)) / (d_r n_L) texels with
    l = f_L (0.5 w_L); taps floor(s + R_s p_k), clamped to the map; blockers
    are taps with SM < d_r - bias; none -> visibility 1.
  penumbra: d_b = (sum of blocker depths, ascending order) / count;
    R_f = (l (d_r - d_b)) / (d_b d_r).
  PCF: visibility = (number of PCF taps with not (SM < d_r - bias)) / n_pcf.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ssao import view_position, camera


@dataclass
class ShadowParams:
    shadow_map: np.ndarray     # f32 [size][size] linear light depth
    view_to_light: np.ndarray  # f32 [3][4]
    light_focal: float         # f_L in texels
    light_size: float          # w_L, side of the square area light
    light_near: float          # n_L
    bias: float                # absolute depth bias
    blocker_disk: np.ndarray   # f32 [nb][2] unit-disk points
    pcf_disk: np.ndarray       # f32 [np][2] unit-disk points


def _valid(z):
    return np.isfinite(z) & (z > 0)


def light_coords(Px, Py, Pz, p: ShadowParams, dtype):
    M = p.view_to_light.astype(dtype)
    Lx = ((M[0, 0] * Px + M[0, 1] * Py) + M[0, 2] * Pz) + M[0, 3]
    Ly = ((M[1, 0] * Px + M[1, 1] * Py) + M[1, 2] * Pz) + M[1, 3]
    Lz = ((M[2, 0] * Px + M[2, 1] * Py) + M[2, 2] * Pz) + M[2, 3]
    size = p.shadow_map.shape[0]
    fL = dtype(p.light_focal)
    cL = dtype(0.5) * dtype(size)
    dr = -Lz
    with np.errstate(all="ignore"):
        inv = dtype(1.0) / dr
        su = cL + (Lx * inv) * fL
        sv = cL - (Ly * inv) * fL
    zero = dtype(0.0)
    sz = dtype(size)
    inside = (dr > zero) & (su >= zero) & (su < sz) & (sv >= zero) & (sv < sz)
    return dr, su, sv, inside


def _tap(sm, su, sv, R, pts, k, dtype, inside):
    size = sm.shape[0]
    with np.errstate(all="ignore"):
        fx = np.floor(su + R * pts[k, 0])
        fy = np.floor(sv + R * pts[k, 1])
    fx = np.where(inside, fx, 0)
    fy = np.where(inside, fy, 0)
    tx = np.clip(fx, 0, size - 1).astype(np.int64)
    ty = np.clip(fy, 0, size - 1).astype(np.int64)
    return sm[ty, tx]


def hard_shadow(zi, focal, level, p: ShadowParams, dtype=np.float32):
    """One-sample shadow test per texel of a level (uint8; background = 0)."""
    Hi, Wi = zi.shape
    f, cx, cy = camera(Wi, Hi, focal, level, dtype)
    ys, xs = np.divmod(np.arange(Hi * Wi), Wi)
    z = zi.astype(dtype).reshape(-1)
    with np.errstate(all="ignore"):
        Px, Py, Pz = view_position(xs, ys, z, f, cx, cy, dtype)
        dr, su, sv, inside = light_coords(Px, Py, Pz, p, dtype)
        sm = p.shadow_map.astype(dtype)
        size = sm.shape[0]
        tx = np.where(inside, np.floor(su), 0).astype(np.int64)
        ty = np.where(inside, np.floor(sv), 0).astype(np.int64)
        thr = dr - dtype(p.bias)
        hard = inside & (sm[np.clip(ty, 0, size - 1), np.clip(tx, 0, size - 1)] < thr)
    hard &= _valid(z)
    return hard.reshape(Hi, Wi).astype(np.uint8)


def shadow_edges(hard, depth):
    """Differentiated hard-shadow image: a geometry pixel is a shadow edge when
    an in-image 4-neighbour that is geometry has the other shadow bit."""
    valid = _valid(depth)
    h = hard.astype(bool)
    E = np.zeros(h.shape, bool)
    d = (h[:, :-1] != h[:, 1:]) & valid[:, :-1] & valid[:, 1:]
    E[:, :-1] |= d
    E[:, 1:] |= d
    d = (h[:-1, :] != h[1:, :]) & valid[:-1, :] & valid[1:, :]
    E[:-1, :] |= d
    E[1:, :] |= d
    return (E & valid).astype(np.uint8)


def pcss_texels(zi, focal, level, xs, ys, p: ShadowParams, dtype=np.float32):
    """Visibility in [0, 1] at the listed texels of a level (1 = fully lit)."""
    Hi, Wi = zi.shape
    f, cx, cy = camera(Wi, Hi, focal, level, dtype)
    z = zi.astype(dtype)[ys, xs]
    valid = _valid(z)
    sm = p.shadow_map.astype(dtype)
    bd = p.blocker_disk.astype(dtype)
    pd = p.pcf_disk.astype(dtype)
    one = dtype(1.0)
    zero = dtype(0.0)
    with np.errstate(all="ignore"):
        Px, Py, Pz = view_position(xs, ys, z, f, cx, cy, dtype)
        dr, su, sv, inside = light_coords(Px, Py, Pz, p, dtype)
        thr = dr - dtype(p.bias)
        nL = dtype(p.light_near)
        lsz = dtype(p.light_focal) * (dtype(0.5) * dtype(p.light_size))
        Rs = (lsz * (dr - nL)) / (dr * nL)
        bsum = np.zeros(z.shape, dtype)
        bcnt = np.zeros(z.shape, np.int64)
        for k in range(bd.shape[0]):
            s = _tap(sm, su, sv, Rs, bd, k, dtype, inside)
            blk = s < thr
            bsum = bsum + np.where(blk, s, zero)
            bcnt += blk
        db = bsum / bcnt.astype(dtype)
        Rf = (lsz * (dr - db)) / (db * dr)
        lit = np.zeros(z.shape, np.int64)
        for k in range(pd.shape[0]):
            s = _tap(sm, su, sv, Rf, pd, k, dtype, inside & (bcnt > 0))
            lit += ~(s < thr)
        vis = lit.astype(dtype) / dtype(pd.shape[0])
    vis = np.where(inside & (bcnt > 0), vis, one)
    return np.where(valid, vis, one).astype(dtype)


def pcss_level(zi, focal, level, p: ShadowParams, stencil=None, dtype=np.float32, fill=np.nan):
    Hi, Wi = zi.shape
    if stencil is None:
        ys, xs = np.divmod(np.arange(Hi * Wi), Wi)
    else:
        ys, xs = np.nonzero(stencil)
    out = np.full((Hi, Wi), fill, dtype)
    if len(xs):
        out[ys, xs] = pcss_texels(zi, focal, level, xs, ys, p, dtype)
    return out
