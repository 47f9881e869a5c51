"""Bilateral blur of SSAO sub-images (Sec. 4.1, rendering of the
sub-images): the occlusion of a level is smoothed to cut the variance of a
small sample count, without carrying values from texels the level did not
render into the ones it did, and without blurring across depth
discontinuities.

reading (the paper names a bilateral filter and nothing more):
  * taps: the (2R+1) x (2R+1) window around a rendered texel p, R in {1, 2};
    only taps inside the level image that the level rendered (stencil 1) and
    whose depth is valid take part;
  * spatial weight: the binomial weights of order 2R per axis (1 2 1 / 4,
    1 4 6 4 1 / 16), their product for a tap (exact in FP32);
  * range weight: max(0, 1 - |z_q - z_p| / (d * z_p)), d the relative depth
    tolerance (0.05, the edge detector's depth ratio, by default), on the
    level's point-sampled depth;
  * result: sum of w * c over the taps divided by the sum of w, both summed
    in window order (rows top to bottom, each row left to right); p itself
    always has weight > 0.  Texels with invalid depth keep their value.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass
from math import comb

import numpy as np


@dataclass
class BilateralParams:
    levels: int = 0b1110      # bit i-1: blur level i (default: every level below full resolution)
    radius: int = 2           # window (2R+1)^2
    depth_rel: float = 0.05   # relative depth tolerance of the range weight


def binomial_weights(radius: int, dtype=np.float32) -> np.ndarray:
    """C(2R, k) / 4^R for k = 0..2R (exact binary fractions)."""
    return np.array([comb(2 * radius, k) / 4.0 ** radius for k in range(2 * radius + 1)], dtype)


def _valid(z):
    return np.isfinite(z) & (z > 0)


def bilateral_level(c, zi, stencil, p: BilateralParams, dtype=np.float32):
    """c: level values [Hi][Wi], defined where stencil != 0 (stencil None:
    everywhere; other values are ignored); zi: the level's depth [Hi][Wi].
    Returns the blurred values, defined where c is."""
    c = np.asarray(c, dtype)
    zi = np.asarray(zi, dtype)
    Hi, Wi = zi.shape
    R = int(p.radius)
    b = binomial_weights(R, dtype)
    defined = np.ones((Hi, Wi), bool) if stencil is None else np.asarray(stencil) != 0
    ok = defined & _valid(zi)
    d = dtype(p.depth_rel) * zi  # the tolerance of each centre texel
    num = np.zeros((Hi, Wi), dtype)
    den = np.zeros((Hi, Wi), dtype)
    one = dtype(1)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            # tap value, depth and usability at q = p + (dx, dy) for every p
            cq = np.zeros((Hi, Wi), dtype)
            zq = np.ones((Hi, Wi), dtype)
            use = np.zeros((Hi, Wi), bool)
            ys, ye = max(0, -dy), min(Hi, Hi - dy)
            xs, xe = max(0, -dx), min(Wi, Wi - dx)
            if ys < ye and xs < xe:
                cq[ys:ye, xs:xe] = np.where(ok[ys + dy:ye + dy, xs + dx:xe + dx],
                                            c[ys + dy:ye + dy, xs + dx:xe + dx], 0)
                zq[ys:ye, xs:xe] = zi[ys + dy:ye + dy, xs + dx:xe + dx]
                use[ys:ye, xs:xe] = ok[ys + dy:ye + dy, xs + dx:xe + dx]
            use &= ok
            with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
                t = np.abs(zq - zi) / d
                wz = np.maximum(one - t, dtype(0))
            w = (b[dy + R] * b[dx + R]) * wz
            w = np.where(use, w, dtype(0)).astype(dtype)
            num = (num + w * cq).astype(dtype)
            den = (den + w).astype(dtype)
    with np.errstate(invalid="ignore", divide="ignore"):
        blurred = (num / den).astype(dtype)
    out = c.copy()
    out[ok] = blurred[ok]
    return out
