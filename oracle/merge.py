"""Upsampling and blending of the sub-images.

Paper passages: Sec. 3.3 (a plain bilinear filter would mix texels that hold
no information into defined pixels; the masks with fixed weights act as the
alpha channel) and Sec. 4.2 with Eq. 1: every sub-image is bilinearly scaled
to full size, then the images are combined one after another starting at the
lowest resolution, c'_L = c_L and c'_i = c_i alpha_i + c'_(next coarser) (1 -
alpha_i) with alpha_i = min(a_i w_i, 1).

reading (Eq. 1 index): the printed recursion refers to c'_(i-1), which would
run from the finest level up; the text starts at the lowest resolution and
works successively upward, so the recursion uses the next coarser enabled
level's composite.

reading (undefined texels): the bilinear taps of level i are restricted to
texels with S_i = 1 and renormalised by the sum of their weights (select,
never multiply undefined values by 0); a_i is bilinear over all taps (it is 0
off the stencil).  Texel-centre convention, clamp-to-edge.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def _bilinear_setup(n_full, s, n_level, dtype):
    """Per full-res coordinate: low tap, high tap (clamped) and fraction.
    u = (X + 0.5) / s - 0.5, x0 = floor(u), f = u - x0."""
    X = np.arange(n_full).astype(dtype)
    u = (X + dtype(0.5)) / dtype(s) - dtype(0.5)
    x0 = np.floor(u)
    fx = u - x0
    i0 = np.clip(x0.astype(np.int64), 0, n_level - 1)
    i1 = np.clip(x0.astype(np.int64) + 1, 0, n_level - 1)
    return i0, i1, fx


def upsampled_alpha(width, height, level, weight, alpha_i, stencil_i, dtype=np.float32):
    """alpha_i at every full-resolution pixel, as the merge blends with it:
    min(A w, 1) with A the bilinear of a_i over the four taps, and 0 where
    none of the taps lies in the stencil (den = 0)."""
    one = dtype(1.0)
    zero = dtype(0.0)
    s = 1 << (level - 1)
    Si = np.asarray(stencil_i).astype(bool)
    Hi, Wi = Si.shape
    xi0, xi1, fx = _bilinear_setup(width, s, Wi, dtype)
    yi0, yi1, fy = _bilinear_setup(height, s, Hi, dtype)
    FX = fx[None, :]
    FY = fy[:, None]
    b = [(one - FX) * (one - FY), FX * (one - FY), (one - FX) * FY, FX * FY]
    taps = [(yi0[:, None], xi0[None, :]), (yi0[:, None], xi1[None, :]),
            (yi1[:, None], xi0[None, :]), (yi1[:, None], xi1[None, :])]
    den = np.zeros((height, width), dtype)
    for t, (ty, tx) in enumerate(taps):
        den = den + np.where(Si[ty, tx], b[t], zero)
    ai = np.asarray(alpha_i).astype(dtype)
    A = np.zeros((height, width), dtype)
    for t, (ty, tx) in enumerate(taps):
        A = A + b[t] * ai[ty, tx]
    al = np.minimum(A * dtype(weight), one)
    return np.where(den > zero, al, zero)


def upsample_merge(width, height, levels, weights, alpha, stencil, level_out, channels=1,
                   dtype=np.float32):
    """Final image [C][H][W] (or [H][W] when channels == 1).

    levels     enabled levels ascending (1-based); the last is the coarsest L.
    weights    level -> w_i (Table 1)
    alpha      level (< L) -> a_i [H_i][W_i]
    stencil    level -> S_i [H_i][W_i] (S_L all ones)
    level_out  level -> c_i [C][H_i][W_i] or [H_i][W_i]; values where S_i = 0
               are never read.
    Per level and pixel: b = ((1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy) over taps
    (x0,y0), (x1,y0), (x0,y1), (x1,y1); A = sum b_t a(t); den = sum over taps
    with S = 1 of b_t; num = the same sum of b_t c(t); C = num / den (0 if den
    = 0); alpha = min(A w, 1) (0 if den = 0).  All sums left to right from +0.
    """
    L = levels[-1]
    one = dtype(1.0)
    zero = dtype(0.0)
    comp = {}
    alph = {}
    for i in levels:
        s = 1 << (i - 1)
        Si = stencil[i].astype(bool)
        Hi, Wi = Si.shape
        ci = level_out[i].astype(dtype)
        if ci.ndim == 2:
            ci = ci[None]
        xi0, xi1, fx = _bilinear_setup(width, s, Wi, dtype)
        yi0, yi1, fy = _bilinear_setup(height, s, Hi, dtype)
        FX = fx[None, :]
        FY = fy[:, None]
        b = [(one - FX) * (one - FY), FX * (one - FY), (one - FX) * FY, FX * FY]
        taps = [(yi0[:, None], xi0[None, :]), (yi0[:, None], xi1[None, :]),
                (yi1[:, None], xi0[None, :]), (yi1[:, None], xi1[None, :])]
        den = np.zeros((height, width), dtype)
        sel = []
        for t, (ty, tx) in enumerate(taps):
            st = Si[ty, tx]
            sel.append(st)
            den = den + np.where(st, b[t], zero)
        num = np.zeros((ci.shape[0], height, width), dtype)
        with np.errstate(invalid="ignore"):
            for t, (ty, tx) in enumerate(taps):
                num = num + np.where(sel[t][None], b[t][None] * ci[:, ty, tx], zero)
            C = np.where(den[None] > zero, num / den[None], zero)
        comp[i] = C
        if i != L:
            ai = alpha[i].astype(dtype)
            A = np.zeros((height, width), dtype)
            for t, (ty, tx) in enumerate(taps):
                A = A + b[t] * ai[ty, tx]
            al = np.minimum(A * dtype(weights[i]), one)
            alph[i] = np.where(den > zero, al, zero)
    out = comp[L]
    for i in reversed(levels[:-1]):
        a = alph[i][None]
        out = comp[i] * a + out * (one - a)
    out = out.astype(dtype)
    return out[0] if channels == 1 else out
