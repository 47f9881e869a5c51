"""The whole per-frame pipeline for one effect (Sec. 3: masks -> sub-images
-> composition), and the naive full-resolution pass it is compared with
(Sec. 5).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .masks import MaskParams, edge_image, foveate, build_pyramid, level_sample, Pyramid
from .ssao import SSAOParams, ssao_level
from .merge import upsample_merge, upsampled_alpha
from .shadow import ShadowParams, hard_shadow, shadow_edges, pcss_level
from .ssgi import SSGIParams, ssgi_level
from .bilateral import BilateralParams, bilateral_level


@dataclass
class Frame:
    out: np.ndarray
    pyramid: Pyramid = None
    level_out: dict = field(default_factory=dict)


def frame(effect, depth, normal, focal, mp: MaskParams, params, multires=True, color=None,
          dtype=np.float32, level_dtype=None, bilateral: BilateralParams = None) -> Frame:
    """effect in {"ssao", "shadow", "ssgi"}; params the matching *Params.

    multires=False is the naive full-resolution pass.  level_dtype (e.g.
    np.float16) stores every sub-image value in that type (rounded to
    nearest) between the evaluation and the merge.  bilateral (SSAO only)
    blurs the sub-images of its levels before the merge (Sec. 4.1); the
    blurred values are stored in level_dtype too."""
    H, W = depth.shape
    channels = 3 if effect == "ssgi" else 1

    def evaluate(level, stencil):
        zi = level_sample(depth, level)
        if effect == "ssao":
            ni = level_sample(normal, level)
            return ssao_level(zi, ni, focal, level, params, stencil, dtype)
        if effect == "shadow":
            return pcss_level(zi, focal, level, params, stencil, dtype)
        ni = level_sample(normal, level)
        ci = level_sample(color, level)
        return ssgi_level(zi, ni, ci, focal, level, params, stencil, dtype)

    if not multires:
        return Frame(out=evaluate(1, None))

    E = edge_image(depth, normal, mp.depth_ratio, mp.normal_cos, dtype)
    if effect == "shadow":
        # Sec. 3.1: shadow edges from a one-sample shadow test, plus the
        # geometry edges, combined by maximum.
        hard = hard_shadow(depth, focal, 1, params, dtype)
        E = E | shadow_edges(hard, depth)
    E = foveate(E, mp.fovea)
    pyr = build_pyramid(E, mp, dtype)
    L = pyr.levels[-1]
    lo = {}
    for i in pyr.levels:
        st = None if i == L else pyr.stencil[i]
        lo[i] = evaluate(i, st)
        if level_dtype is not None:
            lo[i] = lo[i].astype(level_dtype).astype(dtype)
        if bilateral is not None and effect == "ssao" and bilateral.levels >> (i - 1) & 1:
            lo[i] = bilateral_level(lo[i], level_sample(depth, i), st, bilateral, dtype)
            if level_dtype is not None:
                lo[i] = lo[i].astype(level_dtype).astype(dtype)
    weights = {i: mp.weight[i - 1] for i in pyr.levels}
    out = upsample_merge(W, H, pyr.levels, weights, pyr.alpha, pyr.stencil, lo, channels, dtype)
    return Frame(out=out, pyramid=pyr, level_out=lo)


def frame_fullres_levels(depth, normal, focal, mp: MaskParams, level_params: dict, dtype=np.float32) -> Frame:
    """SSAO with the sub-images realised at full resolution with fewer
    samples instead of at a lower resolution (Sec. 6).

    reading: every enabled level keeps its mask (stencil, a_i and the Eq. 1
    blend weight alpha_i at full resolution, exactly as in the merge), but
    its value at a pixel is the SSAO of that full-resolution pixel with the
    level's own sample set level_params[i] (an SSAOParams, typically with
    fewer samples for coarser levels).  The blend is Eq. 1 from the coarsest
    level: out = c_L; out = c_i alpha_i + out (1 - alpha_i) for the finer
    levels, coarse to fine."""
    H, W = depth.shape
    E = edge_image(depth, normal, mp.depth_ratio, mp.normal_cos, dtype)
    E = foveate(E, mp.fovea)
    pyr = build_pyramid(E, mp, dtype)
    L = pyr.levels[-1]
    one = dtype(1)
    lo = {i: ssao_level(depth, normal, focal, 1, level_params[i], None, dtype) for i in pyr.levels}
    out = lo[L]
    for i in reversed(pyr.levels[:-1]):
        a = upsampled_alpha(W, H, i, mp.weight[i - 1], pyr.alpha[i], pyr.stencil[i], dtype)
        out = (lo[i] * a + out * (one - a)).astype(dtype)
    return Frame(out=out, pyramid=pyr, level_out=lo)
