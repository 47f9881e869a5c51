"""Pins of the oracle's fewer-samples-at-full-resolution variant (Sec. 6):
special cases that reduce it to the plain full-resolution pass, exact
regions (alpha = 1, alpha = 0 everywhere finer), a per-pixel brute force of
alpha and the blend on a tiny frame, and the merge's alpha (the two compute
it separately)."""
import math

import numpy as np
import pytest

import oracle
import scenegen

COS25 = float(np.float32(math.cos(math.radians(25.0))))


def setup(W=96, H=64, seed=3, cam=2, S=8, boxes=30):
    sc = scenegen.make_scene(seed, boxes, 8 if boxes > 10 else 0)
    gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(cam), W, H)
    t = scenegen.TABLE1["ssao"]
    mp = oracle.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"],
                           normal_cos=COS25)
    lp = {i: oracle.SSAOParams(scenegen.ssao_kernel(max(1, S >> (i - 1)), seed=40 + i), 1.0, 0.02)
          for i in (1, 2, 3, 4)}
    return gb, mp, lp


def test_same_samples_everywhere_is_the_plain_pass_up_to_rounding():
    gb, mp, _ = setup()
    p = oracle.SSAOParams(scenegen.ssao_kernel(8), 1.0, 0.02)
    f = oracle.frame_fullres_levels(gb.depth, gb.normal, gb.focal, mp, {i: p for i in (1, 2, 3, 4)})
    plain = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, p)
    # c a + c (1 - a) = c up to two roundings per level
    assert np.abs(f.out - plain).max() <= 4e-7
    f64 = oracle.frame_fullres_levels(gb.depth.astype(np.float64), gb.normal.astype(np.float64), gb.focal, mp,
                                      {i: p for i in (1, 2, 3, 4)}, dtype=np.float64)
    plain64 = oracle.ssao_plain(gb.depth.astype(np.float64), gb.normal.astype(np.float64), gb.focal, p,
                                dtype=np.float64)
    assert np.abs(f64.out - plain64).max() <= 1e-15


def test_exact_regions():
    """Where alpha_1 = 1 the pixel is level 1's full-res value; where every
    finer alpha is 0 it is the coarsest level's value, bit for bit."""
    gb, mp, lp = setup(W=256, H=192, boxes=6)
    f = oracle.frame_fullres_levels(gb.depth, gb.normal, gb.focal, mp, lp)
    H, W = gb.depth.shape
    pyr = f.pyramid
    al = {i: oracle.upsampled_alpha(W, H, i, mp.weight[i - 1], pyr.alpha[i], pyr.stencil[i]) for i in (1, 2, 3)}
    c1 = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, lp[1])
    c4 = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, lp[4])
    top = al[1] == 1
    none = (al[1] == 0) & (al[2] == 0) & (al[3] == 0)
    assert top.any() and none.any()
    assert np.array_equal(f.out[top], c1[top])
    assert np.array_equal(f.out[none], c4[none])


def test_brute_force_blend_on_a_tiny_frame():
    gb, mp, lp = setup(W=32, H=24, seed=5, cam=6, S=4)
    f = oracle.frame_fullres_levels(gb.depth, gb.normal, gb.focal, mp, lp)
    H, W = gb.depth.shape
    pyr = f.pyramid
    c = {i: oracle.ssao_plain(gb.depth, gb.normal, gb.focal, lp[i]) for i in (1, 2, 3, 4)}
    F = np.float32
    for y in range(H):
        for x in range(W):
            out = F(c[4][y, x])
            for i in (3, 2, 1):
                s = 1 << (i - 1)
                Si, ai = pyr.stencil[i].astype(bool), pyr.alpha[i]
                Hi, Wi = Si.shape
                u = F(F(F(x) + F(0.5)) / F(s) - F(0.5))
                v = F(F(F(y) + F(0.5)) / F(s) - F(0.5))
                x0, y0 = math.floor(u), math.floor(v)
                fx, fy = F(u - F(x0)), F(v - F(y0))
                xs = [min(max(x0, 0), Wi - 1), min(max(x0 + 1, 0), Wi - 1)]
                ys = [min(max(y0, 0), Hi - 1), min(max(y0 + 1, 0), Hi - 1)]
                wts = [F(F(1 - fx) * F(1 - fy)), F(fx * F(1 - fy)), F(F(1 - fx) * fy), F(fx * fy)]
                tp = [(ys[0], xs[0]), (ys[0], xs[1]), (ys[1], xs[0]), (ys[1], xs[1])]
                den, A = F(0), F(0)
                for wt, (ty, tx) in zip(wts, tp):
                    if Si[ty, tx]:
                        den = F(den + wt)
                    A = F(A + F(wt * F(ai[ty, tx])))
                a = min(F(A * F(mp.weight[i - 1])), F(1)) if den > 0 else F(0)
                out = F(F(F(c[i][y, x]) * a) + F(out * F(1 - a)))
            assert out == f.out[y, x], (y, x)


def test_merge_alpha_agrees():
    """upsampled_alpha is the alpha the merge blends with: a merge of
    constant sub-images 1 (level i) over 0 (coarser) returns it."""
    gb, mp, _ = setup()
    H, W = gb.depth.shape
    E = oracle.edge_image(gb.depth, gb.normal, mp.depth_ratio, mp.normal_cos)
    pyr = oracle.build_pyramid(E, mp)
    for i in (1, 2, 3):
        lv = [i, 4]
        lo = {i: np.ones(pyr.stencil[i].shape, np.float32), 4: np.zeros(pyr.stencil[4].shape, np.float32)}
        m = oracle.upsample_merge(W, H, lv, {i: mp.weight[i - 1], 4: 1.0}, pyr.alpha, pyr.stencil, lo)
        a = oracle.upsampled_alpha(W, H, i, mp.weight[i - 1], pyr.alpha[i], pyr.stencil[i])
        assert np.array_equal(m, a)
