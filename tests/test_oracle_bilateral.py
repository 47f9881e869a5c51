"""Pins of the oracle's bilateral blur of SSAO sub-images (Sec. 4.1) against
facts that do not depend on its code: a brute-force per-texel loop on tiny
inputs, the normalised binomial filter from scipy where depth is flat and
every texel is rendered, closed forms at a depth step and at isolated
texels, and the frame-level contract (undefined texels never leak in)."""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
import scenegen

BP = oracle.BilateralParams


def brute(c, z, stencil, R, drel):
    """Per texel, per tap, in window order, Python floats rounded to float32
    after every operation."""
    f = np.float32
    Hi, Wi = z.shape
    b = [f(math.comb(2 * R, k) / 4 ** R) for k in range(2 * R + 1)]
    out = c.astype(np.float32).copy()

    def ok(y, x):
        return (stencil is None or stencil[y, x]) and np.isfinite(z[y, x]) and z[y, x] > 0

    for y in range(Hi):
        for x in range(Wi):
            if not ok(y, x):
                continue
            zp = f(z[y, x])
            d = f(f(drel) * zp)
            num, den = f(0), f(0)
            for dy in range(-R, R + 1):
                for dx in range(-R, R + 1):
                    qy, qx = y + dy, x + dx
                    if not (0 <= qy < Hi and 0 <= qx < Wi) or not ok(qy, qx):
                        continue
                    t = f(f(abs(f(z[qy, qx] - zp))) / d)
                    wz = max(f(f(1) - t), f(0))
                    w = f(f(b[dy + R] * b[dx + R]) * wz)
                    num = f(num + f(w * f(c[qy, qx])))
                    den = f(den + w)
            out[y, x] = f(num / den)
    return out


@pytest.mark.parametrize("R", [1, 2])
def test_matches_brute_force_on_tiny_inputs(R):
    rng = np.random.default_rng(5 + R)
    Hi, Wi = 7, 9
    z = (5 + rng.random((Hi, Wi)) * 0.6).astype(np.float32)
    z[2, 3] = np.inf         # background texel
    z[5, 1] = 0.0            # invalid depth
    c = rng.random((Hi, Wi)).astype(np.float32)
    st = rng.random((Hi, Wi)) < 0.7
    c[~st] = np.nan          # values the level did not render
    got = oracle.bilateral_level(c, z, st, BP(radius=R, depth_rel=0.05))
    ref = brute(c, z, st, R, 0.05)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[st], ref[st])


def test_flat_depth_full_stencil_is_the_normalised_binomial_filter():
    """Equal depths give range weight 1, so the blur is the binomial filter
    normalised by the weight inside the image (scipy convolution with zero
    padding, divided by the convolved indicator)."""
    rng = np.random.default_rng(3)
    c = rng.random((20, 31)).astype(np.float64)
    z = np.full(c.shape, 4.0)
    got = oracle.bilateral_level(c, z, None, BP(radius=2), dtype=np.float64)
    k1 = np.array([1, 4, 6, 4, 1], float) / 16
    k = np.outer(k1, k1)
    num = ndimage.convolve(c, k, mode="constant", cval=0.0)
    den = ndimage.convolve(np.ones_like(c), k, mode="constant", cval=0.0)
    assert np.allclose(got, num / den, rtol=0, atol=1e-14)
    # interior texels: the full window, weights summing to 1
    assert np.allclose(got[2:-2, 2:-2], ndimage.convolve(c, k)[2:-2, 2:-2], atol=1e-14)


def test_binomial_weights():
    assert oracle.binomial_weights(1).tolist() == [0.25, 0.5, 0.25]
    assert oracle.binomial_weights(2).tolist() == [0.0625, 0.25, 0.375, 0.25, 0.0625]


def test_depth_step_separates_the_two_sides_exactly():
    """Two flat regions whose depths differ by more than the tolerance do
    not mix: constant values on each side come out unchanged."""
    z = np.ones((12, 16), np.float32) * 10
    z[:, 8:] = 12  # 20 % deeper: range weight 0 across the step
    c = np.where(z == 10, np.float32(0.25), np.float32(0.75)).astype(np.float32)
    got = oracle.bilateral_level(c, z, None, BP(radius=2, depth_rel=0.05))
    assert np.array_equal(got, c)


def test_range_weight_closed_form():
    """Centre texel with one neighbour at depth z (1 + t d) and everything
    else outside the stencil: result = (b0^2 c0 + b0 b1 (1 - t) c1) /
    (b0^2 + b0 b1 (1 - t))."""
    z = np.full((5, 5), 8.0)
    z[2, 3] = 8.0 * (1 + 0.5 * 0.05)  # t = 0.5
    st = np.zeros((5, 5), bool)
    st[2, 2] = st[2, 3] = True
    c = np.zeros((5, 5))
    c[2, 2], c[2, 3] = 0.2, 0.6
    got = oracle.bilateral_level(c, z, st, BP(radius=1, depth_rel=0.05), dtype=np.float64)
    b0, b1 = 0.5, 0.25
    w1 = b0 * b1 * 0.5
    assert got[2, 2] == pytest.approx((b0 * b0 * 0.2 + w1 * 0.6) / (b0 * b0 + w1), abs=1e-15)


def test_isolated_and_background_texels_keep_their_value():
    rng = np.random.default_rng(8)
    z = (3 + rng.random((9, 9))).astype(np.float32)
    z[4, 4] = np.inf
    c = rng.random((9, 9)).astype(np.float32)
    st = np.zeros((9, 9), bool)
    st[0, 0] = st[4, 4] = st[8, 8] = True
    got = oracle.bilateral_level(c, z, st, BP(radius=2))
    for y, x in ((0, 0), (4, 4), (8, 8)):
        assert got[y, x] == c[y, x]


def test_frame_blur_reads_only_rendered_texels():
    """Whole SSAO frames with the blur: finite everywhere (sub-image values
    outside the stencils are NaN in the oracle, so a leak would show), equal
    to the unblurred frame when no level is chosen, and different from it
    otherwise."""
    sc = scenegen.make_scene(4, 30, 8)
    W, H = 128, 96
    gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(3), W, H)
    t = scenegen.TABLE1["ssao"]
    mp = oracle.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"])
    op = oracle.SSAOParams(scenegen.ssao_kernel(8), 1.0, 0.02)
    base = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp, op)
    off = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp, op, bilateral=BP(levels=0))
    assert np.array_equal(base.out, off.out)
    on = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp, op, bilateral=BP(levels=0b1111))
    assert np.isfinite(on.out).all() and not np.array_equal(on.out, base.out)
    for i in (1, 2, 3):
        st = on.pyramid.stencil[i] != 0
        assert np.isfinite(on.level_out[i][st]).all()
        assert np.isnan(on.level_out[i][~st]).all()
    # occlusion stays a fraction
    assert on.out.min() >= 0 and on.out.max() <= 1
