"""The oracle's frame split into row bands (the CPU baseline's mode B) gives
oracle.frame's image bit for bit: multi-resolution with Table 1's SSAO
masks and the naive pass, for band splits down to one coarsest texel row
and through the forked process pool the baseline uses."""
import multiprocessing

import numpy as np
import pytest

import oracle
import scenegen
from oracle import timing


@pytest.fixture(scope="module")
def inputs():
    s = scenegen.make_scene(3, 40, 10)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(2), 320, 200)
    t = scenegen.TABLE1["ssao"]
    mp = oracle.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"])
    op = oracle.SSAOParams(scenegen.ssao_kernel(8), 1.0, 0.02)
    ref = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp, op).out
    ref_plain = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp, op, multires=False).out
    return gb, mp, op, ref, ref_plain


def _banded(gb, mp, op, multires, n):
    align = timing.band_context(mp)[0] if multires else 1
    parts = [timing.frame_rows(gb.depth, gb.normal, gb.focal, mp, op, multires, a, b)
             for a, b in timing.bands(gb.depth.shape[0], n, align)]
    return np.concatenate(parts, axis=0)


def test_band_context_covers_the_blur_reach():
    t = scenegen.TABLE1["ssao"]
    mp = oracle.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"])
    # level 3: radius ceil(3 sqrt(3.696)) = 6 texels of 4 rows, plus two texels
    assert timing.band_context(mp) == (8, 32)


@pytest.mark.parametrize("n", [1, 2, 5, 25])
def test_multires_bands_equal_the_frame(inputs, n):
    gb, mp, op, ref, _ = inputs
    got = _banded(gb, mp, op, True, n)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 3, 17])
def test_plain_bands_equal_the_frame(inputs, n):
    gb, mp, op, _, ref_plain = inputs
    assert np.array_equal(_banded(gb, mp, op, False, n), ref_plain)


def test_bands_cover_every_row_once():
    for H, n, a in ((200, 25, 8), (2160, 16, 8), (1080, 16, 8), (7, 3, 1), (8, 5, 8)):
        b = timing.bands(H, n, a)
        assert b[0][0] == 0 and b[-1][1] == H
        assert all(x1 == y0 for (_, x1), (y0, _) in zip(b[:-1], b[1:]))
        assert all(y0 % a == 0 and y1 > y0 for y0, y1 in b)


def test_too_little_context_is_seen(inputs, monkeypatch):
    # a band computed without the blur's reach differs near its cut: the
    # identity above is not reached by accident
    gb, mp, op, ref, _ = inputs
    monkeypatch.setattr(timing, "band_context", lambda mp_: (8, 0))
    got = _banded(gb, mp, op, True, 5)
    assert not np.array_equal(got, ref)


def test_forked_pool(inputs):
    gb, mp, op, ref, ref_plain = inputs
    timing._INPUT = (gb.depth, gb.normal, gb.focal, mp, op)
    try:
        with multiprocessing.get_context("fork").Pool(3) as pool:
            assert np.array_equal(timing.frame_bands(pool, 4, True), ref)
            assert np.array_equal(timing.frame_bands(pool, 4, False), ref_plain)
    finally:
        timing._INPUT = None
