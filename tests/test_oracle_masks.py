"""Pins of the oracle's mask creation (Sec. 3.1, Table 1, Sec. 4.1) against
facts that do not come from the oracle itself: hand-built G-buffers with known
edges, the closed form of a plane's depth second difference, scipy's Gaussian
filter and maximum filter, and brute-force loops on tiny images."""
import math

import numpy as np
import pytest
import scipy.ndimage as nd

import oracle
import scenegen
from conftest import COS25

F32 = np.float32


def flat(H, W, z=10.0):
    d = np.full((H, W), z, F32)
    n = np.zeros((3, H, W), F32)
    n[2] = 1.0
    return d, n


def test_fronto_parallel_plane_has_no_edges():
    d, n = flat(16, 20)
    assert oracle.edge_image(d, n, 0.05, COS25).sum() == 0


def test_depth_step_marks_both_sides_only():
    d, n = flat(12, 16)
    d[:, 8:] = 20.0
    E = oracle.edge_image(d, n, 0.05, COS25)
    # second difference is +10 at x=7 and -10 at x=8, 0 elsewhere
    expect = np.zeros_like(E)
    expect[:, 7:9] = 1
    assert np.array_equal(E, expect)
    # the same step along y
    E = oracle.edge_image(d.T.copy(), np.ascontiguousarray(n.transpose(0, 2, 1)), 0.05, COS25)
    assert np.array_equal(E, expect.T)


def test_depth_threshold_is_relative_and_strict():
    d, n = flat(3, 9)
    # a kink: z = 10 everywhere except one pixel raised by delta
    for delta, edge in [(0.24, False), (0.26, True)]:
        dd = d.copy()
        dd[1, 4] = F32(10.0 - delta)
        # second difference at (1,4) is 2 delta relative to ~10: > 0.05*z iff
        # 2 delta > 0.05 (10 - delta), i.e. delta > 0.2439
        E = oracle.edge_image(dd, n, 0.05, COS25)
        assert bool(E[1, 4]) == edge


def crease(angle_deg, H=6, W=16):
    d, n = flat(H, W)
    a = math.radians(angle_deg)
    n[0, :, 8:] = F32(math.sin(a))
    n[2, :, 8:] = F32(math.cos(a))
    return d, n


def test_normal_crease_threshold_25_degrees():
    d, n = crease(30.0)
    E = oracle.edge_image(d, n, 0.05, COS25)
    expect = np.zeros_like(E)
    expect[:, 7:9] = 1
    assert np.array_equal(E, expect)
    d, n = crease(20.0)
    assert oracle.edge_image(d, n, 0.05, COS25).sum() == 0


def test_normal_tie_is_not_an_edge():
    d, n = flat(1, 2)
    # dot((0,0,1), (s,0,c)) = ((0 s) + (0 0)) + (1 c) = c exactly
    n[0, 0, 1] = F32(math.sqrt(1 - float(COS25) ** 2))
    n[2, 0, 1] = COS25
    assert oracle.edge_image(d, n, 0.05, COS25).sum() == 0
    n[2, 0, 1] = np.nextafter(COS25, F32(0))
    assert oracle.edge_image(d, n, 0.05, COS25).sum() == 2


def test_background_rules():
    d, n = flat(5, 5)
    d[2, 2] = np.inf
    d[0, 0] = 0.0
    E = oracle.edge_image(d, n, 0.05, COS25)
    assert E[2, 2] == 0 and E[0, 0] == 0
    for (y, x) in [(1, 2), (3, 2), (2, 1), (2, 3), (0, 1), (1, 0)]:
        assert E[y, x] == 1


@pytest.mark.parametrize("W,H", [(256, 256), (1920, 1080)])
def test_ground_plane_closed_form_is_edge_free(W, H):
    """On a plane 1/z is affine in screen space, so the relative second
    difference along an axis is 2 q^2 / (1 - q^2) with q = (d(1/z)/dpix)/(1/z);
    at the orbit cameras it stays far below 0.05, so E must be empty."""
    s = scenegen.make_scene(1, 0, 0)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(0), W, H)
    w = 1.0 / gb.depth.astype(np.float64)
    q = max((np.abs(np.diff(w, axis=0)) / w[:-1]).max(), (np.abs(np.diff(w, axis=1)) / w[:, :-1]).max())
    assert 2 * q * q / (1 - q * q) < 0.05 / 50
    E = oracle.edge_image(gb.depth, gb.normal, 0.05, COS25)
    assert E.sum() == 0
    mp = oracle.MaskParams(num_levels=4)
    pyr = oracle.build_pyramid(E, mp)
    # an edge-free plane maps wholly to the coarsest level
    assert (pyr.level_map == 4).all()
    assert all(len(pyr.worklist[i]) == 0 for i in (1, 2, 3))


def test_or_pool_brute_force():
    rng = np.random.default_rng(0)
    E = (rng.random((16, 24)) < 0.05).astype(np.uint8)
    for s in (1, 2, 4, 8):
        P = oracle.or_pool(E, s)
        for y in range(16 // s):
            for x in range(24 // s):
                assert P[y, x] == int(any(E[s * y + dy, s * x + dx] for dy in range(s) for dx in range(s)))


def test_gaussian_weights_closed_form_values():
    # normalised Gaussian over radius ceil(3 sigma): g0..g3 for sigma^2 = 0.924
    g = oracle.gaussian_weights(0.924)
    assert len(g) == 7
    assert np.allclose(g[3:], [0.415085, 0.241618, 0.047655, 0.003185], atol=2e-6)
    assert len(oracle.gaussian_weights(1.848)) == 11
    assert len(oracle.gaussian_weights(3.696)) == 13
    assert np.isclose(oracle.gaussian_weights(3.696)[6], 0.207643, atol=2e-6)
    assert list(oracle.gaussian_weights(0.0)) == [1.0]


@pytest.mark.parametrize("sigma2", [0.924, 1.848, 3.696])
def test_blur_matches_scipy_gaussian_filter(sigma2):
    rng = np.random.default_rng(1)
    E = (rng.random((40, 56)) < 0.03).astype(np.uint8)
    r = oracle.blur_radius(sigma2)
    g = oracle.gaussian_weights(sigma2)
    from oracle.masks import blur
    a = blur(E, g)
    ref = nd.gaussian_filter(E.astype(np.float64), math.sqrt(float(F32(sigma2))), mode="constant",
                             cval=0.0, radius=r)
    assert np.abs(a - ref).max() < 2e-7


def test_isolated_edge_peak_and_straight_line_peak():
    for i, (s2, peak) in enumerate([(0.924, 0.1723), (1.848, 0.0861), (3.696, 0.0431)]):
        E = np.zeros((31, 31), np.uint8)
        E[15, 15] = 1
        from oracle.masks import blur
        a = blur(E, oracle.gaussian_weights(s2))
        assert abs(a.max() - peak) < 1e-4 and a[15, 15] == a.max()
    E = np.zeros((31, 31), np.uint8)
    E[:, 15] = 1
    a = blur(E, oracle.gaussian_weights(0.924))
    assert abs(a[15, 15] - 0.415085) < 1e-5


def table_mp(effect, levels=4):
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else (1 << levels) - 1
    return oracle.MaskParams(num_levels=levels, level_enable=en, sigma2=t["sigma2"], weight=t["weight"])


def random_edges(H, W, seed, p=0.01):
    rng = np.random.default_rng(seed)
    return (rng.random((H, W)) < p).astype(np.uint8)


@pytest.mark.parametrize("effect", ["ssao", "shadow", "ssgi"])
def test_stencil_is_chebyshev_dilation_of_pooled_edges(effect):
    """S_i = (a_i > 0) equals the integer max filter of the OR-pooled edges
    with window 2 r_i + 1 (no float blur involved)."""
    mp = table_mp(effect)
    E = random_edges(64, 96, 3)
    pyr = oracle.build_pyramid(E, mp)
    for i in pyr.levels[:-1]:
        s = 1 << (i - 1)
        pooled = E.reshape(64 // s, s, 96 // s, s).max(axis=(1, 3))
        r = oracle.blur_radius(mp.sigma2[i - 1])
        dil = nd.maximum_filter(pooled, size=2 * r + 1, mode="constant", cval=0)
        assert np.array_equal(pyr.stencil[i], dil)
    assert (pyr.stencil[pyr.levels[-1]] == 1).all()


@pytest.mark.parametrize("effect", ["ssao", "shadow", "ssgi"])
def test_nesting_and_partition(effect):
    mp = table_mp(effect)
    E = random_edges(64, 96, 4, 0.004)
    pyr = oracle.build_pyramid(E, mp)
    lv = pyr.levels
    # nesting: every finer-level stencil texel lies inside the next coarser one
    for a, b in zip(lv[:-1], lv[1:]):
        k = 1 << (b - a)
        Sa, Sb = pyr.stencil[a], pyr.stencil[b]
        for y, x in zip(*np.nonzero(Sa)):
            assert Sb[y // k, x // k] == 1
    # partition: one level per pixel, the finest covering one (brute force)
    lm = pyr.level_map
    for y in range(0, 64, 3):
        for x in range(0, 96, 5):
            cover = [i for i in lv if pyr.stencil[i][y >> (i - 1), x >> (i - 1)]]
            assert lm[y, x] == min(cover)
    assert set(np.unique(lm)) <= set(lv)
    # quadtree consistency: a level-i block is wholly inside or outside {lm <= i}
    for i in lv:
        s = 1 << (i - 1)
        blk = (lm <= i).reshape(64 // s, s, 96 // s, s)
        assert np.all(blk.all(axis=(1, 3)) | ~blk.any(axis=(1, 3)))


def test_work_lists_row_major_brute_force():
    mp = table_mp("ssao")
    E = random_edges(32, 48, 5, 0.01)
    pyr = oracle.build_pyramid(E, mp)
    for i in pyr.levels[:-1]:
        S = pyr.stencil[i]
        bf = [y * S.shape[1] + x for y in range(S.shape[0]) for x in range(S.shape[1]) if S[y, x]]
        assert pyr.worklist[i].dtype == np.uint32
        assert pyr.worklist[i].tolist() == bf
    assert pyr.levels[-1] not in pyr.worklist


def test_level_sample_point():
    a = np.arange(64, dtype=np.float32).reshape(8, 8)
    assert oracle.level_sample(a, 1) is a
    assert oracle.level_sample(a, 2)[1, 2] == a[3, 5]
    assert oracle.level_sample(a, 4)[0, 0] == a[4, 4]


def test_foveate_disks_brute_force():
    """Pixels whose centre is clearly inside r_inner are on, clearly outside
    r_outer are off, and in between keep the edge image (distances in
    float64, pixels within 1e-3 of a circle skipped)."""
    rng = np.random.default_rng(5)
    E = (rng.random((40, 56)) < 0.3).astype(np.uint8)
    g = (21.3, 17.8, 6.5, 14.25)
    F = oracle.foveate(E, g)
    for y in range(40):
        for x in range(56):
            d = math.hypot(x + 0.5 - g[0], y + 0.5 - g[1])
            if abs(d - g[2]) < 1e-3 or abs(d - g[3]) < 1e-3:
                continue
            exp = 1 if d < g[2] else (0 if d > g[3] else E[y, x])
            assert F[y, x] == exp, (x, y)
    assert np.array_equal(oracle.foveate(E, None), E)


def test_foveated_pyramid_owner_levels():
    """The fovea is rendered at level 1 everywhere inside r_inner (minus one
    pixel for the disk's discretisation), the periphery beyond r_outer plus
    the largest blur footprint at the coarsest level."""
    W = H = 128
    E = np.zeros((H, W), np.uint8)
    mp = oracle.MaskParams(num_levels=4, level_enable=0xF, fovea=(64.0, 64.0, 20.0, 40.0))
    pyr = oracle.build_pyramid(oracle.foveate(E, mp.fovea), mp)
    yy, xx = np.mgrid[0:H, 0:W]
    d = np.hypot(xx + 0.5 - 64.0, yy + 0.5 - 64.0)
    assert (pyr.level_map[d < 19.0] == 1).all()
    reach = 40.0 + 8 * (6 + 1)  # outer radius + level-3 blur radius (6) + one texel, in pixels
    assert (pyr.level_map[d > reach] == 4).all()
