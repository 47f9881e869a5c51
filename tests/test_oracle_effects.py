"""Pins of the oracle's soft-shadow and indirect-light estimators and of the
whole frame: the lit and fully blocked special cases, a half-plane blocker
whose PCF visibility is counted in float64, the shadow-edge image, SSGI's
zero cases, the all-finest identity, and the quality bound multi-res vs
plain."""
import math

import numpy as np
import pytest

import oracle
import scenegen

F32 = np.float32


def identity_light(size, focal, sm, bias=0.05, near=1.0, lsize=0.5):
    M = np.zeros((3, 4), F32)
    M[0, 0] = M[1, 1] = M[2, 2] = 1.0
    return oracle.ShadowParams(sm, M, F32(focal), F32(lsize), F32(near), F32(bias),
                               scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12))


def test_ground_only_fully_lit():
    s = scenegen.make_scene(2, 0, 0)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(1), 192, 108)
    si = scenegen.render_shadow_inputs(s, gb.view, 512)
    p = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size,
                            si.light_near, F32(0.05), scenegen.disk_samples(16, 11),
                            scenegen.disk_samples(32, 12))
    assert (oracle.hard_shadow(gb.depth, gb.focal, 1, p) == 0).all()
    assert (oracle.pcss_level(gb.depth, gb.focal, 1, p) == 1).all()


def test_infinite_blocker_plane_fully_dark():
    H, W = 16, 24
    d = np.full((H, W), 10.0, F32)
    sm = np.full((64, 64), 5.0, F32)
    p = identity_light(64, 30.0, sm)
    assert (oracle.pcss_level(d, F32(30.0), 1, p) == 0).all()
    assert (oracle.hard_shadow(d, F32(30.0), 1, p) == 1).all()


def test_half_plane_blocker_pcf_count():
    """Receiver plane z = 10 seen by a light at the camera (identity
    transform, same focal, map = image): texel columns < c block at depth 3.
    Blockers all have depth 3, so d_b = 3 exactly and the PCF radius is
    R_f = l (10 - 3) / (3 * 10); visibility = share of PCF taps landing at
    columns >= c (taps counted in float64, ambiguous texels skipped)."""
    H = W = 64
    f = 40.0
    c = 32
    d = np.full((H, W), 10.0, F32)
    sm = np.full((H, W), np.inf, F32)
    sm[:, :c] = 3.0
    p = identity_light(W, f, sm, bias=0.05, near=1.0, lsize=0.5)
    vis = oracle.pcss_level(d, F32(f), 1, p)
    l = f * 0.25
    Rs = l * (10 - 1) / (10 * 1)
    Rf = l * (10 - 3) / (3 * 10)
    bd = p.blocker_disk.astype(np.float64)
    pd = p.pcf_disk.astype(np.float64)
    checked = 0
    for y in range(H):
        for x in range(W):
            su, sv = x + 0.5, y + 0.5
            ub = su + Rs * bd[:, 0]
            up = su + Rf * pd[:, 0]
            if np.min(np.abs(ub - np.round(ub))) < 1e-4 or np.min(np.abs(up - np.round(up))) < 1e-4:
                continue
            nblk = int((np.clip(np.floor(ub), 0, W - 1) < c).sum())
            if nblk == 0:
                exp = 1.0
            else:
                exp = float((np.clip(np.floor(up), 0, W - 1) >= c).sum()) / 32
            assert vis[y, x] == F32(exp), (x, y, vis[y, x], exp)
            checked += 1
    assert checked > 0.9 * H * W
    assert vis.min() == 0 and vis.max() == 1 and ((vis > 0) & (vis < 1)).any()


def test_shadow_edges_of_hard_bits():
    h = np.zeros((6, 8), np.uint8)
    h[:, 4:] = 1
    d = np.full((6, 8), 5.0, F32)
    E = oracle.shadow_edges(h, d)
    exp = np.zeros_like(E)
    exp[:, 3:5] = 1
    assert np.array_equal(E, exp)


def ssgi_params(S=32, r=2.0):
    return oracle.SSGIParams(scenegen.ssao_kernel(S), r, 0.02)


def test_ssgi_black_colour_is_zero(scene256):
    s, gb = scene256
    col = np.zeros((3, 256, 256), np.float16)
    out = oracle.ssgi_level(gb.depth, gb.normal, col, gb.focal, 1, ssgi_params())
    assert (out == 0).all()


def test_ssgi_plane_is_zero():
    d = np.full((16, 16), 10.0, F32)
    n = np.zeros((3, 16, 16), F32)
    n[2] = 1
    col = np.ones((3, 16, 16), np.float16)
    assert (oracle.ssgi_level(d, n, col, F32(20.0), 1, ssgi_params()) == 0).all()


def test_ssgi_only_where_occluded(scene256):
    s, gb = scene256
    col = scenegen.lambert_color(s, gb)
    g = oracle.ssgi_level(gb.depth, gb.normal, col, gb.focal, 1, ssgi_params(16, 0.5))
    a = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02))
    assert (g >= 0).all()
    assert ((g.max(0) > 0) <= (a > 0)).all()
    assert (g.max(0) > 0).any()


def mp3():
    return oracle.MaskParams(num_levels=3, level_enable=0b111, sigma2=(0.924, 1.848, 0.0),
                             weight=(100.0, 50.0, 1.0))


def test_all_finest_reproduces_plain_bitwise(scene256):
    """Forced S_1 = 1, a_1 = 1 gives alpha_1 = 1, so Eq. 1 returns c_1, and c_1
    is the same estimator at level 1 as the naive full-resolution pass."""
    s, gb = scene256
    p = oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02)
    plain = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, p)
    levels = [1, 2, 3]
    st = {1: np.ones((256, 256), np.uint8), 2: np.ones((128, 128), np.uint8), 3: np.ones((64, 64), np.uint8)}
    al = {1: np.ones((256, 256), F32), 2: np.ones((128, 128), F32)}
    lo = {}
    for i in levels:
        lo[i] = oracle.ssao_level(oracle.level_sample(gb.depth, i), oracle.level_sample(gb.normal, i),
                                  gb.focal, i, p, None if i == 3 else st[i])
    out = oracle.upsample_merge(256, 256, levels, {1: 100, 2: 50, 3: 1}, al, st, lo)
    assert np.array_equal(out, plain)


def test_multires_quality_bound(scene256):
    s, gb = scene256
    p = oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02)
    fr = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp3(), p)
    plain = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, mp3(), p, multires=False).out
    assert np.abs(fr.out - plain).mean() <= 0.01
    assert np.isfinite(fr.out).all()
