"""The seeded input generator (not part of the method)."""
import math

import numpy as np

import scenegen


def test_splitmix64_reference_outputs():
    # splitmix64 (Steele, Lea, Flood 2014) from state 0: published first outputs
    g = scenegen.SplitMix64(0)
    assert g.next() == 0xE220A8397B1DCDAF
    assert g.next() == 0x6E789E6AA1B965F4
    assert g.next() == 0x06C45D188009454F


def test_focal_lengths():
    # f = (H / 2) / tan(30 deg), rounded to FP32
    for h, f in [(256, 221.70250), (1080, 935.30743), (2160, 1870.6149)]:
        assert abs(float(scenegen.focal_px(h)) - f) < 1e-3


def test_ground_depth_matches_closed_form():
    s = scenegen.make_scene(5, 0, 0)
    v = scenegen.orbit_view(2)
    gb = scenegen.render_gbuffer(s, v, 64, 48)
    f = float(gb.focal)
    for (x, y) in [(0, 47), (31, 30), (63, 40)]:
        dv = np.array([(x + 0.5 - 32) / f, (24 - (y + 0.5)) / f, -1.0])
        d = v[3:6] * dv[0] + v[6:9] * dv[1] + v[9:12] * dv[2]
        t = -v[1] / d[1]
        assert abs(gb.depth[y, x] - t) <= 1e-6 * t
        # ground normal (0, 1, 0) in view space = (right.y, up.y, back.y)
        assert np.allclose(gb.normal[:, y, x], [v[4], v[7], v[10]], atol=1e-7)


def test_gbuffer_deterministic_and_unit_normals():
    s = scenegen.make_scene(3, 40, 10)
    a = scenegen.render_gbuffer(s, scenegen.orbit_view(1), 128, 96)
    b = scenegen.render_gbuffer(s, scenegen.orbit_view(1), 128, 96)
    assert np.array_equal(a.depth, b.depth) and np.array_equal(a.normal, b.normal)
    nn = (a.normal.astype(np.float64) ** 2).sum(0)
    assert np.all(np.abs(nn - 1) < 1e-6)
    assert np.isfinite(a.depth).all()  # the orbit cameras see no background


def test_ssao_kernel_above_tangent_plane():
    for S in (16, 32, 64, 256):
        k = scenegen.ssao_kernel(S)
        assert k.shape == (S, 3) and k.dtype == np.float32
        assert (k[:, 2] >= 0.0099).all()
        ln = np.sqrt((k.astype(np.float64) ** 2).sum(1))
        assert (ln <= 1.0 + 1e-6).all() and (ln >= 0.1 - 1e-6).all()


def test_disk_samples_in_unit_disk():
    d = scenegen.disk_samples(32, 7)
    assert (np.hypot(d[:, 0], d[:, 1]) <= 1.0 + 1e-6).all()


def test_table1_presets_match_paper(request):
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))
    for eff in ("ssao", "shadow", "ssgi"):
        for i in range(4):
            if g[eff]["sigma2"][i] is None:
                continue
            assert scenegen.TABLE1[eff]["sigma2"][i] == g[eff]["sigma2"][i]
            assert scenegen.TABLE1[eff]["weight"][i] == g[eff]["weight"][i]
