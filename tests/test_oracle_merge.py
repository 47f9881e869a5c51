"""Pins of the oracle's upsample-and-merge (Sec. 3.3, Sec. 4.2, Eq. 1):
torch's bilinear resize (texel-centre convention, clamped) for the coarsest
level, closed forms of Eq. 1, reproduction of linear ramps, and that values
outside a level's stencil never reach the output."""
import numpy as np
import pytest
import torch

import oracle

F32 = np.float32


def setup(W=64, H=48, levels=(1, 2, 3, 4), seed=0):
    rng = np.random.default_rng(seed)
    L = levels[-1]
    st, al, c = {}, {}, {}
    for i in levels:
        s = 1 << (i - 1)
        Hi, Wi = H // s, W // s
        st[i] = np.ones((Hi, Wi), np.uint8) if i == L else (rng.random((Hi, Wi)) < 0.4).astype(np.uint8)
        if i != L:
            al[i] = np.where(st[i] == 1, rng.random((Hi, Wi)).astype(F32) * F32(0.05), F32(0))
        c[i] = rng.random((Hi, Wi)).astype(F32)
    return st, al, c


def test_coarsest_level_is_torch_bilinear():
    W, H = 64, 48
    rng = np.random.default_rng(3)
    for L in (2, 3, 4):
        s = 1 << (L - 1)
        cL = rng.random((H // s, W // s)).astype(F32)
        st = {L: np.ones_like(cL, np.uint8)}
        out = oracle.upsample_merge(W, H, [L], {L: 1.0}, {}, st, {L: cL})
        ref = torch.nn.functional.interpolate(torch.from_numpy(cL.astype(np.float64))[None, None],
                                              size=(H, W), mode="bilinear", align_corners=False)[0, 0]
        assert np.abs(out - ref.numpy()).max() < 1e-6


def test_alpha_one_selects_finest():
    st, al, c = setup()
    st[1][:] = 1
    al[1][:] = 1.0  # alpha = min(1 * 100, 1) = 1
    out = oracle.upsample_merge(64, 48, [1, 2, 3, 4], {1: 100, 2: 50, 3: 20, 4: 1}, al, st, c)
    assert np.array_equal(out, c[1])


def test_alpha_zero_passes_coarser():
    st, al, c = setup()
    for i in (1, 2, 3):
        al[i][:] = 0.0
    a = oracle.upsample_merge(64, 48, [1, 2, 3, 4], {1: 100, 2: 50, 3: 20, 4: 1}, al, st, c)
    b = oracle.upsample_merge(64, 48, [4], {4: 1}, {}, {4: st[4]}, {4: c[4]})
    assert np.array_equal(a, b)


def test_two_level_eq1_closed_form():
    W, H = 32, 16
    c1 = np.full((H, W), 0.8, F32)
    c2 = np.full((H // 2, W // 2), 0.2, F32)
    st = {1: np.ones((H, W), np.uint8), 2: np.ones((H // 2, W // 2), np.uint8)}
    for a, w in [(0.003, 100.0), (0.02, 50.0), (0.5, 1.0)]:
        al = {1: np.full((H, W), a, F32)}
        out = oracle.upsample_merge(W, H, [1, 2], {1: w, 2: 1}, al, st, {1: c1, 2: c2})
        alpha = min(float(F32(a)) * w, 1.0)
        assert np.allclose(out, 0.8 * alpha + 0.2 * (1 - alpha), atol=1e-6)


def test_constant_levels_give_constant():
    st, al, c = setup()
    for i in c:
        c[i][:] = 0.375
    out = oracle.upsample_merge(64, 48, [1, 2, 3, 4], {1: 100, 2: 50, 3: 20, 4: 1}, al, st, c)
    assert np.abs(out - 0.375).max() <= 2 * np.spacing(F32(0.375))


@pytest.mark.parametrize("level", [2, 3, 4])
def test_linear_ramp_reproduced(level):
    W, H = 64, 48
    s = 1 << (level - 1)
    Wi, Hi = W // s, H // s
    # texel centre of level texel x in full-res pixel coordinates: s (x + 0.5) - 0.5
    xc = s * (np.arange(Wi) + 0.5) - 0.5
    yc = s * (np.arange(Hi) + 0.5) - 0.5
    c = (0.01 * xc[None, :] + 0.02 * yc[:, None] + 0.1).astype(F32)
    out = oracle.upsample_merge(W, H, [level], {level: 1}, {}, {level: np.ones((Hi, Wi), np.uint8)}, {level: c})
    X = np.arange(W)[None, :]
    Y = np.arange(H)[:, None]
    ref = 0.01 * X + 0.02 * Y + 0.1
    lo = s // 2
    inner = (slice(lo, H - lo), slice(lo, W - lo))
    assert np.abs(out[inner] - ref[inner]).max() < 1e-5


def test_undefined_texels_never_leak():
    st, al, c = setup(seed=5)
    for i in (1, 2, 3):
        c[i] = np.where(st[i] == 1, c[i], np.nan).astype(F32)
    out = oracle.upsample_merge(64, 48, [1, 2, 3, 4], {1: 100, 2: 50, 3: 20, 4: 1}, al, st, c)
    assert np.isfinite(out).all()


def test_mask_normalised_taps():
    # level 2 with only the left texel column defined: pixels between a defined
    # and an undefined texel take the defined value exactly
    W, H = 8, 4
    st2 = np.zeros((2, 4), np.uint8)
    st2[:, 1] = 1
    c2 = np.full((2, 4), np.nan, F32)
    c2[:, 1] = 0.6
    al2 = np.where(st2 == 1, F32(1.0), F32(0)).astype(F32)
    st3 = np.ones((1, 2), np.uint8)
    c3 = np.zeros((1, 2), F32)
    out = oracle.upsample_merge(W, H, [2, 3], {2: 1000, 3: 1}, {2: al2}, {2: st2, 3: st3}, {2: c2, 3: c3})
    # pixel x = 3 sits between texels 1 and 2 of level 2 (fx = 0.25): only texel 1 counts
    assert abs(out[1, 3] - 0.6 * min(0.75 * 1000, 1)) < 1e-7
    assert out[1, 7] == 0.0  # no defined tap: alpha = 0, coarser level passes
