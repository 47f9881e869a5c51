"""GPU parity on the edge cases of Sec. 3.1's edge detection and on frames
with background, through the C ABI against the oracle, bit for bit.

A hand-built 256 x 128 G-buffer (width divisible by 128, so mr_frame takes
the compact path; the step entry points take the dense one) holds, on a
fronto-parallel plane at depth 10:
  * background regions of depth +inf, -inf, NaN, 0 and a negative depth;
  * a depth step (10 -> 20);
  * second differences exactly at the threshold (0.05f * 10 = 0.5: a tie,
    not an edge) and one ulp above it;
  * normal pairs whose dot product equals cos 25 deg exactly (a tie) and
    one ulp below it, and creases of 20 and 30 degrees;
  * depth noise (dense stencils).
The same inputs pin the oracle (tests/test_oracle_masks.py), so masks,
lists and frames must match it bit for bit.  A second case is a rendered
scene seen from a low camera, with sky (background) above the horizon, for
all three effects."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from listcheck import check_frame_lists
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

DEV = "cuda"
F32 = np.float32
COS25 = F32(math.cos(math.radians(25.0)))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def handmade():
    W, H = 256, 128
    d = np.full((H, W), 10.0, F32)
    n = np.zeros((3, H, W), F32)
    n[2] = 1.0
    # background of every kind
    d[4:12, 4:20] = np.inf
    d[4:12, 24:40] = -np.inf
    d[4:12, 44:60] = np.nan
    d[4:12, 64:80] = 0.0
    d[4:12, 84:100] = -3.0
    d[20:21, 120:121] = np.inf  # a single background pixel
    # a depth step
    d[20:40, 20:60] = 20.0
    # one raised pixel gives its 4-neighbours a second difference of exactly
    # (10 + 10.5) - 2 * 10 = 0.5 = 0.05f * 10 (a tie, not an edge) ...
    d[50, 101] = F32(10.5)
    d[61, 160] = F32(10.5)
    # ... and two ulps higher (one would be lost in 10 + z), a difference
    # just above the threshold
    d[52, 131] = np.nextafter(np.nextafter(F32(10.5), F32(11.0)), F32(11.0))
    # normal ties: dot((0,0,1), (s,0,c)) = c exactly
    s = F32(math.sqrt(1.0 - float(COS25) ** 2))
    n[0, 80, 30], n[2, 80, 30] = s, COS25                              # tie
    n[0, 84, 30], n[2, 84, 30] = s, np.nextafter(COS25, F32(0))        # one ulp below
    # creases of 20 and 30 degrees (columns 200.. and 230..)
    for ang, x0 in ((20.0, 200), (30.0, 230)):
        a = math.radians(ang)
        n[0, 90:110, x0:x0 + 8] = F32(math.sin(a))
        n[2, 90:110, x0:x0 + 8] = F32(math.cos(a))
    # depth noise: dense stencils
    rng = np.random.default_rng(5)
    d[100:128, 0:96] = (6.0 + 6.0 * rng.random((28, 96))).astype(F32)
    return d, n


def params(lib, effect="ssao"):
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0xF
    return lib.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=float(COS25))


def test_oracle_reading_of_the_handmade_cases():
    """What the oracle says about the hand-built cases (so the GPU
    comparison below is about the cases it claims to be)."""
    d, n = handmade()
    E = oracle.edge_image(d, n, 0.05, COS25)
    assert E[4:12, 4:20].sum() == 0 and E[4:12, 84:100].sum() == 0   # background is never an edge
    assert E[3, 10] == 1 and E[12, 10] == 1                           # geometry next to it is
    assert E[50, 101] == 1                                           # the raised pixel
    assert E[50, 100] == 0 and E[50, 102] == 0                       # ties along x
    assert E[49, 101] == 0 and E[51, 101] == 0                       # ties along y
    assert E[60, 160] == 0 and E[62, 160] == 0
    assert E[52, 130] == 1 and E[52, 132] == 1 and E[51, 131] == 1   # just above
    assert E[80, 30] == 0 and E[80, 29] == 0 and E[84, 30] == 1 and E[84, 29] == 1
    assert E[100, 200:208].sum() == 0 and E[100, 229] == 1 and E[100, 230] == 1


def test_handmade_masks_and_frame_bit_exact():
    d, n = handmade()
    log("[gpu] hand-built edge cases 256x128")
    K = scenegen.ssao_kernel(16)
    focal = F32(100.0)
    ref = oracle.frame("ssao", d, n, focal, params(oracle), oracle.SSAOParams(K, 1.0, 0.02))
    pyr = ref.pyramid
    dd, nn, kk = (torch.from_numpy(a).to(DEV) for a in (d, n, K))
    masks = mr.mr_build_masks(dd, nn, focal, params(mr))
    lo = mr.mr_eval_ssao(dd, nn, focal, kk, 1.0, 0.02, mp=params(mr), masks=masks)
    merged = mr.mr_upsample_merge(focal, params(mr), masks, lo)
    lm = torch.empty(d.shape, dtype=torch.uint8, device=DEV)
    fr = mr.FrameRunner("ssao", dd, nn, focal, params(mr), True, params=mr.ssao_params(kk, 1.0, 0.02), level_map=lm)
    fr()
    plain = mr.FrameRunner("ssao", dd, nn, focal, params(mr), False, params=mr.ssao_params(kk, 1.0, 0.02))()
    torch.cuda.synchronize()
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E)
    assert np.array_equal(masks.level_map.cpu().numpy(), pyr.level_map)
    assert np.array_equal(lm.cpu().numpy(), pyr.level_map)
    cnt = masks.count.cpu().numpy().view(np.uint32)
    for i in (1, 2, 3):
        assert np.array_equal(masks.alpha[i].cpu().numpy().view(np.uint32), pyr.alpha[i].view(np.uint32)), i
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i]), i
        nl = len(pyr.worklist[i])
        assert cnt[i - 1] == nl
        assert np.array_equal(masks.worklist[i][:nl].cpu().numpy().view(np.uint32), pyr.worklist[i]), i
    check_frame_lists(fr.lists(), pyr)
    for i in (1, 2, 3, 4):
        g = lo[i].cpu().numpy()
        sel = np.ones(g.shape, bool) if i == 4 else pyr.stencil[i].astype(bool)
        assert np.array_equal(g[sel], ref.level_out[i][sel]), i
    assert np.array_equal(merged.cpu().numpy(), ref.out)
    assert np.array_equal(fr.out.cpu().numpy(), ref.out)
    rp = oracle.ssao_plain(d, n, focal, oracle.SSAOParams(K, 1.0, 0.02))
    assert np.array_equal(plain.cpu().numpy(), rp)
    bg = ~(np.isfinite(d) & (d > 0))
    assert (ref.out[bg] == 0).all() and (rp[bg] == 0).all()


def sky_view():
    """A low camera looking level: the ground and objects below the
    horizon, background above it."""
    return scenegen.look_at((0.0, 1.5, 13.0), (0.0, 1.5, 0.0))


@pytest.mark.parametrize("effect", ["ssao", "shadow", "ssgi"])
def test_frames_with_background_bit_exact(effect):
    W, H = 384, 256
    log(f"[gpu] background frame {effect} {W}x{H}")
    scene = scenegen.make_scene(4, 60, 15)
    gb = scenegen.render_gbuffer(scene, sky_view(), W, H)
    bg = ~np.isfinite(gb.depth)
    assert 0.2 < bg.mean() < 0.8
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    col = None
    if effect == "shadow":
        si = scenegen.render_shadow_inputs(scene, gb.view, 1024)
        bd, pd = scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12)
        op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                                 F32(0.05), bd, pd)
        ep = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                              si.light_size, si.light_near, 0.05, torch.from_numpy(bd).to(DEV),
                              torch.from_numpy(pd).to(DEV))
    else:
        K = scenegen.ssao_kernel(16)
        r = 1.0 if effect == "ssao" else 2.0
        op = (oracle.SSAOParams if effect == "ssao" else oracle.SSGIParams)(K, r, 0.02)
        ep = mr.ssao_params(torch.from_numpy(K).to(DEV), r, 0.02)
    if effect == "ssgi":
        c16 = scenegen.lambert_color(scene, gb)
        col = torch.from_numpy(c16).to(DEV)
    ref = oracle.frame(effect, gb.depth, gb.normal, gb.focal, params(oracle, effect), op,
                       color=None if col is None else c16.astype(F32))
    lm = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    fr = mr.FrameRunner(effect, d, n, gb.focal, params(mr, effect), True, color=col, params=ep, level_map=lm)
    fr()
    plain = mr.FrameRunner(effect, d, n, gb.focal, params(mr, effect), False, color=col, params=ep)()
    torch.cuda.synchronize()
    assert np.array_equal(lm.cpu().numpy(), ref.pyramid.level_map)
    check_frame_lists(fr.lists(), ref.pyramid)
    assert np.array_equal(fr.out.cpu().numpy(), ref.out)
    rp = oracle.frame(effect, gb.depth, gb.normal, gb.focal, params(oracle, effect), op, multires=False,
                      color=None if col is None else c16.astype(F32)).out
    assert np.array_equal(plain.cpu().numpy(), rp)
