"""SSAO with the dense coarsest level evaluated in 16 x 16 tiles whose depth
(with a halo) is staged in LDS (mr_frame_desc.eval_halo): the frame is
bit-identical to the one that gathers from the depth plane, for every halo,
image sizes whose coarsest level is not a whole number of tiles, FP16
normals, background and invalid depth, and it matches the oracle."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

DEV = "cuda"
COS25 = float(np.float32(math.cos(math.radians(25.0))))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mask_params(lib=mr):
    t = scenegen.TABLE1["ssao"]
    return lib.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


@pytest.mark.parametrize("W,H,S,f16", [(384, 200, 16, False), (640, 360, 32, True), (1280, 720, 64, False),
                                       (3840, 2160, 32, False)])
def test_halo_frames_equal_plane_frames(W, H, S, f16):
    s = scenegen.make_scene(7, 200, 50)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(3), W, H)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    if f16:
        n = n.half()
    p = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(S)).to(DEV), 1.0, 0.02)
    mp = mask_params()
    log(f"[gpu] eval_halo {W}x{H} S={S} f16 normals={f16}")
    ref = mr.mr_frame("ssao", d, n, gb.focal, mp, p)
    for h in (8, 16, 24):
        got = mr.mr_frame("ssao", d, n, gb.focal, mp, p, eval_halo=h)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), h


def test_halo_frame_with_background_matches_oracle():
    W, H = 384, 256
    s = scenegen.make_scene(4, 120, 30)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(5), W, H)
    depth = gb.depth.copy()
    depth[:40, :] = np.inf     # sky
    depth[100:120, 200:260] = 0.0  # invalid depth
    depth[150:160, 10:60] = np.nan
    K = scenegen.ssao_kernel(16)
    p = mr.ssao_params(torch.from_numpy(K).to(DEV), 1.0, 0.02)
    log("[gpu] eval_halo with background and invalid depth vs oracle")
    got = mr.mr_frame("ssao", torch.from_numpy(depth).to(DEV), torch.from_numpy(gb.normal).to(DEV), gb.focal,
                      mask_params(), p, eval_halo=16)
    torch.cuda.synchronize()
    ref = oracle.frame("ssao", depth, gb.normal, gb.focal, mask_params(oracle), oracle.SSAOParams(K, 1.0, 0.02))
    got = got.cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)


def test_frame_tuner_keeps_a_valid_halo_and_the_image():
    """mr_frame_tune times every halo the frame admits and keeps the
    fastest; the image after tuning equals the untuned one.  Frames that
    admit only the depth plane (SSGI, the naive pass) time only halo 0."""
    W, H = 1920, 1080
    s = scenegen.make_scene(2, 200, 50)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(1), W, H)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    p = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(32)).to(DEV), 1.0, 0.02)
    mp = mask_params()
    log(f"[gpu] mr_frame_tune SSAO {W}x{H}")
    r = mr.FrameRunner("ssao", d, n, gb.focal, mp, True, params=p)
    ref = r().clone()
    halo, ms = r.tune(reps=3)
    torch.cuda.synchronize()
    assert halo in (0, 8, 16, 24) and r.desc.eval_halo == halo
    assert sorted(ms) == [0, 8, 16, 24] and all(t > 0.0 for t in ms.values())
    assert ms[halo] == min(ms.values())
    assert torch.equal(r(), ref)
    torch.cuda.synchronize()
    log("[gpu] mr_frame_tune naive pass and SSGI")
    plain = mr.FrameRunner("ssao", d, n, gb.focal, mp, False, params=p)
    halo_p, ms_p = plain.tune(reps=2)
    assert halo_p == 0 and list(ms_p) == [0]
    t = scenegen.TABLE1["ssgi"]
    mpg = mr.MaskParams(num_levels=4, level_enable=0b1101, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)
    col = torch.from_numpy(scenegen.lambert_color(s, gb)).to(DEV)
    gp = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(16)).to(DEV), 2.0, 0.02)
    g = mr.FrameRunner("ssgi", d, n, gb.focal, mpg, True, color=col, params=gp)
    ref_g = g().clone()
    halo_g, ms_g = g.tune(reps=2)
    assert halo_g == 0 and list(ms_g) == [0]
    assert torch.equal(g(), ref_g)
    torch.cuda.synchronize()
