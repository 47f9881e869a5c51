"""mr_frame_cached: a frame whose mask pyramid stays resident.  Building the
pyramid and reusing it (several times, with other frames run in the same
scratch in between) gives the image of mr_frame bit for bit, for every
effect, with FP32 and FP16 sub-image storage and with the level map."""
import math
import sys

import numpy as np
import pytest
import torch

import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

COS25 = float(np.float32(math.cos(math.radians(25.0))))
DEV = "cuda"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(effect, W, H, seed):
    s = scenegen.make_scene(seed, 120, 30)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(seed % 8), W, H)
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0b1111
    mp = mr.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    c = torch.from_numpy(scenegen.lambert_color(s, gb)).to(DEV) if effect == "ssgi" else None
    if effect == "shadow":
        si = scenegen.render_shadow_inputs(s, gb.view, 512)
        ep = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                              si.light_size, si.light_near, 0.05,
                              torch.from_numpy(scenegen.disk_samples(16, 11)).to(DEV),
                              torch.from_numpy(scenegen.disk_samples(32, 12)).to(DEV))
    else:
        ep = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(16)).to(DEV), 1.0 if effect == "ssao" else 2.0,
                            0.02)
    return gb, mp, d, n, c, ep


@pytest.mark.parametrize("effect", ["ssao", "shadow", "ssgi"])
@pytest.mark.parametrize("f16", [False, True])
def test_build_then_reuse_matches_mr_frame(effect, f16):
    W, H = 384, 256
    log(f"[gpu] cached pyramid {effect} {W}x{H} f16={f16}")
    ldt = torch.float16 if f16 else torch.float32
    gb, mp, d, n, c, ep = inputs(effect, W, H, seed=5)
    lm_ref = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    ref = mr.mr_frame(effect, d, n, gb.focal, mp, ep, multires=True, color=c, level_map=lm_ref, level_dtype=ldt)
    npyr, nscr = mr.mr_pyramid_bytes(W, H, gb.focal, mp, mr.EFFECTS[effect])
    pyr = torch.empty(npyr, dtype=torch.uint8, device=DEV)
    scr = torch.empty(nscr, dtype=torch.uint8, device=DEV)
    lm = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    fr = mr.CachedFrameRunner(effect, d, n, gb.focal, mp, pyr, color=c, params=ep, level_map=lm, workspace=scr,
                              level_dtype=ldt)
    built = fr(build=True).clone()
    torch.cuda.synchronize()
    assert torch.equal(built, ref) and torch.equal(lm, lm_ref)
    # another scene's frame in the same scratch: the pyramid alone carries
    # the masks from one frame to the next
    gb2, mp2, d2, n2, c2, ep2 = inputs(effect, W, H, seed=9)
    scr.fill_(0xFF)
    other = mr.CachedFrameRunner(effect, d2, n2, gb2.focal, mp2, torch.empty_like(pyr), color=c2, params=ep2,
                                 workspace=scr, level_dtype=ldt)
    other(build=True)
    lm.zero_()
    fr.out.fill_(float("nan"))
    for _ in range(2):
        again = fr(build=False).clone()
        torch.cuda.synchronize()
        assert torch.equal(again, ref) and torch.equal(lm, lm_ref)


def test_reuse_on_two_streams_at_once():
    """Frames that read one pyramid may overlap: two streams, each with its
    own scratch, after one build."""
    W, H = 640, 384
    log(f"[gpu] cached pyramid on two streams {W}x{H}")
    gb, mp, d, n, c, ep = inputs("ssao", W, H, seed=6)
    ref = mr.mr_frame("ssao", d, n, gb.focal, mp, ep, multires=True)
    npyr, nscr = mr.mr_pyramid_bytes(W, H, gb.focal, mp, mr.MR_EFFECT_SSAO)
    pyr = torch.empty(npyr, dtype=torch.uint8, device=DEV)
    mr.CachedFrameRunner("ssao", d, n, gb.focal, mp, pyr, params=ep,
                         workspace=torch.empty(nscr, dtype=torch.uint8, device=DEV))(build=True)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    runs = [mr.CachedFrameRunner("ssao", d, n, gb.focal, mp, pyr, params=ep,
                                 workspace=torch.empty(nscr, dtype=torch.uint8, device=DEV)) for _ in streams]
    for _ in range(3):
        for r, s in zip(runs, streams):
            r(s, build=False)
    torch.cuda.synchronize()
    for r in runs:
        assert torch.equal(r.out, ref)


def test_refuses_what_it_cannot_serve():
    W, H = 384, 256
    gb, mp, d, n, c, ep = inputs("ssao", W, H, seed=5)
    npyr, nscr = mr.mr_pyramid_bytes(W, H, gb.focal, mp, mr.MR_EFFECT_SSAO)
    small = torch.empty(npyr - 256, dtype=torch.uint8, device=DEV)
    with pytest.raises(ValueError):
        mr.CachedFrameRunner("ssao", d, n, gb.focal, mp, small, params=ep)
    d2 = torch.from_numpy(np.ascontiguousarray(gb.depth[:, :200])).to(DEV)
    n2 = torch.from_numpy(np.ascontiguousarray(gb.normal[:, :, :200])).to(DEV)
    with pytest.raises(mr.MRError):  # width 200: not the compact path
        mr.CachedFrameRunner("ssao", d2, n2, gb.focal, mp, torch.empty(npyr, dtype=torch.uint8, device=DEV),
                             params=ep)
