"""mr_frame_static (the frame with the library's static device scratch, for
callers that cannot allocate) through the C ABI against mr_frame with a
caller workspace: bit-identical images on two calls in a row, the second
with a smaller frame, for each effect; frames larger than the scratch are
rejected before anything is enqueued."""
import math
import sys

import numpy as np
import pytest
import torch

import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

DEV = "cuda"
COS25 = float(np.float32(math.cos(math.radians(25.0))))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def inputs(W, H, seed, cam, effect):
    scene = scenegen.make_scene(seed, 120, 30)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(cam), W, H)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    col = None
    if effect == "ssgi":
        col = torch.from_numpy(scenegen.lambert_color(scene, gb)).to(DEV)
    if effect == "shadow":
        si = scenegen.render_shadow_inputs(scene, gb.view, 512)
        p = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                             si.light_size, si.light_near, 0.05,
                             torch.from_numpy(scenegen.disk_samples(16, 11)).to(DEV),
                             torch.from_numpy(scenegen.disk_samples(32, 12)).to(DEV))
    else:
        k = torch.from_numpy(scenegen.ssao_kernel(16)).to(DEV)
        p = mr.ssao_params(k, 1.0, 0.02)
    return gb, d, n, col, p


def mask_params(effect, levels=4):
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0xF
    return mr.MaskParams(num_levels=levels, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


# (W, H): the first on the compact path, the second smaller; then a pair on
# the dense-mask path (width not divisible by 128)
PAIRS = [((1024, 576), (640, 360)), ((1000, 560), (200, 120))]


@pytest.mark.parametrize("effect", ["ssao", "shadow", "ssgi"])
@pytest.mark.parametrize("pair", range(len(PAIRS)))
def test_static_scratch_frames_equal_workspace_frames(effect, pair):
    mp = mask_params(effect)
    for k, (W, H) in enumerate(PAIRS[pair]):
        log(f"[gpu] static scratch {effect} {W}x{H} call {k}")
        gb, d, n, col, p = inputs(W, H, 5 + k, 2 + k, effect)
        ref = mr.FrameRunner(effect, d, n, gb.focal, mp, True, color=col, params=p)
        st = mr.StaticFrameRunner(effect, d, n, gb.focal, mp, True, color=col, params=p)
        st.out.fill_(float("nan"))
        a = ref().clone()
        b = st()
        torch.cuda.synchronize()
        assert torch.isfinite(b).all()
        assert torch.equal(a, b), (effect, W, H, (a - b).abs().max().item())


def test_static_scratch_rejects_oversized_frames():
    mp = mask_params("ssao")
    W, H = 7680, 4320  # 8K: the compact path's intermediates exceed the scratch
    d = torch.ones((H, W), dtype=torch.float32, device=DEV)
    n = torch.zeros((3, H, W), dtype=torch.float32, device=DEV)
    k = torch.zeros((4, 3), dtype=torch.float32, device=DEV)
    st = mr.StaticFrameRunner("ssao", d, n, 1000.0, mp, True, params=mr.ssao_params(k, 1.0, 0.02))
    st.out.fill_(7.0)
    with pytest.raises(mr.MRError) as e:
        st()
    assert e.value.status == mr.MR_E_WORKSPACE
    torch.cuda.synchronize()
    assert (st.out == 7.0).all()  # nothing was enqueued
