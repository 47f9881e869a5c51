"""Bilateral blur of SSAO sub-images (Sec. 4.1) through mr_frame against the
oracle's frame with the same blur: bit-exact in FP32 and with FP16
sub-image storage, for either radius and different level choices, on
frames with ragged merge and rank tiles."""
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
_cache = {}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def case(W, H, seed, cam, S):
    key = (W, H, seed, cam, S)
    if key not in _cache:
        sc = scenegen.make_scene(seed, 60, 15)
        gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(cam), W, H)
        K = scenegen.ssao_kernel(S)
        _cache[key] = dict(gb=gb, K=K, d=torch.from_numpy(gb.depth).to(DEV), n=torch.from_numpy(gb.normal).to(DEV),
                           k=torch.from_numpy(K).to(DEV))
    return _cache[key]


def params(lib):
    t = scenegen.TABLE1["ssao"]
    return lib.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


@pytest.mark.parametrize("W,H,seed,cam,S,levels,R,f16", [
    (640, 360, 8, 5, 8, 0b1110, 2, False),
    (640, 360, 8, 5, 8, 0b1111, 1, False),
    (384, 200, 9, 2, 16, 0b0001, 2, False),
    (384, 200, 9, 2, 16, 0b1000, 1, False),
    (512, 296, 3, 7, 8, 0b1110, 2, True),
    (256, 136, 4, 1, 4, 0b0110, 1, True),
])
def test_blurred_frame_matches_oracle(W, H, seed, cam, S, levels, R, f16):
    c = case(W, H, seed, cam, S)
    gb = c["gb"]
    bp = mr.Bilateral(levels=levels, radius=R, depth_rel=0.05)
    n = c["n"].half() if f16 else c["n"]
    log(f"[gpu] bilateral {W}x{H} S={S} levels={levels:04b} R={R} f16={f16}")
    out = mr.mr_frame("ssao", c["d"], n, gb.focal, params(mr), mr.ssao_params(c["k"], 1.0, 0.02), bilateral=bp,
                      level_dtype=torch.float16 if f16 else torch.float32)
    torch.cuda.synchronize()
    normal = gb.normal.astype(np.float16).astype(np.float32) if f16 else gb.normal
    ref = oracle.frame("ssao", gb.depth, normal, gb.focal, params(oracle), oracle.SSAOParams(c["K"], 1.0, 0.02),
                       level_dtype=np.float16 if f16 else None,
                       bilateral=oracle.BilateralParams(levels=levels, radius=R, depth_rel=0.05))
    got = out.cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)


def test_blur_changes_only_what_it_should():
    """levels = 0 is the unblurred frame; blurring changes the frame; the
    blurred frame is deterministic."""
    c = case(640, 360, 8, 5, 8)
    gb = c["gb"]
    sp = mr.ssao_params(c["k"], 1.0, 0.02)
    base = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, params(mr), sp).clone()
    off = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, params(mr), sp, bilateral=mr.Bilateral(levels=0)).clone()
    on1 = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, params(mr), sp, bilateral=mr.Bilateral()).clone()
    on2 = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, params(mr), sp, bilateral=mr.Bilateral()).clone()
    torch.cuda.synchronize()
    assert torch.equal(base, off)
    assert not torch.equal(base, on1)
    assert torch.equal(on1, on2)
