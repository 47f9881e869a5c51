"""Precision: FP16 storage of the sub-image values between evaluation and
merge (bit-exact against the oracle with the same rounding), and the error
of the GPU frames against the FP64 oracle per effect, with FP32 inputs and
with FP16 normals, colour and sub-image storage.  Depth, edge thresholds and
all arithmetic stay FP32, so the masks do not change (they are compared
bit for bit)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

COS25 = float(np.float32(math.cos(math.radians(25.0))))
DEV = "cuda"
W, H = 384, 256  # compact frame path: width divisible by 128


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_inputs = {}


def inputs():
    if _inputs:
        return _inputs
    s = scenegen.make_scene(3, 120, 30)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(2), W, H)
    si = scenegen.render_shadow_inputs(s, gb.view, 512)
    bd, pd = scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12)
    col = scenegen.lambert_color(s, gb)
    _inputs.update(s=s, gb=gb, si=si, bd=bd, pd=pd, col=col, K=scenegen.ssao_kernel(16))
    return _inputs


def params(effect, device=True):
    """(mr mask params, oracle mask params, mr effect params, oracle effect
    params); device=False leaves the mr effect params out (None)."""
    I = inputs()
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0b1111  # Table 1: SSGI leaves level 2 out
    mp = mr.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)
    omp = oracle.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"],
                            normal_cos=COS25)
    ep = None
    if effect == "shadow":
        si = I["si"]
        if device:
            ep = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                                  si.light_size, si.light_near, 0.05, torch.from_numpy(I["bd"]).to(DEV),
                                  torch.from_numpy(I["pd"]).to(DEV))
        op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                                 np.float32(0.05), I["bd"], I["pd"])
    else:
        r = 1.0 if effect == "ssao" else 2.0
        if device:
            ep = mr.ssao_params(torch.from_numpy(I["K"]).to(DEV), r, 0.02)
        op = (oracle.SSAOParams if effect == "ssao" else oracle.SSGIParams)(I["K"], r, 0.02)
    return mp, omp, ep, op


def gpu_frame(effect, f16):
    I = inputs()
    gb = I["gb"]
    mp, _, ep, _ = params(effect)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    c = torch.from_numpy(I["col"]).to(DEV) if effect == "ssgi" else None
    if f16:
        n = n.half()
    lm = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    out = mr.mr_frame(effect, d, n, gb.focal, mp, ep, multires=True, color=c, level_map=lm,
                      level_dtype=torch.float16 if f16 else torch.float32)
    torch.cuda.synchronize()
    return out.cpu().numpy(), lm.cpu().numpy()


def oracle_frame(effect, dtype, f16_normals=False, level_dtype=None):
    I = inputs()
    gb = I["gb"]
    _, omp, _, op = params(effect, device=False)
    normal = gb.normal.astype(np.float16).astype(np.float32) if f16_normals else gb.normal
    color = I["col"] if effect == "ssgi" else None
    if dtype == np.float64:
        normal = normal.astype(np.float64)
        color = color.astype(np.float64) if color is not None else None
    return oracle.frame(effect, gb.depth if dtype == np.float32 else gb.depth.astype(np.float64), normal, gb.focal,
                        omp, op, color=color, dtype=dtype, level_dtype=level_dtype)


@pytest.mark.parametrize("effect", ["ssao", "ssgi", "shadow"])
def test_fp16_sub_images_match_oracle_rounding(effect):
    """FP16 normals (and colour) in, FP16 sub-image storage: the GPU frame
    equals the FP32 oracle run on the same FP16-widened inputs that rounds
    every sub-image value to FP16 before the merge."""
    log(f"[gpu] fp16 storage {effect}")
    out, lm = gpu_frame(effect, f16=True)
    ref = oracle_frame(effect, np.float32, f16_normals=True, level_dtype=np.float16)
    assert np.array_equal(lm, ref.pyramid.level_map)
    assert np.abs(out - ref.out).max() <= 1e-4
    assert np.array_equal(out, ref.out)


def test_fp16_storage_needs_the_compact_path():
    I = inputs()
    gb = I["gb"]
    mp, _, ep, _ = params("ssao")
    Wr = 320  # not divisible by 128: dense frame path
    d = torch.from_numpy(np.ascontiguousarray(gb.depth[:, :Wr])).to(DEV)
    n = torch.from_numpy(np.ascontiguousarray(gb.normal[:, :, :Wr])).to(DEV)
    with pytest.raises(mr.MRError) as e:
        mr.mr_frame("ssao", d, n, gb.focal, mp, ep, multires=True, level_dtype=torch.float16)
    assert e.value.status == mr.MR_E_DTYPE


# Stated errors against the FP64 oracle (same method, float64 arithmetic, FP32
# inputs): mean and max absolute difference of the multi-resolution frame, and
# the share of pixels that differ by more than 1e-3 (a flipped discrete
# decision, e.g. one SSAO sample crossing the bias threshold: 1/16 here, one
# PCF tap: 1/32).  The bounds allow a few such flips and nothing more.
BOUNDS = {  # effect: (fp32 mean, fp32 max, fp16 mean, fp16 max)
    "ssao": (1e-6, 0.0626, 1e-4, 0.0626),
    "ssgi": (1e-5, 0.05, 1e-4, 0.05),
    "shadow": (1e-5, 0.0313, 1e-4, 0.0313),
}


@pytest.mark.parametrize("effect", ["ssao", "ssgi", "shadow"])
def test_error_against_fp64_oracle(effect):
    ref = oracle_frame(effect, np.float64).out
    stats = []
    for f16 in (False, True):
        out, _ = gpu_frame(effect, f16=f16)
        diff = np.abs(out.astype(np.float64) - ref)
        stats.append((float(diff.mean()), float(diff.max()), float((diff > 1e-3).mean())))
    b = BOUNDS[effect]
    log(f"[precision] {effect} {W}x{H} vs FP64 oracle: fp32 mean {stats[0][0]:.3e} max {stats[0][1]:.3e} "
        f"flipped {stats[0][2]:.4%}; fp16 storage mean {stats[1][0]:.3e} max {stats[1][1]:.3e} "
        f"flipped {stats[1][2]:.4%}")
    assert stats[0][0] <= b[0] and stats[0][1] <= b[1]
    assert stats[1][0] <= b[2] and stats[1][1] <= b[3]
