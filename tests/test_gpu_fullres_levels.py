"""Sub-images at full resolution with fewer samples (Sec. 6) through
mr_build_masks + mr_eval_ssao_fullres against the oracle's variant, bit for
bit, on frames with 3 and 4 levels, a skipped level, a ragged size and FP16
normals."""
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


CASES = {
    # name: (W, H, boxes, spheres, seed, cam, levels, enable, S at level 1)
    "256_3lv": (256, 256, 8, 0, 1, 0, 3, 0b111, 16),
    "ragged_200x120": (200, 120, 40, 10, 2, 3, 4, 0b1111, 16),
    "skip_level2": (320, 184, 30, 8, 5, 6, 4, 0b1101, 32),
    "640x360": (640, 360, 60, 15, 8, 5, 4, 0b1111, 32),
}


def run(name, f16=False):
    W, H, nb, ns, seed, cam, N, en, S = CASES[name]
    sc = scenegen.make_scene(seed, nb, ns)
    gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(cam), W, H)
    t = scenegen.TABLE1["ssao"]
    sig, wt = t["sigma2"][:N - 1] + (0.0,), t["weight"][:N - 1] + (1.0,)
    mp = mr.MaskParams(num_levels=N, level_enable=en, sigma2=sig, weight=wt, normal_cos=COS25)
    omp = oracle.MaskParams(num_levels=N, level_enable=en, sigma2=sig, weight=wt, normal_cos=COS25)
    levels = [i for i in range(1, N + 1) if en >> (i - 1) & 1]
    K = {i: scenegen.ssao_kernel(max(2, S >> (i - 1)), seed=60 + i) for i in levels}
    kd = {i: torch.from_numpy(K[i]).to(DEV) for i in levels}
    lp = {i: mr.ssao_params(kd[i], 1.0, 0.02) for i in levels}
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    if f16:
        n = n.half()
    log(f"[gpu] fullres levels {name} f16={f16}")
    masks = mr.mr_build_masks(d, n, gb.focal, mp)
    out = mr.mr_eval_ssao_fullres(d, n, gb.focal, mp, masks, lp)
    torch.cuda.synchronize()
    normal = gb.normal.astype(np.float16).astype(np.float32) if f16 else gb.normal
    ref = oracle.frame_fullres_levels(gb.depth, normal, gb.focal, omp,
                                      {i: oracle.SSAOParams(K[i], 1.0, 0.02) for i in levels})
    return out.cpu().numpy(), ref


@pytest.mark.parametrize("name", list(CASES))
def test_matches_oracle(name):
    got, ref = run(name)
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)


def test_fp16_normals():
    got, ref = run("ragged_200x120", f16=True)
    assert np.array_equal(got, ref.out)
