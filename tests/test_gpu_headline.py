"""GPU parity at the configurations that are measured or specified at full
size, through the C ABI, against the oracle on the same seeded inputs.

* The 4K SSAO headline (Sec. 5's 3840x2160 base resolution): the scene
  generator with 200 boxes and 50 spheres, 4 levels with the SSAO column of
  Table 1, 32 samples, radius 1.0; the first of the benchmark's resident
  configurations.  Masks, work lists, per-level SSAO and the merge through
  the step entry points, the whole frame through mr_frame, and the naive
  full-resolution pass on sampled pixels (the oracle evaluates them one list
  at a time).
* Soft shadows at 3840x2160 with a 2048^2 shadow map, 16 blocker and 32 PCF
  samples, FP16 normals: the frame bit-exact against the oracle fed the same
  widened normals, and its error against the FP64 oracle stated.
"""
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
COS25 = float(np.float32(math.cos(math.radians(25.0))))
W, H = 3840, 2160


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mask_params(lib, effect):
    t = scenegen.TABLE1[effect]
    return lib.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def sample_pixels(n, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(W * H, size=n, replace=False)
    return idx // W, idx % W


def test_ssao_4k_headline_configuration():
    log("[gpu] 4K SSAO headline: seed 1, camera 0, 32 samples")
    scene = scenegen.make_scene(1, 200, 50)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(0), W, H)
    K = scenegen.ssao_kernel(32)
    op = oracle.SSAOParams(K, 1.0, 0.02)
    omp = mask_params(oracle, "ssao")
    ref = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, omp, op)
    pyr = ref.pyramid
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    k = torch.from_numpy(K).to(DEV)
    mp = mask_params(mr, "ssao")
    # the step entry points
    masks = mr.mr_build_masks(d, n, gb.focal, mp)
    lo = mr.mr_eval_ssao(d, n, gb.focal, k, 1.0, 0.02, mp=mp, masks=masks)
    merged = mr.mr_upsample_merge(gb.focal, mp, masks, lo)
    # the timed frame and the naive pass
    fr = mr.FrameRunner("ssao", d, n, gb.focal, mp, True, params=mr.ssao_params(k, 1.0, 0.02))
    fr()
    plain = mr.FrameRunner("ssao", d, n, gb.focal, mp, False, params=mr.ssao_params(k, 1.0, 0.02))()
    torch.cuda.synchronize()
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E)
    assert np.array_equal(masks.level_map.cpu().numpy(), pyr.level_map)
    cnt = u32(masks.count)
    for i in (1, 2, 3):
        assert np.array_equal(u32(masks.alpha[i].view(torch.int32)), pyr.alpha[i].view(np.uint32)), i
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i]), i
        nl = len(pyr.worklist[i])
        assert cnt[i - 1] == nl and np.array_equal(u32(masks.worklist[i])[:nl], pyr.worklist[i]), i
    for i in (2, 3, 4):
        assert np.array_equal(masks.level_depth[i].cpu().numpy(), oracle.level_sample(gb.depth, i)), i
    for i in (1, 2, 3, 4):
        g = lo[i].cpu().numpy()
        sel = np.ones(g.shape, bool) if i == 4 else pyr.stencil[i].astype(bool)
        assert np.array_equal(g[sel], ref.level_out[i][sel]), f"level {i}"
    assert np.array_equal(merged.cpu().numpy(), ref.out)
    assert np.array_equal(fr.out.cpu().numpy(), ref.out)
    check_frame_lists(fr.lists(), pyr)
    ys, xs = sample_pixels(200_000, 11)
    exp = oracle.ssao_texels(gb.depth, gb.normal, gb.focal, 1, xs, ys, op)
    got = plain.cpu().numpy()[ys, xs]
    assert np.abs(got - exp).max() <= 1e-4
    assert np.array_equal(got, exp)
    mad = float(np.abs(fr.out.cpu().numpy().astype(np.float64) - plain.cpu().numpy()).mean())
    log(f"[gpu] 4K headline MAD multi-res vs naive {mad:.6f}")
    assert mad <= 0.01


def test_pcss_4k_2048_map_fp16_normals():
    w = scenegen.WORKLOADS["pcss_4k"]
    log("[gpu] 4K PCSS: 2048^2 map, 16 + 32 samples, FP16 normals")
    scene = scenegen.make_scene(2, w["boxes"], w["spheres"])
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(5), W, H)
    si = scenegen.render_shadow_inputs(scene, gb.view, w["sm_size"], light_size=w["light_size"])
    bd, pd = scenegen.disk_samples(w["n_blocker"], 11), scenegen.disk_samples(w["n_pcf"], 12)
    n16 = gb.normal.astype(np.float16)
    nw = n16.astype(np.float32)  # what the kernels read, widened exactly
    omp = mask_params(oracle, "shadow")
    op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                             np.float32(0.05), bd, pd)
    ref = oracle.frame("shadow", gb.depth, nw, gb.focal, omp, op)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(n16).to(DEV)
    sp = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                          si.light_size, si.light_near, 0.05, torch.from_numpy(bd).to(DEV),
                          torch.from_numpy(pd).to(DEV))
    lm = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    fr = mr.FrameRunner("shadow", d, n, gb.focal, mask_params(mr, "shadow"), True, params=sp, level_map=lm)
    fr()
    plain = mr.FrameRunner("shadow", d, n, gb.focal, mask_params(mr, "shadow"), False, params=sp)()
    torch.cuda.synchronize()
    assert np.array_equal(lm.cpu().numpy(), ref.pyramid.level_map)
    check_frame_lists(fr.lists(), ref.pyramid)
    got = fr.out.cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)
    ys, xs = sample_pixels(200_000, 12)
    exp = oracle.pcss_texels(gb.depth, gb.focal, 1, xs, ys, op)
    assert np.array_equal(plain.cpu().numpy()[ys, xs], exp)
    penumbra = float(((ref.out > 0) & (ref.out < 1)).mean())
    assert penumbra > 0.001, "no penumbra in the test frame"
    # error against the FP64 oracle on the same inputs
    ref64 = oracle.frame("shadow", gb.depth, nw, gb.focal, omp, op, dtype=np.float64)
    diff = np.abs(got.astype(np.float64) - ref64.out)
    mean, mx, flipped = float(diff.mean()), float(diff.max()), float((diff > 1e-3).mean())
    log(f"[gpu] 4K PCSS vs FP64 oracle: mean {mean:.3g}, max {mx:.3g}, flipped {100 * flipped:.4f}% "
        f"(penumbra {100 * penumbra:.2f}% of pixels)")
    assert mean < 1e-5 and flipped < 1e-3
