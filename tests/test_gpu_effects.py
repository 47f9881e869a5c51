"""GPU parity of the second and third effects: soft shadows (one-sample hard
shadow bits, shadow-edge masks, PCSS per level, merge, frame) and one-bounce
indirect light (FP16 colour, levels {1, 3, 4} and all four, 3-channel merge,
frame), each against the CPU oracle on the same seeded inputs."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

TOL = 1e-4
COS25 = float(np.float32(math.cos(math.radians(25.0))))
DEV = "cuda"


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def scene(W, H, seed=2, cam=1):
    s = scenegen.make_scene(seed, 120, 30)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(cam), W, H)
    return s, gb


def masks_params(effect, levels=4, enable=None):
    t = scenegen.TABLE1[effect]
    en = enable if enable is not None else (0b1101 if effect == "ssgi" else (1 << levels) - 1)
    m = mr.MaskParams(num_levels=levels, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)
    o = oracle.MaskParams(num_levels=levels, level_enable=en, sigma2=t["sigma2"], weight=t["weight"],
                          normal_cos=COS25)
    return m, o


# widths divisible by 128 take mr_frame's bit-packed path, the others the dense one
@pytest.mark.parametrize("W,H,sm", [(320, 184, 512), (384, 256, 512), (960, 544, 2048)])
def test_pcss_parity(W, H, sm):
    log(f"[gpu] pcss {W}x{H} map {sm}")
    s, gb = scene(W, H)
    si = scenegen.render_shadow_inputs(s, gb.view, sm)
    bd, pd = scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12)
    op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                             np.float32(0.05), bd, pd)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    smt = torch.from_numpy(si.shadow_map).to(DEV)
    sp = mr.shadow_params(smt, si.view_to_light, si.light_focal, si.light_size, si.light_near, 0.05,
                          torch.from_numpy(bd).to(DEV), torch.from_numpy(pd).to(DEV))
    mp, omp = masks_params("shadow")
    hard = mr.mr_shadow_hard(d, gb.focal, sp)
    masks = mr.mr_build_masks(d, n, gb.focal, mp, hard_shadow=hard)
    lo = mr.mr_eval_shadow(d, gb.focal, sp, mp=mp, masks=masks)
    out = mr.mr_upsample_merge(gb.focal, mp, masks, lo)
    multi = mr.mr_frame("shadow", d, n, gb.focal, mp, sp, multires=True)
    plain = mr.mr_frame("shadow", d, n, gb.focal, mp, sp, multires=False)
    torch.cuda.synchronize()
    ref_hard = oracle.hard_shadow(gb.depth, gb.focal, 1, op)
    assert np.array_equal(hard.cpu().numpy(), ref_hard)
    assert ref_hard.any() and not ref_hard.all()
    E = oracle.edge_image(gb.depth, gb.normal, omp.depth_ratio, omp.normal_cos) | oracle.shadow_edges(ref_hard,
                                                                                                    gb.depth)
    pyr = oracle.build_pyramid(E, omp)
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E)
    for i in pyr.levels[:-1]:
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i])
        assert np.array_equal(masks.worklist[i][:len(pyr.worklist[i])].cpu().numpy().view(np.uint32),
                              pyr.worklist[i])
    L = pyr.levels[-1]
    ref = {}
    for i in pyr.levels:
        zi = oracle.level_sample(gb.depth, i)
        ref[i] = oracle.pcss_level(zi, gb.focal, i, op, None if i == L else pyr.stencil[i])
        g = lo[i].cpu().numpy()
        sel = np.ones(g.shape, bool) if i == L else pyr.stencil[i].astype(bool)
        assert np.abs(g[sel] - ref[i][sel]).max(initial=0) <= TOL
        assert np.array_equal(g[sel], ref[i][sel]), f"level {i} not bit-exact"
    oref = oracle.upsample_merge(W, H, pyr.levels, {i: omp.weight[i - 1] for i in pyr.levels}, pyr.alpha,
                                 pyr.stencil, ref)
    assert np.array_equal(out.cpu().numpy(), oref)
    assert np.array_equal(multi.cpu().numpy(), oref)
    rp = oracle.pcss_level(gb.depth, gb.focal, 1, op)
    assert np.array_equal(plain.cpu().numpy(), rp)
    assert ((rp > 0) & (rp < 1)).any(), "no penumbra in the test scene"


@pytest.mark.parametrize("enable,W,H", [(0b1101, 320, 184), (0b1111, 320, 184), (0b1101, 384, 256),
                                        (0b1111, 384, 256)])
def test_ssgi_parity(enable, W, H):
    log(f"[gpu] ssgi levels {enable:04b} {W}x{H}")
    s, gb = scene(W, H, seed=3, cam=4)
    col = scenegen.lambert_color(s, gb)
    K = scenegen.ssao_kernel(24, seed=77)
    op = oracle.SSGIParams(K, 2.0, 0.02)
    mp, omp = masks_params("ssgi", enable=enable)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    c = torch.from_numpy(col).to(DEV)
    k = torch.from_numpy(K).to(DEV)
    masks = mr.mr_build_masks(d, n, gb.focal, mp)
    lo = mr.mr_eval_ssgi(d, n, c, gb.focal, k, 2.0, 0.02, mp=mp, masks=masks)
    out = mr.mr_upsample_merge(gb.focal, mp, masks, lo, channels=3)
    multi = mr.mr_frame("ssgi", d, n, gb.focal, mp, mr.ssao_params(k, 2.0, 0.02), color=c, multires=True)
    plain = mr.mr_frame("ssgi", d, n, gb.focal, mp, mr.ssao_params(k, 2.0, 0.02), color=c, multires=False)
    torch.cuda.synchronize()
    E = oracle.edge_image(gb.depth, gb.normal, omp.depth_ratio, omp.normal_cos)
    pyr = oracle.build_pyramid(E, omp)
    L = pyr.levels[-1]
    ref = {}
    for i in pyr.levels:
        zi = oracle.level_sample(gb.depth, i)
        ni = oracle.level_sample(gb.normal, i)
        ci = oracle.level_sample(col, i)
        ref[i] = oracle.ssgi_level(zi, ni, ci, gb.focal, i, op, None if i == L else pyr.stencil[i])
        g = lo[i].cpu().numpy()
        sel = np.ones(g.shape[1:], bool) if i == L else pyr.stencil[i].astype(bool)
        assert np.abs(g[:, sel] - ref[i][:, sel]).max(initial=0) <= TOL
        assert np.array_equal(g[:, sel], ref[i][:, sel]), f"level {i} not bit-exact"
    oref = oracle.upsample_merge(W, H, pyr.levels, {i: omp.weight[i - 1] for i in pyr.levels}, pyr.alpha,
                                 pyr.stencil, ref, channels=3)
    assert np.array_equal(out.cpu().numpy(), oref)
    assert np.array_equal(multi.cpu().numpy(), oref)
    rp = oracle.ssgi_level(gb.depth, gb.normal, col, gb.focal, 1, op)
    assert np.abs(plain.cpu().numpy() - rp).max() <= TOL
    assert np.array_equal(plain.cpu().numpy(), rp)
    assert rp.max() > 0


def test_ssgi_black_colour_and_plane_are_zero():
    log("[gpu] ssgi zero cases")
    d = torch.full((64, 96), 10.0, device=DEV)
    n = torch.zeros((3, 64, 96), device=DEV)
    n[2] = 1.0
    col = torch.ones((3, 64, 96), dtype=torch.float16, device=DEV)
    k = torch.from_numpy(scenegen.ssao_kernel(32)).to(DEV)
    out = mr.mr_eval_ssgi(d, n, col, 40.0, k, 2.0, 0.02)[1]
    s, gb = scene(128, 96)
    black = torch.zeros((3, 96, 128), dtype=torch.float16, device=DEV)
    out2 = mr.mr_eval_ssgi(torch.from_numpy(gb.depth).to(DEV), torch.from_numpy(gb.normal).to(DEV), black,
                           gb.focal, k, 2.0, 0.02)[1]
    torch.cuda.synchronize()
    assert (out == 0).all() and (out2 == 0).all()


def test_pcss_fully_lit_and_fully_dark():
    log("[gpu] pcss lit / dark")
    d = torch.full((32, 48), 10.0, device=DEV)
    M = np.zeros((3, 4), np.float32)
    M[0, 0] = M[1, 1] = M[2, 2] = 1.0
    bd = torch.from_numpy(scenegen.disk_samples(16, 11)).to(DEV)
    pd = torch.from_numpy(scenegen.disk_samples(32, 12)).to(DEV)
    far = torch.full((64, 64), 100.0, device=DEV)
    near = torch.full((64, 64), 5.0, device=DEV)
    lit = mr.mr_eval_shadow(d, 30.0, mr.shadow_params(far, M, 30.0, 0.5, 1.0, 0.05, bd, pd))[1]
    dark = mr.mr_eval_shadow(d, 30.0, mr.shadow_params(near, M, 30.0, 0.5, 1.0, 0.05, bd, pd))[1]
    torch.cuda.synchronize()
    assert (lit == 1).all() and (dark == 0).all()
