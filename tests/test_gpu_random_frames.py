"""GPU parity over seeded random frame configurations: for each seed a scene,
camera, size, level count and enabled set, blur variances and weights,
effect (SSAO, PCSS or SSGI), sample counts and the normals' storage (FP32
or FP16) are drawn; the mask pyramid of mr_build_masks (edge image, hard
shadow bits, level map, a_i, stencils, work lists and counts, level depth),
the per-level values of the mr_eval_* entry points on their stencils, the
image of mr_upsample_merge, mr_frame's multi-resolution and naive images,
and for SSAO the variant with every level at full resolution and fewer
samples (mr_eval_ssao_fullres, Sec. 6) are compared bit for bit with the
oracle's (Sec. 3-4; the naive pass of Sec. 5).

The draws cover both frame paths: widths that are multiples of 128 with at
most four levels take the compact path (bit-packed stencils, ranked lists),
the others the dense one; sizes are ragged multiples of 2^(N-1) from one
coarsest texel upwards, so that tiles of every kernel are cut at the image
border.  The configurations are fixed by their seeds: every run checks the
same frames.  With FP16 normals the oracle takes the same normals rounded
to FP16 (the kernels widen them exactly)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import mr

DEV = "cuda"
COS25 = float(np.float32(math.cos(math.radians(25.0))))
SEEDS = range(64)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def draw(seed):
    """One frame configuration, a pure function of the seed."""
    rng = np.random.default_rng(9100 + seed)
    effect = str(rng.choice(["ssao", "ssao", "ssgi", "shadow"]))
    N = int(rng.integers(2, 6))
    s = 1 << (N - 1)
    en = 1 | (1 << (N - 1))
    for i in range(1, N - 1):
        en |= int(rng.integers(0, 2)) << i
    if N <= 4 and rng.random() < 0.5:
        W = 128 * int(rng.integers(1, 9))
    else:
        W = s * int(rng.integers(1, 1100 // s + 1))
    H = s * int(rng.integers(1, 600 // s + 1))
    sigma2 = tuple(float(rng.choice([0.0, 0.924, 1.848, 3.696])) for _ in range(N - 1)) + (0.0,)
    weight = tuple(float(rng.choice([1.0, 20.0, 50.0, 100.0, 1000.0])) for _ in range(N - 1)) + (1.0,)
    return dict(effect=effect, N=N, en=en, W=W, H=H, sigma2=sigma2, weight=weight,
                S=int(rng.choice([1, 3, 8, 16, 33])), radius=float(rng.choice([0.5, 1.0, 2.0])),
                scene=(int(rng.integers(1, 1000)), int(rng.integers(5, 120)), int(rng.integers(0, 30))),
                cam=int(rng.integers(0, 8)), sm=int(rng.choice([256, 512])),
                blockers=int(rng.integers(1, 17)), pcf=int(rng.integers(1, 33)), f16=bool(rng.random() < 0.25))


def test_draws_cover_both_paths_and_all_effects():
    cfgs = [draw(k) for k in SEEDS]
    compact = [c["W"] % 128 == 0 and c["N"] <= 4 for c in cfgs]
    assert any(compact) and not all(compact)
    assert {c["effect"] for c in cfgs} == {"ssao", "ssgi", "shadow"}
    assert {c["N"] for c in cfgs} >= {2, 3, 4, 5}
    assert any(c["W"] % 128 and c["W"] < 64 for c in cfgs) or any(c["H"] <= 16 for c in cfgs)
    assert any(c["f16"] for c in cfgs) and not all(c["f16"] for c in cfgs)


@pytest.mark.gpu
@pytest.mark.parametrize("seed", list(SEEDS))
def test_random_frame(seed):
    c = draw(seed)
    log(f"[gpu] random frame {seed}: {c}")
    W, H, N, en = c["W"], c["H"], c["N"], c["en"]
    sc = scenegen.make_scene(*c["scene"])
    gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(c["cam"]), W, H)
    mp = mr.MaskParams(num_levels=N, level_enable=en, sigma2=c["sigma2"], weight=c["weight"],
                       radius=(-1,) * N, normal_cos=COS25)
    omp = oracle.MaskParams(num_levels=N, level_enable=en, sigma2=c["sigma2"], weight=c["weight"],
                            radius=(-1,) * N, normal_cos=COS25)
    nrm = gb.normal.astype(np.float16) if c["f16"] else gb.normal
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(nrm).to(DEV)
    nrm = nrm.astype(np.float32)
    color = None
    if c["effect"] == "shadow":
        si = scenegen.render_shadow_inputs(sc, gb.view, c["sm"])
        bd = scenegen.disk_samples(c["blockers"], 11 + seed)
        pd = scenegen.disk_samples(c["pcf"], 12 + seed)
        op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                                 np.float32(0.05), bd, pd)
        sp = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                              si.light_size, si.light_near, 0.05, torch.from_numpy(bd).to(DEV),
                              torch.from_numpy(pd).to(DEV))
    else:
        K = scenegen.ssao_kernel(c["S"], seed=500 + seed)
        sp_kernel = torch.from_numpy(K).to(DEV)
        sp = mr.ssao_params(sp_kernel, c["radius"], 0.02)
        if c["effect"] == "ssao":
            op = oracle.SSAOParams(K, c["radius"], 0.02)
        else:
            op = oracle.SSGIParams(K, c["radius"], 0.02)
            color = scenegen.lambert_color(sc, gb)
    ct = None if color is None else torch.from_numpy(color).to(DEV)
    # the mask pyramid through the step entry point (Sec. 3.1, 4.1)
    hard = mr.mr_shadow_hard(d, gb.focal, sp) if c["effect"] == "shadow" else None
    masks = mr.mr_build_masks(d, n, gb.focal, mp, hard_shadow=hard)
    # the per-level evaluation and the merge through their step entry points
    if c["effect"] == "shadow":
        lo = mr.mr_eval_shadow(d, gb.focal, sp, mp=mp, masks=masks)
    elif c["effect"] == "ssao":
        lo = mr.mr_eval_ssao(d, n, gb.focal, sp_kernel, c["radius"], 0.02, mp=mp, masks=masks)
    else:
        lo = mr.mr_eval_ssgi(d, n, ct, gb.focal, sp_kernel, c["radius"], 0.02, mp=mp, masks=masks)
    steps = mr.mr_upsample_merge(gb.focal, mp, masks, lo, channels=3 if c["effect"] == "ssgi" else 1)
    multi = mr.mr_frame(c["effect"], d, n, gb.focal, mp, sp, color=ct, multires=True)
    plain = mr.mr_frame(c["effect"], d, n, gb.focal, mp, sp, color=ct, multires=False)
    torch.cuda.synchronize()
    rf = oracle.frame(c["effect"], gb.depth, nrm, gb.focal, omp, op, color=color).out
    rp = oracle.frame(c["effect"], gb.depth, nrm, gb.focal, omp, op, multires=False, color=color).out
    E = oracle.edge_image(gb.depth, nrm, omp.depth_ratio, omp.normal_cos)
    if c["effect"] == "shadow":
        ref_hard = oracle.hard_shadow(gb.depth, gb.focal, 1, op)
        assert np.array_equal(hard.cpu().numpy(), ref_hard), "hard shadow bits"
        E = E | oracle.shadow_edges(ref_hard, gb.depth)
    pyr = oracle.build_pyramid(E, omp)
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E), "edge image"
    assert np.array_equal(masks.level_map.cpu().numpy(), pyr.level_map), "level map"
    cnt = masks.count.cpu().numpy().view(np.uint32)
    for i in pyr.levels:
        if i >= 2:
            assert np.array_equal(masks.level_depth[i].cpu().numpy(), oracle.level_sample(gb.depth, i)), f"depth {i}"
        if i == pyr.levels[-1]:
            continue
        assert np.array_equal(masks.alpha[i].cpu().numpy().view(np.uint32), pyr.alpha[i].view(np.uint32)), f"a_{i}"
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i]), f"stencil {i}"
        k = len(pyr.worklist[i])
        assert cnt[i - 1] == k, f"count {i}"
        assert np.array_equal(masks.worklist[i][:k].cpu().numpy().view(np.uint32), pyr.worklist[i]), f"list {i}"
    m, p = multi.cpu().numpy(), plain.cpu().numpy()
    assert m.shape == rf.shape and p.shape == rp.shape
    assert np.array_equal(m, rf), f"multi-resolution frame: max |d| {np.abs(m - rf).max()}"
    assert np.array_equal(steps.cpu().numpy(), rf), "step entry points"
    # every level's values on its stencil (the coarsest level everywhere)
    L = pyr.levels[-1]
    for i in pyr.levels:
        zi = oracle.level_sample(gb.depth, i)
        st = None if i == L else pyr.stencil[i]
        if c["effect"] == "shadow":
            ref = oracle.pcss_level(zi, gb.focal, i, op, st)
        elif c["effect"] == "ssao":
            ref = oracle.ssao_level(zi, oracle.level_sample(nrm, i), gb.focal, i, op, st)
        else:
            ref = oracle.ssgi_level(zi, oracle.level_sample(nrm, i), oracle.level_sample(color, i), gb.focal, i,
                                    op, st)
        g = lo[i].cpu().numpy()
        sel = np.ones(zi.shape, bool) if st is None else st.astype(bool)
        assert np.array_equal(g[..., sel], ref[..., sel]), f"level {i} values"
    if c["effect"] == "ssao":
        # the same masks with every level at full resolution and its own,
        # smaller sample set (Sec. 6)
        rng = np.random.default_rng(4400 + seed)
        Ks = {i: scenegen.ssao_kernel(max(1, c["S"] >> int(rng.integers(0, i))), seed=600 + 7 * seed + i)
              for i in pyr.levels}
        rs = {i: float(rng.choice([0.5, 1.0, 2.0])) for i in pyr.levels}
        lp = {i: mr.ssao_params(torch.from_numpy(Ks[i]).to(DEV), rs[i], 0.02) for i in pyr.levels}
        fr = mr.mr_eval_ssao_fullres(d, n, gb.focal, mp, masks, lp)
        torch.cuda.synchronize()
        ref = oracle.frame_fullres_levels(gb.depth, nrm, gb.focal, omp,
                                          {i: oracle.SSAOParams(Ks[i], rs[i], 0.02) for i in pyr.levels}).out
        assert np.array_equal(fr.cpu().numpy(), ref), "full-resolution levels with fewer samples"
    assert np.array_equal(p, rp), f"naive frame: max |d| {np.abs(p - rp).max()}"
