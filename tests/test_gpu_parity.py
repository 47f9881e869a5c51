"""GPU parity: every output of the HIP path through the C ABI against the CPU
oracle on the same seeded inputs.

Bar: masks, stencils, owner-level map, work lists and counts bit-exact;
lighting and merge within 1e-4 absolute in FP32 (the kernels follow the
oracle's operation order, so they are expected to be bit-exact as well and
the strict tests check that too)."""
import dataclasses
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


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
CASES = {
    # name: (W, H, boxes, spheres, seed, cam, levels, level_enable, sigma2, weight, S, r, radius)
    "256_3lv": (256, 256, 8, 0, 1, 0, 3, 0b111, (0.924, 1.848, 0.0), (100, 50, 1), 16, 0.5, (-1, -1, -1)),
    "ragged_200x120": (200, 120, 40, 10, 2, 3, 4, 0b1111, (0.924, 1.848, 3.696, 0), (100, 50, 20, 1), 16, 0.7,
                       (-1, -1, -1, -1)),
    "tiny_8x8": (8, 8, 3, 1, 4, 1, 4, 0b1111, (0.924, 1.848, 3.696, 0), (100, 50, 20, 1), 8, 1.0,
                 (-1, -1, -1, -1)),
    "skip_level2": (320, 184, 30, 8, 5, 6, 4, 0b1101, (0.924, 0.0, 0.924, 0), (1000, 1, 100, 1), 16, 1.0,
                    (-1, -1, -1, -1)),
    "nest_r0": (192, 128, 30, 8, 6, 2, 4, 0b1111, (0.924, 0.0, 0.0, 0), (100, 50, 20, 1), 16, 1.0,
                (-1, 0, 0, -1)),
    "wide_radius": (256, 192, 30, 8, 7, 5, 4, 0b1111, (9.0, 1.848, 12.0, 0), (100, 50, 20, 1), 16, 1.0,
                    (-1, 11, 16, -1)),
    "1080p": (1920, 1080, 200, 50, 1, 0, 4, 0b1111, (0.924, 1.848, 3.696, 0), (100, 50, 20, 1), 32, 1.0,
              (-1, -1, -1, -1)),
    # compact frame path (width divisible by 128) with ragged merge tiles
    # (heights not divisible by 16) and a ragged last column of edge tiles
    "lean_640x360": (640, 360, 60, 15, 8, 5, 4, 0b1111, (0.924, 1.848, 3.696, 0), (100, 50, 20, 1), 16, 1.0,
                     (-1, -1, -1, -1)),
    "lean_384x200": (384, 200, 40, 10, 9, 2, 4, 0b1111, (0.924, 1.848, 3.696, 0), (100, 50, 20, 1), 16, 0.8,
                     (-1, -1, -1, -1)),
}

_cache = {}


def case(name):
    if name in _cache:
        return _cache[name]
    W, H, nb, ns, seed, camk, N, en, s2, w, S, r, rad = CASES[name]
    scene = scenegen.make_scene(seed, nb, ns)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(camk), W, H)
    K = scenegen.ssao_kernel(S)
    mp = mr.MaskParams(num_levels=N, level_enable=en, sigma2=s2, weight=w, radius=rad, normal_cos=COS25)
    omp = oracle.MaskParams(num_levels=N, level_enable=en, sigma2=s2, weight=w, radius=rad, normal_cos=COS25)
    E = oracle.edge_image(gb.depth, gb.normal, omp.depth_ratio, omp.normal_cos)
    pyr = oracle.build_pyramid(E, omp)
    c = dict(W=W, H=H, scene=scene, gb=gb, K=K, S=S, r=r, mp=mp, omp=omp, pyr=pyr,
             d=torch.from_numpy(gb.depth).to(DEV), n=torch.from_numpy(gb.normal).to(DEV),
             k=torch.from_numpy(K).to(DEV))
    _cache[name] = c
    return c


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def check_masks(c, masks):
    pyr, W, H = c["pyr"], c["W"], c["H"]
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E), "edge image"
    assert np.array_equal(masks.level_map.cpu().numpy(), pyr.level_map), "level map"
    cnt = u32(masks.count)
    L = pyr.levels[-1]
    for i in pyr.levels:
        if i >= 2:
            zi = oracle.level_sample(c["gb"].depth, i)
            assert np.array_equal(masks.level_depth[i].cpu().numpy(), zi), f"level depth {i}"
        if i == L:
            continue
        a = masks.alpha[i].cpu().numpy()
        assert np.array_equal(a.view(np.uint32), pyr.alpha[i].view(np.uint32)), f"alpha level {i}"
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i]), f"stencil level {i}"
        n = len(pyr.worklist[i])
        assert cnt[i - 1] == n, f"count level {i}: {cnt[i - 1]} vs {n}"
        assert np.array_equal(u32(masks.worklist[i])[:n], pyr.worklist[i]), f"worklist level {i}"
    for i in range(1, 7):
        if i not in pyr.levels or i == L:
            assert cnt[i - 1] == 0


@pytest.mark.parametrize("name", list(CASES))
def test_masks_bit_exact(name):
    log(f"[gpu] masks {name}")
    c = case(name)
    masks = mr.mr_build_masks(c["d"], c["n"], c["gb"].focal, c["mp"])
    torch.cuda.synchronize()
    check_masks(c, masks)


def oracle_levels(c, effect="ssao"):
    gb, pyr = c["gb"], c["pyr"]
    p = oracle.SSAOParams(c["K"], c["r"], 0.02)
    L = pyr.levels[-1]
    out = {}
    for i in pyr.levels:
        zi = oracle.level_sample(gb.depth, i)
        ni = oracle.level_sample(gb.normal, i)
        out[i] = oracle.ssao_level(zi, ni, gb.focal, i, p, None if i == L else pyr.stencil[i])
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_ssao_levels_and_merge(name):
    log(f"[gpu] ssao levels + merge {name}")
    c = case(name)
    masks = mr.mr_build_masks(c["d"], c["n"], c["gb"].focal, c["mp"])
    lo = mr.mr_eval_ssao(c["d"], c["n"], c["gb"].focal, c["k"], c["r"], 0.02, mp=c["mp"], masks=masks)
    out = mr.mr_upsample_merge(c["gb"].focal, c["mp"], masks, lo)
    torch.cuda.synchronize()
    ref = oracle_levels(c)
    pyr = c["pyr"]
    L = pyr.levels[-1]
    for i in pyr.levels:
        g = lo[i].cpu().numpy()
        sel = np.ones(g.shape, bool) if i == L else pyr.stencil[i].astype(bool)
        assert np.abs(g[sel] - ref[i][sel]).max(initial=0) <= TOL, f"level {i}"
        assert np.array_equal(g[sel], ref[i][sel]), f"level {i} not bit-exact"
        if i != L:
            assert np.isnan(g[~sel]).all(), f"level {i} wrote outside its stencil"
    oref = oracle.upsample_merge(c["W"], c["H"], pyr.levels, {i: c["omp"].weight[i - 1] for i in pyr.levels},
                                 pyr.alpha, pyr.stencil, ref)
    o = out.cpu().numpy()
    assert np.abs(o - oref).max() <= TOL
    assert np.array_equal(o, oref), "merge not bit-exact"


# 256_3lv, skip_level2 (width 320 -> dense), wide_radius (radius > 8 -> dense), 1080p:
# mr_frame takes the bit-packed path where it is eligible and the dense one elsewhere
@pytest.mark.parametrize("name", ["256_3lv", "ragged_200x120", "skip_level2", "wide_radius", "1080p", "lean_640x360",
                                  "lean_384x200"])
def test_plain_and_frame(name):
    log(f"[gpu] plain + frame {name}")
    c = case(name)
    gb = c["gb"]
    sp = mr.ssao_params(c["k"], c["r"], 0.02)
    lm = torch.empty((c["H"], c["W"]), dtype=torch.uint8, device=DEV)
    multi = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, c["mp"], sp, multires=True, level_map=lm)
    plain = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, c["mp"], sp, multires=False)
    torch.cuda.synchronize()
    op = oracle.SSAOParams(c["K"], c["r"], 0.02)
    rf = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, c["omp"], op)
    rp = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, c["omp"], op, multires=False).out
    assert np.array_equal(lm.cpu().numpy(), rf.pyramid.level_map)
    m, p = multi.cpu().numpy(), plain.cpu().numpy()
    assert np.abs(p - rp).max() <= TOL and np.array_equal(p, rp), "plain"
    assert np.abs(m - rf.out).max() <= TOL and np.array_equal(m, rf.out), "multi-res frame"
    # quality bound of the method against the naive pass
    assert np.abs(m - p).mean() <= 0.01


@pytest.mark.parametrize("name,fovea", [("256_3lv", (100.3, 140.6, 30.0, 70.5)),
                                        ("lean_640x360", (420.0, 150.5, 60.0, 150.0)),
                                        ("lean_384x200", (-20.0, 90.0, 80.0, 120.0))])
def test_foveated_masks_and_frame(name, fovea):
    """Importance mask of a gaze point combined with the edges (min with the
    outer disk, max with the inner one): masks bit-exact through the mask
    entry point, frames (compact path for the 'lean' cases) against the
    oracle."""
    log(f"[gpu] fovea {name} {fovea}")
    c = case(name)
    gb = c["gb"]
    mp = dataclasses.replace(c["mp"], fovea=fovea)
    omp = dataclasses.replace(c["omp"], fovea=fovea)
    E = oracle.foveate(oracle.edge_image(gb.depth, gb.normal, omp.depth_ratio, omp.normal_cos), fovea)
    pyr = oracle.build_pyramid(E, omp)
    masks = mr.mr_build_masks(c["d"], c["n"], gb.focal, mp)
    torch.cuda.synchronize()
    check_masks(dict(c, pyr=pyr), masks)
    sp = mr.ssao_params(c["k"], c["r"], 0.02)
    lm = torch.empty((c["H"], c["W"]), dtype=torch.uint8, device=DEV)
    out = mr.mr_frame("ssao", c["d"], c["n"], gb.focal, mp, sp, multires=True, level_map=lm)
    torch.cuda.synchronize()
    rf = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, omp, oracle.SSAOParams(c["K"], c["r"], 0.02))
    assert np.array_equal(lm.cpu().numpy(), rf.pyramid.level_map)
    o = out.cpu().numpy()
    assert np.abs(o - rf.out).max() <= TOL and np.array_equal(o, rf.out)


def test_all_finest_masks_reproduce_plain_bitwise():
    """Hand-built masks with S_1 = 1 and a_1 = 1 everywhere give alpha_1 = 1,
    so the merged image must equal the naive full-resolution pass bit for bit."""
    log("[gpu] all-finest")
    c = case("256_3lv")
    W, H = c["W"], c["H"]
    mp = c["mp"]
    masks = mr.alloc_masks(W, H, c["gb"].focal, mp, DEV)
    for i in (1, 2):
        Wi, Hi = W >> (i - 1), H >> (i - 1)
        masks.alpha[i].fill_(1.0)
        masks.stencil[i].fill_(1)
        masks.worklist[i].copy_(torch.arange(Wi * Hi, dtype=torch.int32, device=DEV))
        masks.count[i - 1] = Wi * Hi
    masks.level_depth.clear()
    lo = mr.mr_eval_ssao(c["d"], c["n"], c["gb"].focal, c["k"], c["r"], 0.02, mp=mp, masks=masks)
    out = mr.mr_upsample_merge(c["gb"].focal, mp, masks, lo)
    plain = mr.mr_eval_ssao(c["d"], c["n"], c["gb"].focal, c["k"], c["r"], 0.02)[1]
    torch.cuda.synchronize()
    assert torch.equal(out, plain)


def test_edge_free_plane_is_coarsest_and_unoccluded():
    log("[gpu] edge-free plane")
    s = scenegen.make_scene(1, 0, 0)
    gb = scenegen.render_gbuffer(s, scenegen.orbit_view(2), 320, 240)
    d, n = torch.from_numpy(gb.depth).to(DEV), torch.from_numpy(gb.normal).to(DEV)
    mp = mr.MaskParams(normal_cos=COS25)
    masks = mr.mr_build_masks(d, n, gb.focal, mp)
    k = torch.from_numpy(scenegen.ssao_kernel(32)).to(DEV)
    out = mr.mr_frame("ssao", d, n, gb.focal, mp, mr.ssao_params(k, 1.0, 0.02))
    torch.cuda.synchronize()
    assert (masks.level_map == 4).all()
    assert int(masks.edge.sum()) == 0
    assert (u32(masks.count) == 0).all()
    assert (out == 0).all()


def test_fronto_parallel_plane_is_exactly_unoccluded():
    log("[gpu] fronto-parallel plane")
    d = torch.full((64, 96), 10.0, device=DEV)
    n = torch.zeros((3, 64, 96), device=DEV)
    n[2] = 1.0
    k = torch.from_numpy(scenegen.ssao_kernel(64)).to(DEV)
    out = mr.mr_eval_ssao(d, n, 40.0, k, 1.0, 0.02)[1]
    torch.cuda.synchronize()
    assert (out == 0).all()


def test_fp16_normals_path():
    """FP16 normals are widened exactly; the oracle is fed the same widened
    values, so masks stay bit-exact and the lighting matches."""
    log("[gpu] fp16 normals")
    c = case("ragged_200x120")
    gb = c["gb"]
    n16 = gb.normal.astype(np.float16)
    nw = n16.astype(np.float32)
    omp = c["omp"]
    E = oracle.edge_image(gb.depth, nw, omp.depth_ratio, omp.normal_cos)
    pyr = oracle.build_pyramid(E, omp)
    op = oracle.SSAOParams(c["K"], c["r"], 0.02)
    rf = oracle.frame("ssao", gb.depth, nw, gb.focal, omp, op)
    nt = torch.from_numpy(n16).to(DEV)
    masks = mr.mr_build_masks(c["d"], nt, gb.focal, c["mp"])
    out = mr.mr_frame("ssao", c["d"], nt, gb.focal, c["mp"], mr.ssao_params(c["k"], c["r"], 0.02))
    torch.cuda.synchronize()
    assert np.array_equal(masks.edge.cpu().numpy(), pyr.E)
    for i in pyr.levels[:-1]:
        assert np.array_equal(masks.stencil[i].cpu().numpy(), pyr.stencil[i])
    assert np.array_equal(out.cpu().numpy(), rf.out)


def test_deterministic_across_runs():
    log("[gpu] determinism")
    c = case("1080p")
    sp = mr.ssao_params(c["k"], c["r"], 0.02)
    fr = mr.FrameRunner("ssao", c["d"], c["n"], c["gb"].focal, c["mp"], params=sp)
    a = fr().clone()
    b = fr().clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("multires", [True, False])
def test_stage_events(multires):
    """The stage events bracket the frame in order and leave its output
    unchanged."""
    log(f"[gpu] stage events multires={multires}")
    c = case("1080p")
    sp = mr.ssao_params(c["k"], c["r"], 0.02)
    fr = mr.FrameRunner("ssao", c["d"], c["n"], c["gb"].focal, c["mp"], multires, params=sp)
    ref = fr().clone()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(mr.MR_FRAME_EVENTS)]
    fr.set_stage_events(ev)
    out = fr().clone()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    t = [ev[k].elapsed_time(ev[k + 1]) for k in range(3)]
    assert all(x >= 0 for x in t)
    assert abs(sum(t) - ev[0].elapsed_time(ev[3])) <= 1e-3 + 1e-3 * sum(t)
    assert t[1] > 0  # the evaluation kernel runs between events 1 and 2
    # event 4 (the edge image done) lies between events 0 and 1
    e4 = (ev[0].elapsed_time(ev[4]), ev[4].elapsed_time(ev[1]))
    assert min(e4) >= 0 and abs(sum(e4) - t[0]) <= 1e-3 + 1e-3 * t[0]
    if multires:
        assert e4[0] > 0 and e4[1] > 0  # the edge kernel, then the ranking
    fr.set_stage_events(None)
    assert torch.equal(fr(), ref)
    dv = [mr.DeviceEvent() for _ in range(mr.MR_FRAME_EVENTS)]
    fr.set_stage_events(dv)
    out = fr().clone()
    torch.cuda.synchronize()
    fr.set_stage_events(None)
    assert torch.equal(out, ref)
    t = [dv[k].elapsed_ms(dv[k + 1]) for k in range(3)]
    assert all(x >= 0 for x in t) and t[1] > 0


def test_fast_reciprocal_is_exact_over_its_range():
    """The evaluators replace the IEEE division 1/d by the hardware reciprocal
    and one Newton-Raphson step on [2^-126, 2^126); every float there must
    give the same bits (native program built with the library's flags)."""
    import os
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "_bin", "recip_check")
    assert os.path.exists(exe), "tests/native programs are not built (run __graft_entry__.build())"
    log("[gpu] recip_check (exhaustive)")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    log(r.stdout.strip())
    assert r.returncode == 0 and "mismatches 0" in r.stdout, r.stdout + r.stderr


def test_errors_enqueue_nothing():
    log("[gpu] error paths")
    c = case("256_3lv")
    masks = mr.alloc_masks(c["W"], c["H"], c["gb"].focal, c["mp"], DEV)
    masks.edge.fill_(7)
    bad = mr.MaskParams(num_levels=3, level_enable=0b111, sigma2=(0.924, 1.848, 0.0), weight=(100, -1, 1),
                        normal_cos=COS25)
    with pytest.raises(mr.MRError) as e:
        mr.mr_build_masks(c["d"], c["n"], c["gb"].focal, bad, masks=masks)
    assert e.value.status == mr.MR_E_PARAM
    small = torch.empty(16, dtype=torch.uint8, device=DEV)
    m2 = mr.alloc_masks(c["W"], c["H"], c["gb"].focal, c["mp"], DEV)
    m2.workspace = small
    m2.edge.fill_(7)
    with pytest.raises(mr.MRError) as e:
        mr.mr_build_masks(c["d"], c["n"], c["gb"].focal, c["mp"], masks=m2)
    assert e.value.status == mr.MR_E_WORKSPACE
    torch.cuda.synchronize()
    assert int((masks.edge != 7).sum()) == 0 and int((m2.edge != 7).sum()) == 0
