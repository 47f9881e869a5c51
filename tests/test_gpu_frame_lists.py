"""Work lists of the timed frame path (Sec. 4.1: the stencil texels each
level renders), read back from mr_frame's workspace and compared bit for bit
with the oracle's stencils: the list in ranking-tile order (a fixed
permutation of the row-major list, see listcheck.py), the stencil words and
the per-word ranks.  Also: the same lists on every run, and the frame image
against the oracle, at the 1080p workload and the 4K headline workload (the
scene generator with 200 boxes and 50 spheres, 4 levels, SSAO with 32
samples, radius 1.0)."""
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

CASES = {
    # name: (W, H, boxes, spheres, seed, camera, samples, radius)
    "384x200": (384, 200, 40, 10, 9, 2, 16, 0.8),
    "640x360": (640, 360, 60, 15, 8, 5, 16, 1.0),
    "1080p": (1920, 1080, 200, 50, 1, 0, 32, 1.0),
    "4k_seed2_cam3": (3840, 2160, 200, 50, 2, 3, 32, 1.0),
    "4k_seed3_cam6": (3840, 2160, 200, 50, 3, 6, 32, 1.0),
}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def params(lib):
    t = scenegen.TABLE1["ssao"]
    return lib.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


@pytest.mark.parametrize("name", list(CASES))
def test_frame_path_lists_and_image_match_the_oracle(name):
    W, H, nb, ns, seed, cam, S, r = CASES[name]
    log(f"[gpu] frame lists {name} {W}x{H}")
    scene = scenegen.make_scene(seed, nb, ns)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(cam), W, H)
    K = scenegen.ssao_kernel(S)
    ref = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, params(oracle), oracle.SSAOParams(K, r, 0.02))
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    k = torch.from_numpy(K).to(DEV)
    fr = mr.FrameRunner("ssao", d, n, gb.focal, params(mr), True, params=mr.ssao_params(k, r, 0.02))
    fr()
    torch.cuda.synchronize()
    first = fr.lists()
    check_frame_lists(first, ref.pyramid)
    got = fr.out.cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)
    # run to run: the same lists after other frames have used the GPU
    for _ in range(3):
        fr()
    torch.cuda.synchronize()
    again = fr.lists()
    for i in first:
        for a, b in zip(first[i], again[i]):
            assert np.array_equal(a, b), f"level {i} changed between runs"
    assert np.array_equal(fr.out.cpu().numpy(), got)


@pytest.mark.parametrize("W,H", [(16384, 512), (512, 16384)])
def test_maximum_dimensions(W, H):
    """Width or height at MR_MAX_DIM (16384): rows of 512 words, 128
    ranking tiles across a level-1 row, 2048 edge tiles down a column.  The
    frame path's lists and image and the naive pass equal the oracle's."""
    assert max(W, H) == mr.MR_MAX_DIM
    log(f"[gpu] maximum dimensions {W}x{H}")
    scene = scenegen.make_scene(5, 200, 50)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(4), W, H)
    K = scenegen.ssao_kernel(16)
    op = oracle.SSAOParams(K, 1.0, 0.02)
    ref = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, params(oracle), op)
    ref_plain = oracle.frame("ssao", gb.depth, gb.normal, gb.focal, params(oracle), op, multires=False).out
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    p = mr.ssao_params(torch.from_numpy(K).to(DEV), 1.0, 0.02)
    fr = mr.FrameRunner("ssao", d, n, gb.focal, params(mr), True, params=p)
    fr()
    torch.cuda.synchronize()
    check_frame_lists(fr.lists(), ref.pyramid)
    assert np.array_equal(fr.out.cpu().numpy(), ref.out)
    plain = mr.FrameRunner("ssao", d, n, gb.focal, params(mr), False, params=p)()
    torch.cuda.synchronize()
    assert np.array_equal(plain.cpu().numpy(), ref_plain)


@pytest.mark.parametrize("effect", ["ssao", "ssgi"])
def test_largest_frame(effect):
    """A 16384 x 16384 frame (MR_MAX_DIM in both directions: 268 M pixels;
    the third FP32 normal plane, and for SSGI the third output plane, start
    2^31 bytes in).  The oracle cannot run a whole frame of this size, so the
    checks are ones that hold at any size: the naive pass at sampled pixels
    equals the oracle's estimator there (it gathers from the full level
    images), and at every edge pixel of six windows (the oracle's edge image
    of the window; a_1 w_1 >= 1 there, so Eq. 1 returns c_1 exactly) the
    multi-resolution image equals the naive pass and the pixel's owner level
    is 1."""
    W = H = mr.MR_MAX_DIM
    log(f"[gpu] largest frame {effect} {W}x{H}")
    scene = scenegen.make_scene(6, 200, 50)
    gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(1), W, H)
    K = scenegen.ssao_kernel(16)
    col = scenegen.lambert_color(scene, gb) if effect == "ssgi" else None
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0xF
    mpg = mr.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)
    d = torch.from_numpy(gb.depth).to(DEV)
    n = torch.from_numpy(gb.normal).to(DEV)
    c = torch.from_numpy(col).to(DEV) if col is not None else None
    p = mr.ssao_params(torch.from_numpy(K).to(DEV), 1.0, 0.02)
    lm = torch.zeros((H, W), dtype=torch.uint8, device=DEV)
    multi = mr.FrameRunner(effect, d, n, gb.focal, mpg, True, color=c, params=p, level_map=lm)().cpu().numpy()
    plain = mr.FrameRunner(effect, d, n, gb.focal, mpg, False, color=c, params=p)().cpu().numpy()
    owner = lm.cpu().numpy()
    del d, n, c, lm
    torch.cuda.empty_cache()
    rng = np.random.default_rng(16384)
    ys = np.concatenate([rng.integers(0, H, 1500), [0, H - 1, 0, H - 1]])
    xs = np.concatenate([rng.integers(0, W, 1500), [0, 0, W - 1, W - 1]])
    if effect == "ssao":
        ref = oracle.ssao_texels(gb.depth, gb.normal, gb.focal, 1, xs, ys, oracle.SSAOParams(K, 1.0, 0.02))
        assert np.array_equal(plain[ys, xs], ref.astype(np.float32))
    else:
        ref = oracle.ssgi_texels(gb.depth, gb.normal, col.astype(np.float32), gb.focal, 1, xs, ys,
                                 oracle.SSGIParams(K, 1.0, 0.02))
        assert np.array_equal(plain[:, ys, xs], ref.astype(np.float32))
    omp = params(oracle)
    edges = 0
    for (y0, x0) in ((0, 0), (8000, 8000), (H - 1024, W - 1024), (4096, 12000), (12000, 2000), (2000, 6000)):
        y1, x1 = y0 + 1024, x0 + 1024
        ya, xa = max(y0 - 1, 0), max(x0 - 1, 0)
        E = oracle.edge_image(gb.depth[ya:y1 + 1, xa:x1 + 1], gb.normal[:, ya:y1 + 1, xa:x1 + 1],
                              omp.depth_ratio, omp.normal_cos)
        # the window's core: every pixel's neighbours lie in the one-pixel
        # margin computed around it (or outside the image, as for the whole
        # image), so its edge value is the whole image's
        ey, ex = np.nonzero(E[y0 - ya:y0 - ya + 1024, x0 - xa:x0 - xa + 1024])
        ey, ex = ey + y0, ex + x0
        edges += len(ey)
        assert np.array_equal(multi[..., ey, ex], plain[..., ey, ex])
        assert np.all(owner[ey, ex] == 1)
    log(f"[gpu] {edges} edge pixels checked")
    assert edges > 300
