"""Compact frame path with a stencil that covers most of a ranking tile.

Depth noise over the left half of a 1024 x 64 frame puts nearly every texel
of level 1 there on the stencil (Sec. 3.1 edges, Sec. 4.1 stencil), so the
ranking tiles of 512 x 32 texels on that side hold more list entries than a
tile builds in LDS and store them directly, while the tiles on the smooth
side build theirs in LDS.  Both run in one frame, which must equal the
oracle's bit for bit: the level map, the frame path's lists, stencil words
and ranks (in ranking-tile order, see listcheck.py) and the image."""
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
W, H = 1024, 64
TILE_W, TILE_H = 512, 32    # texels of a ranking tile at level 1 (16 x 32 words)
STAGED_MAX = 8192           # entries a ranking tile builds in LDS


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gbuffer(seed):
    rng = np.random.default_rng(seed)
    depth = np.full((H, W), 6.0, np.float32)
    depth[:, : W // 2] = (4.0 + 4.0 * rng.random((H, W // 2))).astype(np.float32)
    normal = np.zeros((3, H, W), np.float32)
    normal[2] = 1.0
    return depth, normal, scenegen.focal_px(H)


def params(lib):
    t = scenegen.TABLE1["ssao"]
    return lib.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


@pytest.mark.parametrize("seed", [3, 4])
def test_dense_and_sparse_ranking_tiles_in_one_frame(seed):
    depth, normal, focal = gbuffer(seed)
    K = scenegen.ssao_kernel(8)
    ref = oracle.frame("ssao", depth, normal, focal, params(oracle), oracle.SSAOParams(K, 1.0, 0.02))
    s1 = ref.pyramid.stencil[1]
    # the case this test is for: a tile over the noise holds more entries
    # than are built in LDS, a tile on the smooth side fewer
    assert int(s1[:TILE_H, :TILE_W].sum()) > STAGED_MAX
    assert int(s1[:TILE_H, TILE_W:].sum()) <= STAGED_MAX
    log(f"[gpu] dense stencil {W}x{H} seed={seed}")
    d = torch.from_numpy(depth).to(DEV)
    n = torch.from_numpy(normal).to(DEV)
    k = torch.from_numpy(K).to(DEV)
    lm = torch.empty((H, W), dtype=torch.uint8, device=DEV)
    fr = mr.FrameRunner("ssao", d, n, focal, params(mr), True, params=mr.ssao_params(k, 1.0, 0.02), level_map=lm)
    out = fr()
    torch.cuda.synchronize()
    assert np.array_equal(lm.cpu().numpy(), ref.pyramid.level_map)
    check_frame_lists(fr.lists(), ref.pyramid)
    got = out.cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)
