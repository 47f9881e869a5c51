"""Single frames captured in a HIP graph (torch.cuda.graph): mr_frame with a
workspace and mr_frame_static (the entry point for callers that cannot
allocate, such as code under capture).  Each graph is replayed several times
with new inputs copied in and eager frames run in between; every replay
equals an eager run of the same inputs, and the first also equals the
oracle.  The frame path clears its counters inside its kernels, so a replay
starts from the same state as an eager run."""
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


def views(W, H, effect):
    s = scenegen.make_scene(11, 120, 30)
    out = []
    for cam in (0, 3, 5, 7):
        gb = scenegen.render_gbuffer(s, scenegen.orbit_view(cam), W, H)
        col = scenegen.lambert_color(s, gb) if effect == "ssgi" else None
        out.append((gb, col))
    return out


def masks(lib, effect):
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0xF
    return lib.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"], normal_cos=COS25)


@pytest.mark.parametrize("effect,W,H,static", [("ssao", 640, 360, False), ("ssgi", 384, 200, False),
                                               ("ssao", 640, 360, True)])
def test_captured_frame_replays_to_eager(effect, W, H, static):
    log(f"[gpu] graph of one {effect} frame {W}x{H} static={static}")
    vs = views(W, H, effect)
    gb0, col0 = vs[0]
    d = torch.from_numpy(gb0.depth).to(DEV)
    n = torch.from_numpy(gb0.normal).to(DEV)
    c = torch.from_numpy(col0).to(DEV) if col0 is not None else None
    K = scenegen.ssao_kernel(16)
    p = mr.ssao_params(torch.from_numpy(K).to(DEV), 1.0, 0.02)
    Runner = mr.StaticFrameRunner if static else mr.FrameRunner
    fr = Runner(effect, d, n, gb0.focal, masks(mr, effect), True, color=c, params=p)
    # an eager runner on separate buffers gives the reference of each replay
    de, ne = d.clone(), n.clone()
    ce = c.clone() if c is not None else None
    eager = mr.FrameRunner(effect, de, ne, gb0.focal, masks(mr, effect), True, color=ce, params=p)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        fr(st)  # first call outside the capture (the static entry point sets up its scratch)
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        fr(st)
    for rep, (gb, col) in enumerate(vs + vs[:1]):
        for dst, src in ((d, gb.depth), (n, gb.normal)) + (((c, col),) if c is not None else ()):
            dst.copy_(torch.from_numpy(src).to(DEV))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = fr.out.clone()
        de.copy_(d)
        ne.copy_(n)
        if c is not None:
            ce.copy_(c)
        ref = eager()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
        if rep == 0:
            op = (oracle.SSGIParams if effect == "ssgi" else oracle.SSAOParams)(K, 1.0, 0.02)
            want = oracle.frame(effect, gb.depth, gb.normal, gb.focal, masks(oracle, effect), op, color=col).out
            assert np.array_equal(got.cpu().numpy(), want)
