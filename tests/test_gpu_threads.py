"""mr_frame from several host threads at once, each with its own stream,
workspace and output (the calls release the interpreter lock, so they run
in the library concurrently): every frame equals the same frame run alone,
for SSAO on the compact path, SSGI, PCSS on the dense path and the naive
pass."""
import math
import sys
import threading

import numpy as np
import pytest
import torch

import scenegen
from paper_1906_04576_amd import mr

pytestmark = pytest.mark.gpu

DEV = "cuda"
COS25 = float(np.float32(math.cos(math.radians(25.0))))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def runner(effect, W, H, seed, multires=True):
    sc = scenegen.make_scene(seed, 80, 20)
    gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(seed % 8), W, H)
    t = scenegen.TABLE1[effect]
    mp = mr.MaskParams(num_levels=4, level_enable=0b1101 if effect == "ssgi" else 0b1111, sigma2=t["sigma2"],
                       weight=t["weight"], normal_cos=COS25)
    d, n = torch.from_numpy(gb.depth).to(DEV), torch.from_numpy(gb.normal).to(DEV)
    color = None
    if effect == "shadow":
        si = scenegen.render_shadow_inputs(sc, gb.view, 512)
        sp = mr.shadow_params(torch.from_numpy(si.shadow_map).to(DEV), si.view_to_light, si.light_focal,
                              si.light_size, si.light_near, 0.05,
                              torch.from_numpy(scenegen.disk_samples(16, 11)).to(DEV),
                              torch.from_numpy(scenegen.disk_samples(32, 12)).to(DEV))
    else:
        sp = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(16, seed=seed)).to(DEV), 1.0, 0.02)
        if effect == "ssgi":
            color = torch.from_numpy(scenegen.lambert_color(sc, gb)).to(DEV)
    return mr.FrameRunner(effect, d, n, gb.focal, mp, multires, color, sp), (d, n, color, sp)


def test_frames_from_four_threads_equal_frames_alone():
    cases = [("ssao", 640, 360, 3, True), ("ssgi", 384, 256, 4, True), ("shadow", 320, 184, 5, True),
             ("ssao", 256, 256, 6, False)]
    runs = [runner(*c) for c in cases]
    refs = []
    for r, _ in runs:
        refs.append(r().clone())
    torch.cuda.synchronize()
    log("[gpu] four threads, 25 frames each")
    bad = []
    gate = threading.Barrier(len(runs), timeout=120)

    def work(k):
        try:
            r = runs[k][0]
            st = torch.cuda.Stream()
            gate.wait()
            for i in range(25):
                with torch.cuda.stream(st):
                    r.out.fill_(float("nan"))  # a frame that wrote nothing would not pass
                r(st)
                st.synchronize()
                if not torch.equal(r.out, refs[k]):
                    bad.append((k, i))
        except Exception as e:  # a thread that raised must fail the test
            bad.append((k, repr(e)))

    ts = [threading.Thread(target=work, args=(k,)) for k in range(len(runs))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not bad, bad[:8]
