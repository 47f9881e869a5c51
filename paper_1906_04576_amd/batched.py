"""Batched SSGI over frames of uneven sizes: one launch per stage for all
frames (mr_batch_setup / mr_batch_run), the launch configuration chosen by
the autotuner (mr_batch_tune), one batch run captured in a HIP graph.

Workload: 24 seeded frames, sizes drawn uniformly from 640x360, 1280x720,
1920x1080, 2560x1440 and 3840x2160, each a box/sphere scene (200 boxes + 50
spheres) with a Lambert-lit FP16 colour buffer; SSGI with 64 samples and
radius 2.0, 4 levels with the SSGI column of Table 1 (level 2 left out).

    python -m paper_1906_04576_amd.batched
prints one JSON line: the graph-replayed batch against the same frames run
one after another through mr_frame and against the naive full-resolution
pass, in Mpixels/s.
"""
from __future__ import annotations

import json
import math
import sys
import time

import numpy as np
import torch

from . import mr

SIZES = ((640, 360), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))
FRAMES = 24
SAMPLES = 64
RADIUS = 2.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_frames(n=FRAMES, seed=24, device="cuda"):
    import scenegen
    rng = np.random.default_rng(seed)
    pick = rng.integers(len(SIZES), size=n)
    frames = []
    for k in range(n):
        W, H = SIZES[pick[k]]
        sc = scenegen.make_scene(1000 + k, 200, 50)
        gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(k % 8), W, H)
        col = scenegen.lambert_color(sc, gb)
        frames.append(dict(depth=torch.from_numpy(gb.depth).to(device), normal=torch.from_numpy(gb.normal).to(device),
                           color=torch.from_numpy(col).to(device), focal=float(gb.focal)))
    return frames


def mask_params():
    import scenegen
    t = scenegen.TABLE1["ssgi"]
    return mr.MaskParams(num_levels=4, level_enable=0b1101, sigma2=t["sigma2"], weight=t["weight"],
                         normal_cos=float(np.float32(math.cos(math.radians(25.0)))))


def _wall(fn, steps):
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / steps


def measure(steps=20, frames=None, device="cuda"):
    import scenegen
    t0 = time.time()
    frames = frames or make_frames(device=device)
    npx = sum(f["depth"].numel() for f in frames)
    log(f"[batched] {len(frames)} frames, {npx / 1e6:.1f} Mpixels, resident in {time.time() - t0:.1f}s")
    mp = mask_params()
    p = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(SAMPLES)).to(device), RADIUS, 0.02)

    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b = mr.Batch("ssgi", frames, mp, p, stream=st)
        b(st)
        t_default = _wall(lambda: b(st), steps)
        cfg = b.tune(reps=3, stream=st)
        t_tuned = _wall(lambda: b(st), steps)
    st.synchronize()

    def graph_time(config):
        b.config = config
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=st):
            b(st)
        gr.replay()
        t = _wall(gr.replay, steps)
        b.check(st)  # no wait of a persistent run gave up
        return gr, t

    # the staged launches and the persistent launch, each with the tuner's
    # other choices, both replayed from graphs; the tuned one is kept
    t_mode = {}
    for mode in (0, 1):
        _, t_mode[mode] = graph_time(dict(cfg, persistent=mode))
    g, t_graph = graph_time(cfg)
    log(f"[batched] batch {t_default * 1e3:.3f} ms (default config), {t_tuned * 1e3:.3f} ms (tuned {cfg}), "
        f"{t_graph * 1e3:.3f} ms (graph); staged {t_mode[0] * 1e3:.3f} ms, persistent {t_mode[1] * 1e3:.3f} ms")

    # the same frames one after another (one workspace), and the naive pass
    nws = max(mr.mr_workspace_bytes(f["depth"].shape[1], f["depth"].shape[0], f["focal"], mp, mr.MR_EFFECT_SSGI)
              for f in frames)
    ws = torch.empty(nws, dtype=torch.uint8, device=device)
    seq = [mr.FrameRunner("ssgi", f["depth"], f["normal"], f["focal"], mp, True, color=f["color"], params=p,
                          workspace=ws) for f in frames]
    plain = [mr.FrameRunner("ssgi", f["depth"], f["normal"], f["focal"], mp, False, color=f["color"], params=p)
             for f in frames]

    def run_all(rs):
        for r in rs:
            r()

    run_all(seq)
    t_seq = _wall(lambda: run_all(seq), steps)
    run_all(plain)
    t_plain = _wall(lambda: run_all(plain), max(1, steps // 4))
    log(f"[batched] one after another {t_seq * 1e3:.3f} ms, naive {t_plain * 1e3:.3f} ms")

    # the batch's outputs equal the frames run alone
    g.replay()
    torch.cuda.synchronize()
    outs = [o.clone() for o in b.outs]
    run_all(seq)
    torch.cuda.synchronize()
    same = all(torch.equal(o, r.out) for o, r in zip(outs, seq))
    return {
        "workload": f"{len(frames)} SSGI frames of uneven sizes (640x360..3840x2160), {SAMPLES} samples "
                    f"r={RADIUS}, 4 levels, FP16 colour",
        "frames": len(frames), "mpixels": round(npx / 1e6, 3),
        "batch_ms": round(t_graph * 1e3, 4), "mpixels_s": round(npx / t_graph / 1e6, 2),
        "batch_default_config_ms": round(t_default * 1e3, 4), "batch_tuned_eager_ms": round(t_tuned * 1e3, 4),
        "tuned_config": cfg,
        "staged_graph_ms": round(t_mode[0] * 1e3, 4), "persistent_graph_ms": round(t_mode[1] * 1e3, 4),
        "sequential_ms": round(t_seq * 1e3, 4), "sequential_mpixels_s": round(npx / t_seq / 1e6, 2),
        "plain_ms": round(t_plain * 1e3, 4), "plain_mpixels_s": round(npx / t_plain / 1e6, 2),
        "speedup_vs_plain": round(t_plain / t_graph, 3), "speedup_vs_sequential": round(t_seq / t_graph, 3),
        "identical_to_frames_alone": bool(same),
    }


def measure_ssao(steps=20, frames=None, device="cuda", samples=32):
    """The same uneven frames as one SSAO batch (Table 1 SSAO masks, all four
    levels): graph-replayed staged launches with the dense coarsest level's
    depth gathered from the plane (eval_halo 0) and from LDS tiles with a halo
    of 8, 16 and 24 texels, the tuner's choice, and the frames one after
    another."""
    import scenegen
    frames = [dict(f, color=None) for f in (frames or make_frames(device=device))]
    npx = sum(f["depth"].numel() for f in frames)
    t = scenegen.TABLE1["ssao"]
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"],
                       normal_cos=float(np.float32(math.cos(math.radians(25.0)))))
    p = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(samples)).to(device), 1.0, 0.02)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b = mr.Batch("ssao", frames, mp, p, stream=st)
        b(st)
    st.synchronize()
    ms, outs = {}, {}
    for h in (0, 8, 16, 24):
        b.config = dict(eval_halo=h)
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr, stream=st):
            b(st)
        gr.replay()
        ms[h] = round(_wall(gr.replay, steps) * 1e3, 4)
        outs[h] = [o.clone() for o in b.outs]
    b.config = dict(eval_halo=0)
    with torch.cuda.stream(st):
        cfg = b.tune(reps=3, stream=st)
    st.synchronize()
    gr = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gr, stream=st):
        b(st)
    gr.replay()
    t_tuned = _wall(gr.replay, steps)
    nws = max(mr.mr_workspace_bytes(f["depth"].shape[1], f["depth"].shape[0], f["focal"], mp, mr.MR_EFFECT_SSAO)
              for f in frames)
    ws = torch.empty(nws, dtype=torch.uint8, device=device)
    seq = [mr.FrameRunner("ssao", f["depth"], f["normal"], f["focal"], mp, True, params=p, workspace=ws)
           for f in frames]

    def run_all():
        for r in seq:
            r()

    run_all()
    t_seq = _wall(run_all, steps)
    same = True
    for r, k in zip(seq, range(len(seq))):
        r()
        torch.cuda.synchronize()
        same = same and all(torch.equal(outs[h][k], r.out) for h in outs)
    log(f"[batched] SSAO batch ms by eval_halo {ms}, tuned {cfg} {t_tuned * 1e3:.3f} ms, "
        f"one after another {t_seq * 1e3:.3f} ms")
    return {
        "workload": f"{len(frames)} SSAO frames of uneven sizes (640x360..3840x2160), {samples} samples r=1.0, "
                    f"4 levels",
        "mpixels": round(npx / 1e6, 3), "graph_ms_by_eval_halo": {str(h): v for h, v in ms.items()},
        "mpixels_s": round(npx / (ms[0] * 1e-3) / 1e6, 2), "tuned_config": cfg,
        "tuned_graph_ms": round(t_tuned * 1e3, 4), "tuned_mpixels_s": round(npx / t_tuned / 1e6, 2),
        "sequential_ms": round(t_seq * 1e3, 4), "speedup_vs_sequential": round(t_seq * 1e3 / ms[0], 3),
        "identical_to_frames_alone": bool(same),
    }


def main():
    print(json.dumps(measure()), flush=True)


if __name__ == "__main__":
    main()
