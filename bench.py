#!/usr/bin/env python3
"""Multi-resolution vs naive full-resolution SSAO at 3840x2160 on one MI355X.

Workload: the seeded box/sphere scene generator (200 boxes + 50 spheres on a
ground plane) at 3840x2160, 4 levels (full, 1/2, 1/4, 1/8) with the SSAO
column of Table 1, SSAO with 32 samples and radius 1.0, edge thresholds 0.05
(depth ratio) and 25 degrees (normals).  3 scene seeds x 8 orbit cameras = 24
configurations stay resident in HBM (3.2 GB, far above the 256 MB
Infinity Cache) and the timed frames cycle through them.

One step = one multi-resolution frame through mr_frame: edge image + level
G-buffers, mask blur/stencils, work-list compaction, per-level SSAO and the
Eq. 1 merge.  The naive full-resolution pass is timed the same way for the
speedup.  Progress goes to stderr; stdout gets one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
# FP32 arithmetic pipe: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one non-fused,
# non-packed FP32 add / multiply / divide step per lane and clock (the
# bit-exact contract rules out FMA contraction and packed FP32): 157.3 TFLOP/s
# / 4.  A stream of independent v_add_f32 ran at 37.7 T lane-ops/s on an MI355X
# (4.17 cycles per wave64 instruction).
FP32_PIPE_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic FP32 arithmetic of the SSAO estimator (Sec. 2.4 reading):
# per sample the sample point (9 multiplies + 9 adds), the reciprocal of its
# depth, the projection (2 x (2 multiplies + 1 add)), the biased depth
# (multiply + subtract) and the range difference (subtract) = 28; per texel
# the view position (2 x (add, subtract, divide) + 2 multiplies), the
# tangent frame (13), the scaled frame (9 multiplies) and the final divide
# = 31.  Tests, floors, conversions and the count are not FP32 arithmetic.
SSAO_FP32_PER_SAMPLE = 28
SSAO_FP32_PER_TEXEL = 31
# HBM bytes per launch of the dominant kernel from the FETCH_SIZE and
# WRITE_SIZE counters (profiles/ssao_4k_hbm_counters.md), scaled by the
# copy-kernel calibration
TRAFFIC_BYTES = {"k_ssao_multi": 61812084}
# VALU wave instructions per launch (SQ_INSTS_VALU,
# profiles/ssao_4k_eval_valu_issue.md) of the multi-resolution evaluation and
# of the naive pass, which runs the same per-sample code densely over every
# pixel: the ratio of their instruction rates is the launch's VALU issue
# relative to the rate that code sustains
VALU_INSTS = {"k_ssao_multi": 20600129, "k_ssao_plain": 206263552}
# the counters above hold for the kernels of this machine code only: the
# SHA-256 of the gfx950 code built from k_ssao.hip (libmr.code.json) when
# they were taken.  Any other code reports them as null.
COUNTER_CODE = {"k_ssao_multi": ("k_ssao.hip", "541f790742ecc6e2535f3fe93b9d578eea324b7db4de9de0325f33b68d3b06fb")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def built_code_sha256(src, path=None):
    """SHA-256 of a source's gfx950 machine code in the built library
    (libmr.code.json, written by the build), or None."""
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1906_04576_amd", "libmr.code.json")
    try:
        with open(path) as f:
            return json.load(f).get(src)
    except (OSError, ValueError):
        return None


def counters_current(kernel, path=None):
    src, digest = COUNTER_CODE[kernel]
    return built_code_sha256(src, path) == digest


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=240)
    ap.add_argument("--warmup", type=int, default=12)
    ap.add_argument("--width", type=int, default=3840)
    ap.add_argument("--height", type=int, default=2160)
    ap.add_argument("--samples", type=int, default=32)
    ap.add_argument("--radius", type=float, default=1.0)
    ap.add_argument("--seeds", type=int, default=3)
    ap.add_argument("--cameras", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stages", action="store_true")
    ap.add_argument("--streams", type=int, default=2,
                    help="also report throughput with frames spread over this many streams (1 = off)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the paper variants (bilateral blur, foveated mask, fewer samples at full resolution)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched uneven-frame SSGI and SSAO measurements (24 frames, 640x360..3840x2160)")
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the sample-count sweep (16..256 at 4K) and the resolution sweep (720p..4K at S = 64)")
    ap.add_argument("--no-pcss", action="store_true",
                    help="skip the 4K soft-shadow frames (2048^2 map, 16 + 32 samples, FP16 normals)")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-loop measurement")
    ap.add_argument("--no-quality", action="store_true", help="profile helper: skip the multi vs naive comparison")
    ap.add_argument("--plain", action="store_true", help="profile helper: time only the naive pass")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profile helper: first run a 256 MiB device-to-device copy (known HBM traffic)")
    return ap.parse_args()


def _wall(fn, steps, warm=2):
    """Seconds per call of fn over `steps` calls, between device syncs."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _cycle(runners):
    """Callable running the next runner of the list on each call."""
    state = {"k": 0}

    def go():
        runners[state["k"] % len(runners)]()
        state["k"] += 1
    return go


def sweep_samples(frames, W, H, focal, mp, dev, samples=(16, 32, 64, 128, 256), radius=1.0):
    """4K frame time, multi-resolution and naive, for every SSAO sample count
    (the analogue of the paper's speedup-vs-samples figure), over the
    resident configurations; RMS of multi-res vs naive on 4 of them."""
    import torch
    import scenegen
    from paper_1906_04576_amd import mr
    ws = torch.empty(mr.mr_workspace_bytes(W, H, focal, mp, mr.MR_EFFECT_SSAO), dtype=torch.uint8, device=dev)
    res = []
    for S in samples:
        sp = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(S)).to(dev), radius, 0.02)
        multi = [mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, True, params=sp, workspace=ws) for f in frames]
        plain = [mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, False, params=sp) for f in frames]
        nf = len(frames)
        tm = _wall(_cycle(multi), 2 * nf)
        tp = _wall(_cycle(plain), max(nf // 2, 8) if S >= 128 else nf)
        rms = []
        for k in range(min(4, nf)):
            a = multi[k]().clone()
            b = plain[k]()
            rms.append(float((a - b).double().pow(2).mean().sqrt()))
        res.append({"samples": S, "multi_ms": round(tm * 1e3, 5), "plain_ms": round(tp * 1e3, 5),
                    "speedup": round(tp / tm, 3), "multi_mpixels_s": round(W * H / tm / 1e6, 2),
                    "rms_vs_plain": round(float(np.mean(rms)), 6)})
        log(f"[bench] sweep S={S}: multi {tm * 1e3:.4f} ms, naive {tp * 1e3:.4f} ms, {tp / tm:.2f}x")
    return res


def sweep_resolution(dev, samples=64, radius=1.0, cams=8):
    """Frame time at 720p .. 4K with 64 samples (the analogue of the
    paper's speedup-vs-resolution figure), scene seed 1, 8 cameras."""
    import torch
    import scenegen
    from paper_1906_04576_amd import mr
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=scenegen.TABLE1["ssao"]["sigma2"],
                       weight=scenegen.TABLE1["ssao"]["weight"])
    sp = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(samples)).to(dev), radius, 0.02)
    scene = scenegen.make_scene(1, 200, 50)
    res = []
    for (W, H) in ((1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)):
        gbs = [scenegen.render_gbuffer(scene, scenegen.orbit_view(c), W, H) for c in range(cams)]
        focal = gbs[0].focal
        ds = [(torch.from_numpy(g.depth).to(dev), torch.from_numpy(g.normal).to(dev)) for g in gbs]
        ws = torch.empty(mr.mr_workspace_bytes(W, H, focal, mp, mr.MR_EFFECT_SSAO), dtype=torch.uint8, device=dev)
        multi = [mr.FrameRunner("ssao", d, n, focal, mp, True, params=sp, workspace=ws) for d, n in ds]
        plain = [mr.FrameRunner("ssao", d, n, focal, mp, False, params=sp) for d, n in ds]
        tm = _wall(_cycle(multi), 4 * cams)
        tp = _wall(_cycle(plain), 2 * cams)
        res.append({"width": W, "height": H, "samples": samples, "multi_ms": round(tm * 1e3, 5),
                    "plain_ms": round(tp * 1e3, 5), "speedup": round(tp / tm, 3),
                    "multi_mpixels_s": round(W * H / tm / 1e6, 2)})
        log(f"[bench] sweep {W}x{H} S={samples}: multi {tm * 1e3:.4f} ms, naive {tp * 1e3:.4f} ms, {tp / tm:.2f}x")
    return res


def pcss_4k(dev, cams=4):
    """Soft shadows at 3840x2160: a 2048^2 shadow map from one square light
    of side 0.5, 16 blocker + 32 PCF samples, FP16 normals, 4 levels with the
    soft-shadow column of Table 1; frame time multi-res vs naive."""
    import torch
    import scenegen
    from paper_1906_04576_amd import mr
    w = scenegen.WORKLOADS["pcss_4k"]
    W, H = w["width"], w["height"]
    t = scenegen.TABLE1["shadow"]
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=t["sigma2"], weight=t["weight"])
    scene = scenegen.make_scene(2, w["boxes"], w["spheres"])
    bd = torch.from_numpy(scenegen.disk_samples(w["n_blocker"], 11)).to(dev)
    pd = torch.from_numpy(scenegen.disk_samples(w["n_pcf"], 12)).to(dev)
    multi, plain, keep = [], [], []
    ws = None
    for c in range(cams):
        gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(c), W, H)
        si = scenegen.render_shadow_inputs(scene, gb.view, w["sm_size"], light_size=w["light_size"])
        d = torch.from_numpy(gb.depth).to(dev)
        n = torch.from_numpy(gb.normal.astype(np.float16)).to(dev)
        sp = mr.shadow_params(torch.from_numpy(si.shadow_map).to(dev), si.view_to_light, si.light_focal,
                              si.light_size, si.light_near, 0.05, bd, pd)
        if ws is None:
            ws = torch.empty(mr.mr_workspace_bytes(W, H, gb.focal, mp, mr.MR_EFFECT_SHADOW), dtype=torch.uint8,
                             device=dev)
        multi.append(mr.FrameRunner("shadow", d, n, gb.focal, mp, True, params=sp, workspace=ws))
        plain.append(mr.FrameRunner("shadow", d, n, gb.focal, mp, False, params=sp))
        keep.append(sp)
    tm = _wall(_cycle(multi), 8 * cams)
    tp = _wall(_cycle(plain), 4 * cams)
    mad = float(np.mean([float((multi[k]().clone() - plain[k]()).double().abs().mean()) for k in range(cams)]))
    log(f"[bench] 4K PCSS: multi {tm * 1e3:.4f} ms, naive {tp * 1e3:.4f} ms, {tp / tm:.2f}x")
    return {"workload": f"pcss_4k: {W}x{H}, 2048^2 shadow map, 16 blocker + 32 PCF samples, FP16 normals, "
                        f"4 levels, {cams} cameras of scene seed 2",
            "multi_ms": round(tm * 1e3, 5), "plain_ms": round(tp * 1e3, 5), "speedup": round(tp / tm, 3),
            "multi_mpixels_s": round(W * H / tm / 1e6, 2), "mad_vs_plain": round(mad, 6)}


def serving(qps=4000.0, seconds=1.5):
    """The request loop (serve.py) on a Poisson stream: p50 / p99 latency and
    Mpixels/s on the same requests, multi-resolution with the scenes' mask
    pyramids resident, multi-resolution rebuilding the masks per request,
    multi-resolution with same-effect requests batched (up to 4 per launch
    set), and naive."""
    from paper_1906_04576_amd import serve
    pool = serve.Pool(2)
    reqs = serve.poisson_requests(pool, qps, seconds)
    out = {"qps": qps, "seconds": seconds, "requests": len(reqs), "slots": 4, "budget_gb": 64}
    for name, multires, resident, bmax in (("multires", True, True, 0), ("multires_rebuild", True, False, 0),
                                           ("multires_batched", True, True, 4), ("plain", False, False, 0)):
        srv = serve.Server(pool, 4, 64 << 30, multires, resident_masks=resident, batch_max=bmax)
        srv.run(reqs[: min(len(reqs), 64)])
        s_ = serve.summary(srv.run(reqs))
        s_["saturated_mpixels_s"] = serve.summary(srv.run(reqs, realtime=False))["mpixels_s"]
        out[name] = s_
        log(f"[bench] serving {name}: {s_}")
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the multi-resolution path is one frame per GPU "
              "and every frame fits one GPU; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import scenegen
    from paper_1906_04576_amd import mr

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration copy: 3 x 256 MiB device-to-device")
    W, H, S = args.width, args.height, args.samples
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=scenegen.TABLE1["ssao"]["sigma2"],
                       weight=scenegen.TABLE1["ssao"]["weight"])
    K = scenegen.ssao_kernel(S)
    kdev = torch.from_numpy(K).to(dev)
    sp = mr.ssao_params(kdev, args.radius, 0.02)

    # ---------------- resident inputs ----------------
    t0 = time.time()
    frames = []
    for seed in range(1, args.seeds + 1):
        scene = scenegen.make_scene(seed, 200, 50)
        for cam in range(args.cameras):
            gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(cam), W, H)
            frames.append(dict(seed=seed, cam=cam, gb=gb, d=torch.from_numpy(gb.depth).to(dev),
                               n=torch.from_numpy(gb.normal).to(dev)))
    focal = frames[0]["gb"].focal
    log(f"[bench] {len(frames)} configurations at {W}x{H} generated and resident in {time.time() - t0:.1f}s")

    ws = torch.empty(mr.mr_workspace_bytes(W, H, focal, mp, mr.MR_EFFECT_SSAO), dtype=torch.uint8, device=dev)
    multi = [mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, True, params=sp, workspace=ws) for f in frames]
    plain = [mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, False, params=sp) for f in frames]
    nf = len(frames)

    def timed(runners, steps, warm):
        """Throughput: `steps` frames back to back, bracketed by device
        synchronisations and nothing else on the stream.  Latency: the same
        frames again, each between two timing events (device-scope release);
        each event adds a few microseconds of its own to the stream.  Host
        latency: the same frames once more, each from before its ctypes call
        to the return of a device synchronisation after it (the submission
        alone is the time until the call returns)."""
        for k in range(warm):
            runners[k % nf]()
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(steps):
            runners[k % nf]()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        ev = [(mr.DeviceEvent(), mr.DeviceEvent()) for _ in range(steps)]
        stream = torch.cuda.current_stream()
        for k in range(steps):
            mr.record(ev[k][0], stream)
            runners[k % nf]()
            mr.record(ev[k][1], stream)
        torch.cuda.synchronize()
        lat = np.array([a.elapsed_ms(b) for a, b in ev])
        host = np.zeros((steps, 2))
        for k in range(steps):
            t0 = time.perf_counter()
            runners[k % nf]()
            t1 = time.perf_counter()
            torch.cuda.synchronize()
            host[k] = (t1 - t0, time.perf_counter() - t0)
        return wall, lat, host * 1e3

    def concurrent(multires, streams, steps):
        """Throughput with frames spread round robin over `streams` HIP
        streams (one workspace each), so that one frame's memory-bound stages
        overlap another's evaluation; reported beside the one-stream figure."""
        ss = [torch.cuda.Stream() for _ in range(streams)]
        nws = mr.mr_workspace_bytes(W, H, focal, mp, mr.MR_EFFECT_SSAO) if multires else 256
        wss = [torch.empty(nws, dtype=torch.uint8, device=dev) for _ in range(streams)]
        outs = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(streams)]
        rs = [[mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, multires, params=sp, workspace=wss[j], out=outs[j])
               for f in frames] for j in range(streams)]
        for k in range(streams * 4):
            rs[k % streams][k % nf](ss[k % streams])
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(steps):
            rs[k % streams][k % nf](ss[k % streams])
        torch.cuda.synchronize()
        return (time.perf_counter() - t_start) / steps

    if args.plain:
        wall, lat, _ = timed(plain, args.steps, args.warmup)
        log(f"[bench] plain {args.steps} frames {wall * 1e3 / args.steps:.3f} ms/frame")
        return

    wall_m, lat_m, host_m = timed(multi, args.steps, args.warmup)
    log(f"[bench] multi-res: {wall_m * 1e3 / args.steps:.3f} ms/frame")
    wall_p, lat_p, host_p = timed(plain, args.steps, args.warmup)
    log(f"[bench] plain:     {wall_p * 1e3 / args.steps:.3f} ms/frame")

    npx = W * H
    value = npx * args.steps / wall_m / 1e6
    plain_mpx = npx * args.steps / wall_p / 1e6
    conc = None
    if args.streams > 1:
        tm2 = concurrent(True, args.streams, args.steps)
        tp2 = concurrent(False, args.streams, args.steps)
        conc = {"streams": args.streams, "mpixels_s": round(npx / tm2 / 1e6, 2),
                "plain_mpixels_s": round(npx / tp2 / 1e6, 2), "speedup_vs_plain": round(tp2 / tm2, 3)}
        log(f"[bench] {args.streams} streams: multi-res {tm2 * 1e3:.3f} ms/frame, plain {tp2 * 1e3:.3f} ms/frame")

    # ---------------- paper variants on the same frames ----------------
    # bilateral blur of the SSAO sub-images, a foveated mask (gaze at the
    # centre), and the sub-images at full resolution with fewer samples
    # (S, S/2, S/4, S/8 per level) from the dense masks
    variants = None
    if not args.no_variants:
        def wall(runners, steps):
            for k in range(4):
                runners[k % nf]()
            torch.cuda.synchronize()
            t_start = time.perf_counter()
            for k in range(steps):
                runners[k % nf]()
            torch.cuda.synchronize()
            return (time.perf_counter() - t_start) / steps

        vsteps = max(24, args.steps // 4)
        variants = {}
        for name, bl in (("bilateral_levels_2_4", mr.Bilateral(levels=0b1110, radius=2)),
                         ("bilateral_all_levels", mr.Bilateral(levels=0b1111, radius=2))):
            rs = [mr.FrameRunner("ssao", f["d"], f["n"], focal, mp, True, params=sp, workspace=ws, bilateral=bl)
                  for f in frames]
            variants[name + "_ms"] = round(wall(rs, vsteps) * 1e3, 5)
        fmp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=mp.sigma2, weight=mp.weight,
                            fovea=(W / 2, H / 2, 0.15 * H, 0.45 * H))
        rs = [mr.FrameRunner("ssao", f["d"], f["n"], focal, fmp, True, params=sp, workspace=ws) for f in frames]
        variants["fovea_ms"] = round(wall(rs, vsteps) * 1e3, 5)
        Kl = {i: scenegen.ssao_kernel(max(1, S >> (i - 1)), seed=70 + i) for i in (1, 2, 3, 4)}
        Kd = {i: torch.from_numpy(Kl[i]).to(dev) for i in Kl}
        lp = {i: mr.ssao_params(Kd[i], args.radius, 0.02) for i in Kl}
        dmasks = mr.alloc_masks(W, H, focal, mp, dev, level_map=False)
        fr_out = torch.empty((H, W), dtype=torch.float32, device=dev)

        class _Full:
            def __init__(self, f):
                self.m = mr.prepare_build_masks(f["d"], f["n"], focal, mp, dmasks)
                self.e = mr.FullresRunner(f["d"], f["n"], focal, mp, dmasks, lp, out=fr_out)

            def __call__(self):
                self.m()
                return self.e()

        rs = [_Full(f) for f in frames]
        t_full = wall(rs, vsteps)
        mad_full = []
        for k in range(0 if args.no_quality else min(nf, 8)):
            a = rs[k]().clone()
            b = plain[k]()
            mad_full.append(float((a - b).double().abs().mean()))
        variants.update({"fullres_fewer_samples_ms": round(t_full * 1e3, 5),
                         "fullres_fewer_samples_mpixels_s": round(npx / t_full / 1e6, 2),
                         "fullres_fewer_samples_samples": [int(max(1, S >> (i - 1))) for i in (1, 2, 3, 4)],
                         "fullres_fewer_samples_mad_vs_plain": round(float(np.mean(mad_full)), 6) if mad_full else None})
        # the frame tuner (mr_frame_tune) on configuration 0: how the
        # coarsest level's evaluation gathers its depth
        tr = mr.FrameRunner("ssao", frames[0]["d"], frames[0]["n"], focal, mp, True, params=sp, workspace=ws)
        halo, ms = tr.tune(reps=20)
        variants["frame_tune"] = {"chosen_eval_halo": halo, "ms_per_eval_halo": {h: round(t, 5) for h, t in ms.items()}}
        log("[bench] variants: " + ", ".join(f"{k}={v}" for k, v in variants.items()))

    # ---------------- quality: multi-res vs naive on every configuration ----------------
    mads, rmss = [], []
    for k in range(0 if args.no_quality else nf):
        a = multi[k]().clone()
        b = plain[k]()
        diff = (a - b).double()
        mads.append(float(diff.abs().mean()))
        rmss.append(float(diff.pow(2).mean().sqrt()))

    # ---------------- per-stage GPU time of the same frames ----------------
    # mr_frame records the caller's events (device-scope release) at its
    # stage boundaries: [0] start, [1] masks and work lists done, [2]
    # per-level evaluation done (one kernel launch), [3] merge done.  Each
    # stage time is the event difference minus the stream time of one event.
    # A long naive frame is queued first so that the stream runs ahead of
    # the host and the events bracket back-to-back GPU work.
    stages = {}
    roofline = None
    if not args.no_stages:
        def stage_times(runners, reps):
            """Per frame, from the frame's five events: masks ([0] to [1]),
            evaluation ([1] to [2]), merge ([2] to [3]), edge image ([0] to
            [4]) and ranking ([4] to [1]); and the spacing of two events
            recorded back to back after it (the stream time one event takes;
            it sits inside every interval, twice inside the masks)."""
            sets = []
            stream = torch.cuda.current_stream()
            runners[0]()
            plain[0]()
            for rep in range(reps):
                for k in range(nf):
                    e = [mr.DeviceEvent() for _ in range(mr.MR_FRAME_EVENTS + 2)]
                    runners[k].set_stage_events(e[:mr.MR_FRAME_EVENTS])
                    runners[k]()
                    mr.record(e[5], stream)
                    mr.record(e[6], stream)
                    sets.append(e)
            torch.cuda.synchronize()
            for r in runners:
                r.set_stage_events(None)
            pairs = ((0, 1), (1, 2), (2, 3), (5, 6), (0, 4), (4, 1))
            return np.array([[e[a].elapsed_ms(e[b]) for a, b in pairs] for e in sets])  # ms

        reps = max(1, 96 // nf)
        tm = stage_times(multi, reps)
        tp = stage_times(plain, reps)
        ev_ms = float(np.median(np.concatenate([tm[:, 3], tp[:, 3]])))
        stages["multi_masks_ms"] = round(float(tm[:, 0].mean()) - 2 * ev_ms, 5)
        for j, nm in ((1, "eval"), (2, "merge"), (4, "edges"), (5, "rank")):
            stages[f"multi_{nm}_ms"] = round(float(tm[:, j].mean()) - ev_ms, 5)
        stages["plain_eval_ms"] = round(float(tp[:, 1].mean()) - ev_ms, 5)
        stages["event_ms"] = round(ev_ms, 5)
        stages["stage_samples"] = len(tm)

        # stencil coverage of every configuration (identical masks through the
        # separate mask entry point)
        masks = mr.alloc_masks(W, H, focal, mp, dev, level_map=False)
        counts = []
        for k in range(nf):
            f = frames[k]
            mr.prepare_build_masks(f["d"], f["n"], focal, mp, masks)()
            counts.append(masks.count[:3].clone())
        cnt = np.array([c.cpu().numpy().view(np.uint32) for c in counts], np.float64).mean(0)
        n = [npx >> (2 * (i - 1)) for i in (1, 2, 3, 4)]
        cov = [cnt[0] / n[0], cnt[1] / n[1], cnt[2] / n[2]]
        F = cov[0] + cov[1] / 4 + cov[2] / 16 + 1 / 64
        listed = cnt[0] + cnt[1] + cnt[2]
        evaluated = listed + n[3]
        nb = n[0] + n[1] + n[2]  # texels of the list levels (one bit each in the bit masks)
        # algorithmic bytes per stage of the multi-resolution frame:
        # compulsory reads and writes, sample gathers excluded
        b_edges = 16 * n[0] + nb / 8 + 4 * (n[1] + n[2] + n[3])  # G-buffer in, edge bits + level depth out
        b_rank = (nb / 8 + nb / 8                                 # stencil: edge bits in, stencil bits out
                  + nb / 8 + 4 * nb / 32 + 4 * listed)            # ranks and lists
        b_masks = b_edges + b_rank
        b_eval = 4 * listed + 16 * evaluated + nb / 8 + 4 * evaluated + 4 * listed
        b_merge = nb / 8 + 4 * nb / 32 + 8 * listed + 4 * n[3] + 4 * n[0]
        b_frame = b_masks + b_eval + b_merge
        t_frame = wall_m / args.steps
        ops_multi = evaluated * (SSAO_FP32_PER_SAMPLE * S + SSAO_FP32_PER_TEXEL)
        ops_plain = n[0] * (SSAO_FP32_PER_SAMPLE * S + SSAO_FP32_PER_TEXEL)
        t_eval = stages["multi_eval_ms"] * 1e-3
        stages.update({
            "coverage_f1_f2_f3": [round(c, 5) for c in cov], "F": round(F, 5),
            "evaluated_texels": int(evaluated),
            "frame_alg_bytes": int(b_frame),
            "frame_hbm_frac": round(b_frame / t_frame / (HBM_PEAK_GBS * 1e9), 4),
            "frame_hbm_frac_incl_gathers": round((b_frame + 4.0 * S * evaluated) / t_frame / (HBM_PEAK_GBS * 1e9), 4),
            "masks_hbm_frac": round(b_masks / (stages["multi_masks_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "edges_hbm_frac": round(b_edges / (stages["multi_edges_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "rank_hbm_frac": round(b_rank / (stages["multi_rank_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "merge_hbm_frac": round(b_merge / (stages["multi_merge_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "eval_multi_fp32_frac": round(ops_multi / t_eval / (FP32_PIPE_PEAK_TOPS * 1e12), 4),
            "eval_plain_fp32_frac": round(ops_plain / (stages["plain_eval_ms"] * 1e-3) / (FP32_PIPE_PEAK_TOPS * 1e12),
                                          4),
        })
        # dominant kernel of the multi-resolution frame: the per-level SSAO
        # evaluation, one launch per frame bracketed by events [1] and [2]
        achieved = ops_multi / t_eval / 1e12
        fresh = counters_current("k_ssao_multi")
        if not fresh:
            log("[bench] the evaluation kernels' machine code is not the one their counters were taken on: "
                "traffic and VALU issue are reported as null")
        roofline = {"kernel": "k_ssao<float, true, true> (all levels of one frame in one launch)", "bound": "alu",
                    "achieved": round(achieved, 3), "peak": round(FP32_PIPE_PEAK_TOPS, 2), "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_PIPE_PEAK_TOPS, 4), "traffic": TRAFFIC_BYTES.get("k_ssao_multi") if fresh else None,
                    "launch_ms": stages["multi_eval_ms"], "counters_match_code": fresh,
                    "basis": f"algorithmic FP32 arithmetic ({SSAO_FP32_PER_SAMPLE} per sample, "
                             f"{SSAO_FP32_PER_TEXEL} per texel) of {int(evaluated)} evaluated texels per launch "
                             "against the non-fused, non-packed FP32 pipe (157.3 TFLOP/s / 4)"}
        roofline["valu_rate_vs_plain"] = None
        if fresh:
            # VALU wave instructions per second of this launch against the
            # naive pass's, both from the counters and this run's launch times
            rate_m = VALU_INSTS["k_ssao_multi"] / t_eval
            rate_p = VALU_INSTS["k_ssao_plain"] / (stages["plain_eval_ms"] * 1e-3)
            roofline["valu_rate_vs_plain"] = round(rate_m / rate_p, 4)
        log("[bench] stages (ms): " + ", ".join(f"{k}={v}" for k, v in stages.items() if k.endswith("_ms")))

    # ---------------- batched uneven SSGI and SSAO frames (graph-replayed batches) ----------------
    batched = batched_ssao = None
    if not args.no_batch:
        from paper_1906_04576_amd import batched as batched_mod
        batched = batched_mod.measure(steps=20, device=dev)
        log(f"[bench] batched SSGI: {batched['mpixels_s']} Mpixels/s, {batched['speedup_vs_plain']}x naive, "
            f"{batched['speedup_vs_sequential']}x one after another")
        batched_ssao = batched_mod.measure_ssao(steps=20, device=dev)
        log(f"[bench] batched SSAO: {batched_ssao['mpixels_s']} Mpixels/s, by eval_halo "
            f"{batched_ssao['graph_ms_by_eval_halo']} ms, tuned eval_halo {batched_ssao['tuned_config']['eval_halo']}")

    # ---------------- sweeps, soft shadows at 4K, serving ----------------
    sweeps = None
    if not args.no_sweeps:
        sweeps = {"samples_4k": sweep_samples(frames, W, H, focal, mp, dev),
                  "resolution_s64": sweep_resolution(dev)}
    pcss = None if args.no_pcss else pcss_4k(dev)
    serving_res = None if args.no_serving else serving()

    # ---------------- CPU oracle: modes A and B at 1080p and 4K; quality at 1080p ----------------
    # The oracle runs in a child process that never touches the GPU
    # (oracle.timing): one warm-up and three runs of the multi-resolution
    # and naive frame of configuration 0's scene and camera, in one process
    # on one thread (mode A) and in row bands over one process per core the
    # host gives this job (mode B, bit-identical).  Its 1080p images are
    # compared with this path's at the same inputs.
    cpu = None
    cpu_protocol = None
    quality_1080p = None
    if not args.no_cpu_baseline:
        import subprocess
        import tempfile
        qW, qH = 1920, 1080
        gbq = scenegen.render_gbuffer(scenegen.make_scene(1, 200, 50), scenegen.orbit_view(0), qW, qH)
        dq, nq = torch.from_numpy(gbq.depth).to(dev), torch.from_numpy(gbq.normal).to(dev)
        gq = {key: mr.FrameRunner("ssao", dq, nq, gbq.focal, mp, key == "multires", params=sp)().cpu().numpy()
              for key in ("multires", "plain")}
        with tempfile.TemporaryDirectory() as tmp:
            cmd = [sys.executable, "-m", "oracle.timing", "--resolutions", f"{qW}x{qH},{W}x{H}",
                   "--samples", str(S), "--radius", str(args.radius), "--seed", "1", "--camera", "0",
                   "--save", tmp, "--save-res", f"{qW}x{qH}"]
            log("[bench] cpu oracle: " + " ".join(cmd[1:]))
            t_c = time.perf_counter()
            pr = subprocess.run(cmd, cwd=os.path.dirname(os.path.abspath(__file__)), stdout=subprocess.PIPE,
                                text=True, timeout=900)
            if pr.returncode != 0:
                raise RuntimeError(f"oracle timing exited with {pr.returncode}")
            cpu_protocol = json.loads(pr.stdout.strip().splitlines()[-1])
            cpu_protocol["seconds"] = round(time.perf_counter() - t_c, 1)
            ref = {key: np.load(os.path.join(tmp, f"oracle_{qW}x{qH}_{key}.npy")) for key in ("multires", "plain")}
        dm = gq["multires"].astype(np.float64)
        quality_1080p = {
            "resolution": f"{qW}x{qH}",
            "inputs": cpu_protocol["inputs"],
            "max_abs_multires_vs_oracle_multires": float(np.max(np.abs(dm - ref["multires"]))),
            "max_abs_plain_vs_oracle_plain": float(np.max(np.abs(gq["plain"].astype(np.float64) - ref["plain"]))),
            "mad_multires_vs_oracle_plain": round(float(np.mean(np.abs(dm - ref["plain"]))), 6),
            "rms_multires_vs_oracle_plain": round(float(np.sqrt(np.mean((dm - ref["plain"]) ** 2))), 6),
        }
        ma = cpu_protocol["resolutions"][f"{W}x{H}"]["mode_a"]
        cpu = {"value": ma["multires_mpixels_s"], "unit": "Mpixels/s", "cores": 1, "kind": "oracle",
               "sample": f"one multi-resolution SSAO frame at {W}x{H} (configuration 0: scene seed 1, camera 0), "
                         f"oracle.frame in one process on one thread, 1 warm-up + median of 3 runs "
                         f"({', '.join(f'{t:.2f}' for t in ma['multires_s'])} s)"}
        log(f"[bench] cpu oracle: {json.dumps(cpu_protocol)}")
        log(f"[bench] quality at 1080p against the oracle: {quality_1080p}")

    cfg = np.arange(args.steps) % nf
    per_cfg = [float(np.median(lat_p[cfg == c]) / np.median(lat_m[cfg == c])) for c in range(nf) if np.any(cfg == c)]

    def host_latency(h):
        return {"p50_ms": round(float(np.percentile(h[:, 1], 50)), 4),
                "p99_ms": round(float(np.percentile(h[:, 1], 99)), 4),
                "submit_p50_us": round(float(np.percentile(h[:, 0], 50)) * 1e3, 1)}

    res = {
        "metric": "Mpixels/s multi-res vs full-res SSAO at 4K (HBM %); p50/p99 frame latency",
        "value": round(value, 2),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_m * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ssao_4k: seeded scenes (200 boxes + 50 spheres) at {W}x{H}, 4 levels, "
                               f"SSAO {S} samples r={args.radius}, {nf} resident configurations",
                   "width": W, "height": H, "levels": 4, "samples": S, "radius": args.radius,
                   "configurations": nf, "parallelism": "single GPU"},
        "plain_mpixels_s": round(plain_mpx, 2),
        "speedup_vs_plain": round(value / plain_mpx, 3),
        "p50_ms": round(float(np.percentile(lat_m, 50)), 4),
        "p99_ms": round(float(np.percentile(lat_m, 99)), 4),
        "plain_p50_ms": round(float(np.percentile(lat_p, 50)), 4),
        "plain_p99_ms": round(float(np.percentile(lat_p, 99)), 4),
        "speedup_per_config_mean": round(float(np.mean(per_cfg)), 3),
        "host_latency": {"multires": host_latency(host_m), "plain": host_latency(host_p)},
        "mad_vs_plain": round(float(np.mean(mads)), 6) if mads else None,
        "rms_vs_plain": round(float(np.mean(rmss)), 6) if rmss else None,
        "concurrent": conc,
        "stages": stages,
        "roofline": roofline,
        "variants": variants,
        "batched_ssgi": batched,
        "batched_ssao": batched_ssao,
        "sweeps": sweeps,
        "pcss_4k": pcss,
        "serving": serving_res,
        "quality_1080p_vs_oracle": quality_1080p,
        "cpu_baseline": cpu,
        "cpu_protocol": cpu_protocol,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
