"""The oracle's SSAO frame timed on the host's cores: in one process (mode A)
and split into row bands over one process per core (mode B).

TEST INFRASTRUCTURE ONLY (see the package docstring).  The CPU-baseline leg
of the benchmark runs this module as a child process (``python -m
oracle.timing``) that never touches a GPU, and the test suite checks that
the banded frame equals ``oracle.frame`` bit for bit.

Row bands.  Every output pixel of the multi-resolution frame depends only on
the G-buffer rows near it, except for the estimator's depth gathers, which
may reach anywhere in the level image:

* the edge image (Sec. 3.1) reads one row above and below;
* OR-pooling to level i covers the 2^(i-1) rows of a texel, and the level's
  blur (Table 1 variance) reaches r_i texels, i.e. r_i 2^(i-1) rows;
* the nesting of stencils (Sec. 4.1) ORs a finer level's texels into the
  coarser texel that holds them, which adds no reach beyond one coarse texel;
* the merge (Eq. 1, bilinear taps) reads one texel of every level around a
  pixel, at most 2^(L-1) rows for the coarsest level L.

A band of rows [y0, y1), with y0 a multiple of 2^(L-1), is therefore computed
from the edge image and pyramid of the rows [y0 - m - c, y1 + m + c), where m
is one coarsest texel and c the mask reach, and from the estimator at every
texel of the rows [y0 - m, y1 + m) with full level images for its gathers.
The band's own boundary rows are then outside everything its output reads,
and every value is the one ``oracle.frame`` computes (the arithmetic of each
texel and pixel is unchanged; only which texels are computed differs).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing
import os
import sys
import time

import numpy as np

from .masks import MaskParams, edge_image, build_pyramid, level_sample, level_dims, blur_radius
from .ssao import SSAOParams, ssao_texels
from .merge import upsample_merge
from .frame import frame


def band_context(mp: MaskParams):
    """(m, c): rows of one coarsest texel, and the rows of mask context
    beyond them, both multiples of 2^(L-1)."""
    levels = mp.enabled()
    L = levels[-1]
    sl = 1 << (L - 1)
    reach = 2  # the edge image's own rows
    for i in levels[:-1]:
        reach = max(reach, (blur_radius(mp.sigma2[i - 1], mp.radius[i - 1]) + 2) << (i - 1))
    return sl, -(-reach // sl) * sl


def frame_rows(depth, normal, focal, mp: MaskParams, op: SSAOParams, multires, y0, y1, dtype=np.float32):
    """Rows [y0, y1) of oracle.frame("ssao", ...).out, computed from the
    rows they depend on (y0 a multiple of 2^(L-1) for the multi-resolution
    frame).  The naive frame is the estimator at every pixel of the rows."""
    H, W = depth.shape
    if not multires:
        ys, xs = np.divmod(np.arange(y0 * W, y1 * W), W)
        return ssao_texels(depth, normal, focal, 1, xs, ys, op, dtype).astype(dtype).reshape(y1 - y0, W)
    if mp.fovea is not None:
        raise ValueError("frame_rows: foveated masks are not split into bands")
    levels = mp.enabled()
    L = levels[-1]
    m, c = band_context(mp)
    if y0 % m:
        raise ValueError(f"frame_rows: y0 = {y0} is not a multiple of {m}")
    ya, yb = max(0, y0 - m - c), min(H, y1 + m + c)     # mask rows
    ma, mb = max(0, y0 - m), min(H, y1 + m)              # merge window
    E = edge_image(depth[ya:yb], normal[:, ya:yb], mp.depth_ratio, mp.normal_cos, dtype)
    pyr = build_pyramid(E, mp, dtype)
    alpha, stencil, lo = {}, {}, {}
    for i in levels:
        s = 1 << (i - 1)
        Wi, Hi = level_dims(W, mb - ma, i)
        ra = (ma - ya) // s                               # window's first texel row in the band
        if i == L:
            st = np.ones((Hi, Wi), np.uint8)
        else:
            st = pyr.stencil[i][ra:ra + Hi]
            alpha[i] = pyr.alpha[i][ra:ra + Hi]
        stencil[i] = st
        ys, xs = np.nonzero(st)
        v = np.zeros((Hi, Wi), dtype)
        if len(xs):
            zi, ni = level_sample(depth, i), level_sample(normal, i)
            v[ys, xs] = ssao_texels(zi, ni, focal, i, xs, ys + ma // s, op, dtype)
        lo[i] = v
    out = upsample_merge(W, mb - ma, levels, {i: mp.weight[i - 1] for i in levels}, alpha, stencil, lo, 1, dtype)
    return out[y0 - ma:y1 - ma]


def bands(H, n, align):
    """n row bands of nearly equal height, every start a multiple of align."""
    units = -(-H // align)
    cuts = [min(H, (k * units // n) * align) for k in range(n + 1)]
    return [(a, b) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]


_INPUT = None  # (depth, normal, focal, mp, op), inherited by the forked workers


def _band_task(task):
    multires, y0, y1 = task
    depth, normal, focal, mp, op = _INPUT
    return frame_rows(depth, normal, focal, mp, op, multires, y0, y1)


def frame_bands(pool, nbands, multires):
    """The frame over row bands, one task per band on `pool` (forked after
    _INPUT was set)."""
    depth = _INPUT[0]
    H = depth.shape[0]
    align = band_context(_INPUT[3])[0] if multires else 1
    parts = pool.map(_band_task, [(multires, a, b) for a, b in bands(H, nbands, align)])
    return np.concatenate(parts, axis=0)


def _median_runs(fn, warmup, runs):
    for _ in range(warmup):
        out = fn()
    ts = []
    for _ in range(runs):
        t = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t)
    return out, ts


def main(argv=None):
    ap = argparse.ArgumentParser(description="time the oracle's SSAO frame on the host's cores")
    ap.add_argument("--resolutions", default="1920x1080,3840x2160")
    ap.add_argument("--samples", type=int, default=32)
    ap.add_argument("--radius", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--camera", type=int, default=0)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--runs", type=int, default=3)
    ap.add_argument("--processes", type=int, default=0, help="mode B processes (0: the cores this process may use)")
    ap.add_argument("--save", default="", help="directory for the mode A images of the resolutions in --save-res")
    ap.add_argument("--save-res", default="1920x1080")
    args = ap.parse_args(argv)

    import scenegen
    from threadpoolctl import threadpool_limits

    global _INPUT
    visible = len(os.sched_getaffinity(0))
    nproc = args.processes or visible
    t1 = scenegen.TABLE1["ssao"]
    mp = MaskParams(num_levels=4, level_enable=0xF, sigma2=t1["sigma2"], weight=t1["weight"])
    op = SSAOParams(scenegen.ssao_kernel(args.samples), args.radius, 0.02)
    scene = scenegen.make_scene(args.seed, 200, 50)
    save_res = set(args.save_res.split(",")) if args.save else set()
    res = {"cores_visible": visible, "processes": nproc, "warmup": args.warmup, "runs": args.runs,
           "inputs": f"scene seed {args.seed} (200 boxes + 50 spheres), camera {args.camera}, "
                     f"SSAO {args.samples} samples r={args.radius}, 4 levels",
           "resolutions": {}}
    ctx = multiprocessing.get_context("fork")
    for wh in args.resolutions.split(","):
        W, H = (int(v) for v in wh.split("x"))
        gb = scenegen.render_gbuffer(scene, scenegen.orbit_view(args.camera), W, H)
        r = {"mode_a": {}, "mode_b": {}, "bit_identical": True}
        outs = {}
        with threadpool_limits(limits=1):
            for multires in (True, False):
                key = "multires" if multires else "plain"
                out, ts = _median_runs(lambda: frame("ssao", gb.depth, gb.normal, gb.focal, mp, op, multires).out,
                                       args.warmup, args.runs)
                outs[key] = out
                r["mode_a"][key + "_s"] = [round(t, 4) for t in ts]
                print(f"[oracle.timing] {wh} one process, {key}: {r['mode_a'][key + '_s']} s", file=sys.stderr, flush=True)
            _INPUT = (gb.depth, gb.normal, gb.focal, mp, op)
            with ctx.Pool(nproc) as pool:
                for multires in (True, False):
                    key = "multires" if multires else "plain"
                    out, ts = _median_runs(lambda: frame_bands(pool, nproc, multires), args.warmup, args.runs)
                    r["mode_b"][key + "_s"] = [round(t, 4) for t in ts]
                    print(f"[oracle.timing] {wh} {nproc} processes, {key}: {r['mode_b'][key + '_s']} s",
                          file=sys.stderr, flush=True)
                    r["bit_identical"] &= bool(np.array_equal(out, outs[key], equal_nan=True))
            _INPUT = None
        for mode in ("mode_a", "mode_b"):
            for key in ("multires", "plain"):
                r[mode][key + "_mpixels_s"] = round(W * H / float(np.median(r[mode][key + "_s"])) / 1e6, 4)
        if wh in save_res:
            for key, out in outs.items():
                np.save(os.path.join(args.save, f"oracle_{wh}_{key}.npy"), out)
        res["resolutions"][wh] = r
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
