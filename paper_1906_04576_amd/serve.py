"""Continuous-batching request loop for multi-resolution lighting frames.

Requests (a resident seeded scene at some resolution, one of the three
effects) arrive as a Poisson stream.  A request is admitted as soon as one of
the slots is free and its working memory (scratch and output) fits the HBM
budget next to the requests in flight and the resident data; each slot is a
HIP stream with its own scratch, so admitted requests overlap on the device
while others keep arriving.  The scenes' G-buffers stay resident, and so do
their mask pyramids: the first request for a (scene, effect) pair builds the
pyramid (mr_frame_cached with build = 1), later ones evaluate and merge on
it (build = 0, after the build's completion on the device).  Latency is
completion minus arrival, throughput the pixels finished per second of wall
time.  This module only schedules; every frame runs in the library.

    python -m paper_1906_04576_amd.serve --qps 4000 --seconds 2
prints one JSON line with p50/p99 latency and Mpixels/s, multi-resolution
and naive, on the same request stream, and the throughput with the same
requests admitted back to back (the loop's capacity).
"""
from __future__ import annotations

import argparse
import collections
import itertools
import json
import sys
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import mr

RESOLUTIONS = ((1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))
RES_WEIGHTS = (0.2, 0.4, 0.2, 0.2)
EFFECTS = ("ssao", "shadow", "ssgi")


@dataclass
class Scene:
    """Resident inputs of one seeded scene at one resolution (and their host
    copies, for checking results)."""
    W: int
    H: int
    focal: float
    depth: torch.Tensor
    normal: torch.Tensor
    color: torch.Tensor
    shadow: mr.mr_shadow_params
    bytes: int
    host: dict = None


@dataclass
class Pyramid:
    """Resident mask pyramid of one (scene, effect) pair."""
    mem: torch.Tensor
    built: bool = False
    ready: torch.cuda.Event = None  # completion of the request that built it


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the stream
    effect: str
    scene: int      # index into the resident scene pool


@dataclass
class Done:
    rid: int
    arrival: float
    start: float
    end: float
    pixels: int
    out: torch.Tensor | None = None


def _mask_params(effect: str) -> mr.MaskParams:
    import scenegen
    t = scenegen.TABLE1[effect]
    en = 0b1101 if effect == "ssgi" else 0b1111  # Table 1: SSGI leaves level 2 out
    return mr.MaskParams(num_levels=4, level_enable=en, sigma2=t["sigma2"], weight=t["weight"])


class Pool:
    """Resident scenes (G-buffer, colour, shadow map) and effect parameters."""

    def __init__(self, scenes_per_res: int = 2, device="cuda", resolutions=RESOLUTIONS, shadow_map=2048):
        import scenegen
        self.device = device
        self.scenes: list[Scene] = []
        self.res_index: dict[tuple, list[int]] = {}
        for (W, H) in resolutions:
            for k in range(scenes_per_res):
                seed = 100 + 10 * len(self.res_index) + k
                sc = scenegen.make_scene(seed, 200, 50)
                gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(k % 8), W, H)
                si = scenegen.render_shadow_inputs(sc, gb.view, shadow_map)
                col = scenegen.lambert_color(sc, gb)
                d = torch.from_numpy(gb.depth).to(device)
                n = torch.from_numpy(gb.normal).to(device)
                c = torch.from_numpy(col).to(device)
                sm = torch.from_numpy(si.shadow_map).to(device)
                bd = torch.from_numpy(scenegen.disk_samples(16, 11)).to(device)
                pd = torch.from_numpy(scenegen.disk_samples(32, 12)).to(device)
                sp = mr.shadow_params(sm, si.view_to_light, si.light_focal, si.light_size, si.light_near, 0.05,
                                      bd, pd)
                nbytes = sum(t.numel() * t.element_size() for t in (d, n, c, sm))
                self.res_index.setdefault((W, H), []).append(len(self.scenes))
                self.scenes.append(Scene(W, H, float(gb.focal), d, n, c, sp, nbytes,
                                         host={"gb": gb, "shadow": si, "color": col}))
        self.mp = {e: _mask_params(e) for e in EFFECTS}
        self.ssao = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(32)).to(device), 1.0, 0.02)
        self.ssgi = mr.ssao_params(torch.from_numpy(scenegen.ssao_kernel(64)).to(device), 2.0, 0.02)
        self.pyramids: dict[tuple, Pyramid] = {}
        self._compact: dict[tuple, bool] = {}

    def resident_bytes(self) -> int:
        return sum(sc.bytes for sc in self.scenes) + sum(p.mem.numel() for p in self.pyramids.values())

    def pyramid_bytes(self, scene: int, effect: str) -> int:
        sc = self.scenes[scene]
        return mr.mr_pyramid_bytes(sc.W, sc.H, sc.focal, self.mp[effect], mr.EFFECTS[effect])[0]

    def pyramid(self, scene: int, effect: str) -> Pyramid:
        key = (scene, effect)
        if key not in self.pyramids:
            self.pyramids[key] = Pyramid(torch.empty(self.pyramid_bytes(scene, effect), dtype=torch.uint8,
                                                     device=self.device))
        return self.pyramids[key]

    def scratch_bytes(self) -> int:
        """Per-frame memory when pyramids stay resident: the scratch of a
        compact frame, the whole workspace of any other; the largest over the
        resident resolutions and the effects."""
        return max(mr.mr_pyramid_bytes(sc.W, sc.H, sc.focal, self.mp[e], mr.EFFECTS[e])[1]
                   if self.compact(k, e) else mr.mr_workspace_bytes(sc.W, sc.H, sc.focal, self.mp[e], mr.EFFECTS[e])
                   for k, sc in enumerate(self.scenes) for e in EFFECTS)

    def params(self, effect: str, scene: Scene):
        return {"ssao": self.ssao, "shadow": scene.shadow, "ssgi": self.ssgi}[effect]

    def workspace_bytes(self) -> int:
        """Workspace of a frame that builds its own masks: the largest over
        the resident resolutions and the effects."""
        return max(mr.mr_workspace_bytes(sc.W, sc.H, sc.focal, self.mp[e], mr.EFFECTS[e])
                   for sc in self.scenes for e in EFFECTS)

    def compact(self, scene: int, effect: str) -> bool:
        """Whether the scene's frames take the compact path, the one whose
        mask pyramid can stay resident."""
        key = (scene, effect)
        if key not in self._compact:
            sc = self.scenes[scene]
            self._compact[key] = mr.mr_frame_workspace_layout(mr.camera(sc.W, sc.H, sc.focal), self.mp[effect].c(),
                                                              mr.EFFECTS[effect]).compact == 1
        return self._compact[key]


def poisson_requests(pool: Pool, qps: float, seconds: float, seed: int = 7) -> list[Request]:
    """Arrivals at rate qps (exponential gaps), resolution by RES_WEIGHTS
    (pool resolutions outside that mix: equal weights), effect uniform, scene
    uniform among that resolution's resident scenes."""
    rng = np.random.default_rng(seed)
    reqs, t, rid = [], 0.0, 0
    res = list(pool.res_index)
    # the serving mix's weights for its resolutions, equal weights otherwise
    w = np.array([RES_WEIGHTS[RESOLUTIONS.index(r)] if r in RESOLUTIONS else 1.0 for r in res], float)
    w /= w.sum()
    while True:
        t += rng.exponential(1.0 / qps)
        if t >= seconds:
            break
        r = res[rng.choice(len(res), p=w)]
        reqs.append(Request(rid, t, EFFECTS[rng.integers(3)], int(rng.choice(pool.res_index[r]))))
        rid += 1
    return reqs


class Server:
    """slots concurrent launches (one stream and workspace each) under an HBM
    budget for the working memory of the requests in flight.  batch_max >= 2:
    when a slot frees up, the oldest pending request takes with it up to
    batch_max - 1 other arrived requests of the same effect (SSAO or SSGI,
    compact path), and they run as one batch with one launch per stage for
    all of them.  With resident pyramids only requests whose pyramid is
    built are batched, and the batch evaluates and merges on those pyramids
    (mr_batch_setup_cached); without, the batch builds its masks
    (mr_batch_setup_async).  A request that finds no partner runs alone, and
    so does a frame of more than batch_pixels pixels: a frame that fills the
    GPU by itself runs faster alone (a batch streams every frame through each
    stage, so its evaluation no longer finds the frame's depth in the caches
    its edge kernel filled)."""

    def __init__(self, pool: Pool, slots: int = 4, budget_bytes: int = 64 << 30, multires: bool = True,
                 level_dtype=torch.float32, keep_outputs: bool = False, resident_masks: bool = True,
                 batch_max: int = 0, batch_pixels: int = 2560 * 1440):
        self.pool, self.multires, self.level_dtype, self.keep = pool, multires, level_dtype, keep_outputs
        self.cached = multires and resident_masks
        self.budget = budget_bytes
        ws = (pool.scratch_bytes() if self.cached else pool.workspace_bytes()) if multires else 256
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.ws = [torch.empty(ws, dtype=torch.uint8, device=pool.device) for _ in range(slots)]
        self.ws_bytes = ws
        self.batch_max = batch_max if multires else 0
        self.batch_pixels = batch_pixels
        self.batched = 0  # requests served in batches of two or more
        self.slots_b = []
        self.batch_ws_bytes = 0
        if self.batch_max >= 2:
            nws, nst = 0, 0
            for e in ("ssao", "ssgi"):
                ks = [k for k in range(len(pool.scenes))
                      if pool.compact(k, e) and pool.scenes[k].W * pool.scenes[k].H <= batch_pixels]
                if not ks:
                    continue
                big = max(ks, key=lambda k: pool.scenes[k].W * pool.scenes[k].H)
                w, t = mr.BatchSlot.sizes(e, [self._frame(big, e)] * self.batch_max, pool.mp[e],
                                          pool.params(e, pool.scenes[big]), level_dtype, cached=self.cached)
                nws, nst = max(nws, w), max(nst, t)
            self.slots_b = [mr.BatchSlot(nws, nst, pool.device) for _ in range(slots)]
            self.batch_ws_bytes = nws

    def _frame(self, scene: int, effect: str, out=None) -> dict:
        sc = self.pool.scenes[scene]
        return dict(depth=sc.depth, normal=sc.normal, focal=sc.focal, color=sc.color if effect == "ssgi" else None,
                    out=out)

    def _batchable(self, req: Request) -> bool:
        if self.batch_max < 2 or req.effect not in ("ssao", "ssgi") or not self.pool.compact(req.scene, req.effect):
            return False
        sc = self.pool.scenes[req.scene]
        if sc.W * sc.H > self.batch_pixels:
            return False
        if self.cached:  # its pyramid must be built (the first request builds it alone)
            pyr = self.pool.pyramids.get((req.scene, req.effect))
            return pyr is not None and pyr.built
        return True

    def _out(self, req: Request, st):
        sc = self.pool.scenes[req.scene]
        C = 3 if req.effect == "ssgi" else 1
        with torch.cuda.stream(st):
            return torch.empty((C, sc.H, sc.W) if C > 1 else (sc.H, sc.W), dtype=torch.float32,
                               device=self.pool.device)

    def _launch(self, req: Request, slot: int):
        sc = self.pool.scenes[req.scene]
        st = self.streams[slot]
        out = self._out(req, st)
        color = sc.color if req.effect == "ssgi" else None
        params = self.pool.params(req.effect, sc)
        cached = self.cached and self.pool.compact(req.scene, req.effect)
        if cached:
            pyr = self.pool.pyramid(req.scene, req.effect)
            build = not pyr.built
            if not build and pyr.ready is not None:
                st.wait_event(pyr.ready)  # the build may still run on another slot
            fr = mr.CachedFrameRunner(req.effect, sc.depth, sc.normal, sc.focal, self.pool.mp[req.effect], pyr.mem,
                                      color=color, params=params, out=out, workspace=self.ws[slot],
                                      level_dtype=self.level_dtype)
            fr(st, build=build)
        else:
            fr = mr.FrameRunner(req.effect, sc.depth, sc.normal, sc.focal, self.pool.mp[req.effect], self.multires,
                                color=color, params=params, out=out, workspace=self.ws[slot],
                                level_dtype=self.level_dtype)
            fr(st)
        ev = torch.cuda.Event()
        ev.record(st)
        if cached and build:
            pyr.built, pyr.ready = True, ev
        return [out], ev, out.numel() * 4 + self.ws_bytes

    def _launch_batch(self, reqs: list[Request], slot: int):
        st = self.streams[slot]
        e = reqs[0].effect
        outs = [self._out(r, st) for r in reqs]
        frames = [self._frame(r.scene, e, o) for r, o in zip(reqs, outs)]
        pyrs = None
        if self.cached:
            pyrs = []
            for r in reqs:
                pyr = self.pool.pyramids[(r.scene, e)]
                if pyr.ready is not None:
                    st.wait_event(pyr.ready)  # built on another slot
                pyrs.append(pyr.mem)
        self.slots_b[slot].run(e, frames, self.pool.mp[e], self.pool.params(e, self.pool.scenes[reqs[0].scene]),
                               stream=st, level_dtype=self.level_dtype, pyramids=pyrs)
        ev = torch.cuda.Event()
        ev.record(st)
        self.batched += len(reqs)
        return outs, ev, sum(o.numel() * 4 for o in outs) + self.batch_ws_bytes

    def _group(self, pending: list[Request], now: float, realtime: bool) -> list[Request]:
        """The oldest pending request and, if it can be batched, up to
        batch_max - 1 more arrived requests of its effect."""
        first = pending[0]
        group = [first]
        if not self._batchable(first):
            return group
        for r in itertools.islice(pending, 1, None):
            if len(group) == self.batch_max or (realtime and r.arrival > now):
                break
            if r.effect == first.effect and self._batchable(r):
                group.append(r)
        return group

    def run(self, reqs: list[Request], realtime: bool = True) -> list[Done]:
        """Serve the request stream; realtime=False admits every request as
        soon as a slot is free (arrival times ignored).  Completions are
        found by polling the slots' events: the loop must also admit
        requests the moment they arrive, and a blocking wait would add the
        runtime's wake-up time to requests that take about 0.1 ms."""
        pending = collections.deque(reqs)
        free = list(range(len(self.streams)))
        inflight = {}  # slot -> (reqs, outs, event, bytes, start)
        used = 0
        done: list[Done] = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while pending or inflight:
            now = time.perf_counter() - t0
            for slot in list(inflight):
                group, outs, ev, nb, start = inflight[slot]
                if ev.query():
                    end = time.perf_counter() - t0
                    for req, out in zip(group, outs):
                        sc = self.pool.scenes[req.scene]
                        done.append(Done(req.rid, req.arrival if realtime else start, start, end, sc.W * sc.H,
                                         out if self.keep else None))
                    used -= nb
                    del inflight[slot]
                    free.append(slot)
            while pending and free and (not realtime or pending[0].arrival <= now):
                group = self._group(pending, now, realtime)
                need = 0
                for req in group:
                    sc = self.pool.scenes[req.scene]
                    need += (3 if req.effect == "ssgi" else 1) * sc.W * sc.H * 4
                if len(group) > 1:
                    need += self.batch_ws_bytes
                else:
                    req = group[0]
                    need += self.ws_bytes
                    if self.cached and (req.scene, req.effect) not in self.pool.pyramids and \
                            self.pool.compact(req.scene, req.effect):
                        need += self.pool.pyramid_bytes(req.scene, req.effect)  # becomes resident
                if used + need + self.pool.resident_bytes() > self.budget and inflight:
                    break  # admitted when memory frees up
                pending.popleft()
                for r in group[1:]:
                    pending.remove(r)  # near the front: within the arrived requests
                slot = free.pop(0)
                if len(group) > 1:
                    outs, ev, nb = self._launch_batch(group, slot)
                else:
                    outs, ev, nb = self._launch(group[0], slot)
                used += nb
                inflight[slot] = (group, outs, ev, nb, time.perf_counter() - t0)
        torch.cuda.synchronize()
        return sorted(done, key=lambda d: d.rid)


def summary(done: list[Done]) -> dict:
    lat = np.array([d.end - d.arrival for d in done]) * 1e3
    span = max(d.end for d in done) - min(d.arrival for d in done)
    px = sum(d.pixels for d in done)
    return {"requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4), "mpixels_s": round(px / span / 1e6, 2)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--qps", type=float, default=4000.0)
    ap.add_argument("--seconds", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--scenes-per-res", type=int, default=2)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    args = ap.parse_args(argv)
    t = time.time()
    pool = Pool(args.scenes_per_res)
    print(f"[serve] {len(pool.scenes)} resident scenes in {time.time() - t:.1f}s", file=sys.stderr, flush=True)
    reqs = poisson_requests(pool, args.qps, args.seconds)
    res = {"qps": args.qps, "seconds": args.seconds, "slots": args.slots, "budget_gb": args.budget_gb}
    for name, multires, resident, bmax in (("multires", True, True, 0), ("multires_rebuild", True, False, 0),
                                           ("multires_batched", True, True, 4), ("plain", False, False, 0)):
        srv = Server(pool, args.slots, int(args.budget_gb * (1 << 30)), multires, resident_masks=resident,
                     batch_max=bmax)
        srv.run(reqs[: min(len(reqs), 64)])  # warm-up (builds the resident pyramids)
        s = summary(srv.run(reqs))
        # the same requests admitted back to back: the loop's capacity
        sat = summary(srv.run(reqs, realtime=False))
        s["saturated_mpixels_s"] = sat["mpixels_s"]
        res[name] = s
        print(f"[serve] {name}: {s}", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
