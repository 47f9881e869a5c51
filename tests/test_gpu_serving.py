"""The continuous-batching request loop: a served request of each effect is
the oracle's frame (both the request that builds the scene's resident mask
pyramid and one that reuses it), every request's frame is the same bit for
bit alone and in a mix of overlapping requests (other effects and
resolutions on other streams), the HBM budget limits what is in flight, and
the latency/throughput summary is well formed."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import serve

pytestmark = pytest.mark.gpu

_pool = {}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def pool():
    if not _pool:
        _pool["p"] = serve.Pool(scenes_per_res=1, resolutions=((384, 256), (640, 360)), shadow_map=512)
    return _pool["p"]


def oracle_frame(p, scene, effect):
    sc = p.scenes[scene]
    gb = sc.host["gb"]
    mp = p.mp[effect]
    omp = oracle.MaskParams(num_levels=mp.num_levels, level_enable=mp.level_enable, depth_ratio=mp.depth_ratio,
                            normal_cos=float(np.float32(mp.normal_cos)), sigma2=mp.sigma2, weight=mp.weight)
    if effect == "shadow":
        si = sc.host["shadow"]
        op = oracle.ShadowParams(si.shadow_map, si.view_to_light, si.light_focal, si.light_size, si.light_near,
                                 np.float32(0.05), scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12))
    elif effect == "ssao":
        op = oracle.SSAOParams(scenegen.ssao_kernel(32), 1.0, 0.02)
    else:
        op = oracle.SSGIParams(scenegen.ssao_kernel(64), 2.0, 0.02)
    return oracle.frame(effect, gb.depth, gb.normal, gb.focal, omp, op,
                        color=sc.host["color"] if effect == "ssgi" else None).out


@pytest.mark.parametrize("effect", serve.EFFECTS)
def test_served_requests_match_the_oracle(effect):
    p = pool()
    scene = p.res_index[(384, 256)][0]
    assert p.compact(scene, effect)
    p.pyramids.pop((scene, effect), None)
    reqs = [serve.Request(0, 0.0, effect, scene), serve.Request(1, 0.0, effect, scene)]
    log(f"[gpu] served {effect} scene {scene}: build, then reuse on another slot")
    done = serve.Server(p, slots=2, keep_outputs=True).run(reqs, realtime=False)
    assert p.pyramids[(scene, effect)].built
    ref = oracle_frame(p, scene, effect)
    for d in done:
        got = d.out.cpu().numpy()
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() <= 1e-4
        assert np.array_equal(got, ref), d.rid


def test_results_identical_alone_and_in_the_mix():
    p = pool()
    reqs = serve.poisson_requests(p, qps=20000.0, seconds=0.0015, seed=3)
    assert len(reqs) >= 12 and {r.effect for r in reqs} == set(serve.EFFECTS)
    log(f"[gpu] serving mix of {len(reqs)} requests")
    mix = serve.Server(p, slots=4, keep_outputs=True).run(reqs, realtime=False)
    assert [d.rid for d in mix] == [r.rid for r in reqs]
    for r, d in zip(reqs, mix):
        alone = serve.Server(p, slots=1, keep_outputs=True).run([r], realtime=False)[0]
        assert torch.equal(alone.out, d.out), (r.rid, r.effect)
        assert torch.isfinite(d.out).all()


def test_batched_requests_equal_requests_alone():
    """Same-effect requests served as batches (up to 4 per batch, set up
    without waiting) give the frames of the same requests served alone; a
    batched SSGI request also equals the oracle."""
    p = pool()
    reqs = [serve.Request(k, 0.0, ("ssao", "ssgi", "shadow")[k % 3], k % len(p.scenes)) for k in range(18)]
    log(f"[gpu] batched serving of {len(reqs)} requests")
    srv = serve.Server(p, slots=2, keep_outputs=True, batch_max=4)
    mix = srv.run(reqs, realtime=False)
    assert srv.batched >= 8
    for r, d in zip(reqs, mix):
        alone = serve.Server(p, slots=1, keep_outputs=True).run([r], realtime=False)[0]
        assert torch.equal(alone.out, d.out), (r.rid, r.effect)
    k = next(i for i, r in enumerate(reqs) if r.effect == "ssgi" and p.scenes[r.scene].W == 384)
    ref = oracle_frame(p, reqs[k].scene, "ssgi")
    assert np.array_equal(mix[k].out.cpu().numpy(), ref)
    # frames above batch_pixels run alone
    solo = serve.Server(p, slots=2, keep_outputs=True, batch_max=4, batch_pixels=1)
    done = solo.run(reqs, realtime=False)
    assert solo.batched == 0
    assert all(torch.equal(a.out, b.out) for a, b in zip(done, mix))


def test_budget_limits_requests_in_flight():
    p = pool()
    reqs = serve.poisson_requests(p, qps=20000.0, seconds=0.001, seed=4)
    srv = serve.Server(p, slots=4, budget_bytes=1, keep_outputs=True)  # every request exceeds it
    done = srv.run(reqs, realtime=False)
    # one request at a time: no two intervals overlap
    iv = sorted((d.start, d.end) for d in done)
    assert all(b[0] >= a[1] - 1e-9 for a, b in zip(iv, iv[1:]))
    ref = serve.Server(p, slots=4, keep_outputs=True).run(reqs, realtime=False)
    for a, b in zip(done, ref):
        assert torch.equal(a.out, b.out)


def test_poisson_stream_summary():
    p = pool()
    reqs = serve.poisson_requests(p, qps=5000.0, seconds=0.02, seed=5)
    s = serve.summary(serve.Server(p, slots=3).run(reqs))
    log(f"[gpu] serving summary {s}")
    assert s["requests"] == len(reqs) and 0 < s["p50_ms"] <= s["p99_ms"] and s["mpixels_s"] > 0
