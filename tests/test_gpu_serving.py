"""The continuous-batching request loop: every request's frame is the same
bit for bit alone and in a mix of overlapping requests (other effects and
resolutions on other streams), the HBM budget limits what is in flight, and
the latency/throughput summary is well formed."""
import sys

import numpy as np
import pytest
import torch

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
