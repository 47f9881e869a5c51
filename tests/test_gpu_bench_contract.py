"""bench.py's JSON line on a short run: one line on stdout with the fields
and types the benchmark contract names, a roofline for the evaluation
kernel whose counter fields are present exactly when the kernel's code is
the one they were taken on, and the stage and latency figures."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_line():
    print("[gpu] bench.py --steps 8 on two configurations", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "8", "--warmup", "2", "--seeds", "1",
           "--cameras", "2", "--no-variants", "--no-batch", "--no-sweeps", "--no-pcss", "--no-serving",
           "--no-cpu-baseline"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    j = json.loads(lines[0])
    for k, t in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                 ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                 ("dtype", str), ("data", str), ("config", dict), ("roofline", dict)):
        assert isinstance(j[k], t), k
    assert j["n_gpus"] == 1 and j["steps"] == 8 and j["warmup"] == 2
    assert j["value"] > 0 and j["ms_per_step"] > 0 and j["higher_is_better"] is True
    assert j["vs_baseline"] is None and j["data"] == "synthetic"
    assert "workload" in j["config"] and j["config"]["width"] == 3840 and j["config"]["height"] == 2160
    ro = j["roofline"]
    assert ro["bound"] in ("hbm", "mfma", "alu") and ro["unit"] in ("GB/s", "TFLOP/s")
    assert 0 < ro["achieved"] <= ro["peak"] and abs(ro["frac"] - ro["achieved"] / ro["peak"]) < 1e-3
    fresh = bench.counters_current("k_ssao_multi")
    assert ro["counters_match_code"] is fresh
    if fresh:
        assert ro["traffic"] == bench.TRAFFIC_BYTES["k_ssao_multi"]
        assert 0 < ro["valu_rate_vs_plain"] < 1.2
    else:
        assert ro["traffic"] is None and ro["valu_rate_vs_plain"] is None
    st = j["stages"]
    for k in ("multi_masks_ms", "multi_eval_ms", "multi_merge_ms", "plain_eval_ms"):
        assert st[k] > 0, k
    assert 0 < j["p50_ms"] <= j["p99_ms"]
    for path in ("multires", "plain"):
        h = j["host_latency"][path]
        assert 0 < h["p50_ms"] <= h["p99_ms"] and h["submit_p50_us"] > 0
    assert j["speedup_vs_plain"] > 1 and j["speedup_per_config_mean"] > 1
    assert j["cpu_baseline"] is None and j["cpu_protocol"] is None  # --no-cpu-baseline
