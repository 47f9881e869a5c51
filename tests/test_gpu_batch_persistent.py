"""The persistent batch launch (mr_batch_config.persistent = 1): one launch
whose blocks take every stage's tiles from one ticket queue.  Its outputs are
bit-identical to the staged launches' for both effects and every input type,
on repeated runs (the kernel clears its counters for the next run) and in a
replayed HIP graph; a frame of a 64-sample SSGI batch (the batched workload's
sample count) matches the oracle; no wait runs out (mr_batch_check)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1906_04576_amd import mr
from test_gpu_batch import SIZES, alone, effect_params, frames_for, mask_params, scene

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


PERSISTENT = [dict(persistent=1), dict(persistent=1, eval_items=2), dict(persistent=1, worker_pixels=4096),
              dict(persistent=1, worker_pixels=1 << 20, eval_items=4), dict(persistent=1, merge_generic=1),
              dict(persistent=1, tiles_per_ticket=1), dict(persistent=1, tiles_per_ticket=7)]


@pytest.mark.parametrize("effect,level_dtype,f16n", [("ssao", torch.float32, False), ("ssgi", torch.float32, False),
                                                     ("ssao", torch.float16, True), ("ssgi", torch.float16, True)])
def test_persistent_equals_staged(effect, level_dtype, f16n):
    mp = mask_params(effect)
    _, _, p = effect_params(effect)
    fr = frames_for(effect, SIZES, f16n)
    b = mr.Batch(effect, fr, mp, p, level_dtype=level_dtype)
    log(f"[gpu] staged batch {effect} {level_dtype} f16 normals={f16n}")
    ref = [o.clone() for o in b()]
    torch.cuda.synchronize()
    for cfg in PERSISTENT:
        log(f"[gpu] persistent batch {effect} {cfg}")
        b.config = cfg
        for rep in range(2):  # the second run starts from the counters the first left
            for o in b.outs:
                o.fill_(float("nan"))
            b()
            b.check()
            for k, (o, r) in enumerate(zip(b.outs, ref)):
                assert torch.equal(o, r), (cfg, rep, SIZES[k])


def test_persistent_frame_matches_oracle_at_64_samples():
    effect = "ssgi"
    mp = mask_params(effect)
    K, r, p = effect_params(effect, S=64)
    fr = frames_for(effect, SIZES)
    b = mr.Batch(effect, fr, mp, p)
    b.config = dict(persistent=1)
    log("[gpu] persistent ssgi batch, 64 samples, vs oracle")
    outs = b()
    b.check()
    sc = scene(384, 200, 1)
    gb = sc["gb"]
    ref = oracle.frame(effect, gb.depth, gb.normal, gb.focal, mask_params(effect, oracle), oracle.SSGIParams(K, r, 0.02),
                       color=sc["col"].astype(np.float32), dtype=np.float32)
    got = outs[1].cpu().numpy()
    assert np.abs(got - ref.out).max() <= 1e-4
    assert np.array_equal(got, ref.out)
    assert torch.equal(outs[0], alone(effect, fr[0], mp, p))


def test_persistent_max_batch():
    effect = "ssao"
    mp = mask_params(effect)
    _, _, p = effect_params(effect, S=8)
    small = ((128, 64), (256, 64), (128, 128), (384, 40), (256, 136))
    base = frames_for(effect, small)
    fr = [dict(base[k % len(small)]) for k in range(mr.MR_MAX_BATCH)]
    b = mr.Batch(effect, fr, mp, p)
    b.config = dict(persistent=1)
    log(f"[gpu] persistent batch of {len(fr)} frames")
    outs = b()
    b.check()
    refs = [alone(effect, f, mp, p) for f in base]
    for k, o in enumerate(outs):
        assert torch.equal(o, refs[k % len(small)]), k


def test_persistent_graph_replays_to_eager():
    effect = "ssgi"
    mp = mask_params(effect)
    _, _, p = effect_params(effect)
    sizes = ((640, 360), (256, 128), (384, 200))
    depth = [scene(W, H, k)["depth"].clone() for k, (W, H) in enumerate(sizes)]
    fr = [dict(depth=d, normal=scene(W, H, k)["normal"], focal=float(scene(W, H, k)["gb"].focal),
               color=scene(W, H, k)["color"]) for k, ((W, H), d) in enumerate(zip(sizes, depth))]
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b = mr.Batch(effect, fr, mp, p, stream=st)
        b.config = dict(persistent=1)
        b(st)
    st.synchronize()
    log("[gpu] capturing a persistent batch run")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        b(st)
    for rep, v in enumerate((0, 3, 6, 1)):
        W, H = sizes[0]
        depth[0].copy_(scene(W, H, v)["depth"])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in b.outs]
        b()
        b.check()
        for k in range(len(sizes)):
            assert torch.equal(got[k], b.outs[k]), (rep, k)
        assert torch.equal(got[0], alone(effect, fr[0], mp, p)), rep


def test_persistent_needs_its_limits():
    mp = mask_params("ssao")
    _, _, p = effect_params("ssao", S=300)  # more samples than the persistent launch stages
    b = mr.Batch("ssao", frames_for("ssao", SIZES[:2]), mp, p)
    with pytest.raises(mr.MRError) as e:
        b.config = dict(persistent=1)
    assert e.value.status == mr.MR_E_PARAM
    assert b.config["persistent"] == 0
