"""GPU parity of batches over seeded random sets of uneven frames: for each
seed an effect (SSAO or SSGI), 2-4 levels with a random enabled set, the
samples, the sub-image storage (FP32 or FP16) and 1-9 frames of random
sizes, scenes and cameras are drawn; the batch runs with one launch per
stage and as one persistent launch (Sec. 3-4 for a set of frames), SSAO
batches also with LDS depth tiles of the dense coarsest level, and every
frame's image equals the oracle's frame bit for bit.

Batched frames take the compact path, so widths are multiples of 128 and
heights multiples of 2^(N-1) (ragged merge, edge and ranking tiles).  The
draws are fixed by their seeds."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import scenegen
from paper_1906_04576_amd import mr

DEV = "cuda"
COS25 = float(np.float32(math.cos(math.radians(25.0))))
SEEDS = range(16)
CONFIGS = (dict(persistent=0), dict(persistent=1), dict(persistent=1, tiles_per_ticket=1, eval_items=2))


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


VARIANCES = (0.0, 0.924, 1.848, 3.696)


def radius(s2):
    """Blur radius of a variance (Table 1: ceil(3 sigma); 0 without blur)."""
    return 0 if s2 <= 0 else math.ceil(3.0 * math.sqrt(float(np.float32(s2))))


def draw(seed):
    """One batch, a pure function of the seed."""
    rng = np.random.default_rng(7300 + seed)
    effect = str(rng.choice(["ssao", "ssgi"]))
    N = int(rng.integers(2, 5))
    en = 1 | (1 << (N - 1))
    for i in range(1, N - 1):
        en |= int(rng.integers(0, 2)) << i
    s = 1 << (N - 1)
    n = int(rng.integers(1, 10))
    n = 1 if seed == 0 else n  # one batch of a single frame
    frames = [dict(W=128 * int(rng.integers(1, 9)), H=s * int(rng.integers(1, 600 // s + 1)),
                   scene=(int(rng.integers(1, 1000)), int(rng.integers(5, 120)), int(rng.integers(0, 30))),
                   cam=int(rng.integers(0, 8))) for _ in range(n)]
    sigma2 = [float(rng.choice(VARIANCES)) for _ in range(N - 1)] + [0.0]
    # the compact path needs blur radii that make the nesting step a no-op:
    # r_c >= ceil(r_f / 2^(c - f)) for consecutive enabled levels f < c below
    # the coarsest; raise the coarser level's variance where it is not so
    below = [i for i in range(1, N) if (en >> (i - 1)) & 1]
    for f, c in zip(below, below[1:]):
        need = -(-radius(sigma2[f - 1]) // (1 << (c - f)))
        sigma2[c - 1] = min((v for v in VARIANCES if radius(v) >= need and v >= sigma2[c - 1]), key=radius)
    return dict(effect=effect, N=N, en=en, frames=frames, sigma2=tuple(sigma2),
                weight=tuple(float(rng.choice([1.0, 20.0, 100.0, 1000.0])) for _ in range(N - 1)) + (1.0,),
                S=int(rng.choice([1, 5, 16, 40])), radius=float(rng.choice([0.5, 1.0, 2.0])),
                f16=bool(rng.random() < 0.3))


def test_draws_cover_effects_levels_and_storage():
    b = [draw(k) for k in SEEDS]
    assert {x["effect"] for x in b} == {"ssao", "ssgi"}
    assert {x["N"] for x in b} == {2, 3, 4}
    assert any(x["f16"] for x in b) and not all(x["f16"] for x in b)
    assert min(len(x["frames"]) for x in b) == 1
    assert max(len(x["frames"]) for x in b) >= 7
    for x in b:
        lv = [i for i in range(1, x["N"]) if (x["en"] >> (i - 1)) & 1]
        assert all(radius(x["sigma2"][c - 1]) >= -(-radius(x["sigma2"][f - 1]) // (1 << (c - f)))
                   for f, c in zip(lv, lv[1:]))


@pytest.mark.gpu
@pytest.mark.parametrize("seed", list(SEEDS))
def test_random_batch(seed):
    b = draw(seed)
    log(f"[gpu] random batch {seed}: {b['effect']} N={b['N']} en={b['en']:b} S={b['S']} f16={b['f16']} "
        f"sizes={[(f['W'], f['H']) for f in b['frames']]}")
    mp = mr.MaskParams(num_levels=b["N"], level_enable=b["en"], sigma2=b["sigma2"], weight=b["weight"],
                       radius=(-1,) * b["N"], normal_cos=COS25)
    omp = oracle.MaskParams(num_levels=b["N"], level_enable=b["en"], sigma2=b["sigma2"], weight=b["weight"],
                            radius=(-1,) * b["N"], normal_cos=COS25)
    K = scenegen.ssao_kernel(b["S"], seed=900 + seed)
    op = (oracle.SSAOParams if b["effect"] == "ssao" else oracle.SSGIParams)(K, b["radius"], 0.02)
    frames, refs = [], []
    for f in b["frames"]:
        sc = scenegen.make_scene(*f["scene"])
        gb = scenegen.render_gbuffer(sc, scenegen.orbit_view(f["cam"]), f["W"], f["H"])
        col = scenegen.lambert_color(sc, gb) if b["effect"] == "ssgi" else None
        frames.append(dict(depth=torch.from_numpy(gb.depth).to(DEV), normal=torch.from_numpy(gb.normal).to(DEV),
                           focal=float(gb.focal), color=None if col is None else torch.from_numpy(col).to(DEV)))
        refs.append(oracle.frame(b["effect"], gb.depth, gb.normal, gb.focal, omp, op, color=col,
                                 level_dtype=np.float16 if b["f16"] else None).out)
    sp = mr.ssao_params(torch.from_numpy(K).to(DEV), b["radius"], 0.02)
    st = torch.cuda.current_stream()
    batch = mr.Batch(b["effect"], frames, mp, sp, level_dtype=torch.float16 if b["f16"] else torch.float32,
                     stream=st)
    extra = (dict(persistent=0, eval_halo=(8, 16, 24)[seed % 3]),) if b["effect"] == "ssao" else ()
    for cfg in CONFIGS + extra:
        batch.config = cfg
        for o in batch.outs:
            o.fill_(-1.0)
        outs = batch(st)
        batch.check(st)
        torch.cuda.synchronize()
        for k, (o, ref) in enumerate(zip(outs, refs)):
            g = o.cpu().numpy()
            assert g.shape == ref.shape
            assert np.array_equal(g, ref), f"{cfg} frame {k}: max |d| {np.abs(g - ref).max()}"
