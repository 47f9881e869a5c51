"""Host-side validation of batches (no GPU): mr_batch_workspace_bytes and
mr_batch_setup reject what a batch cannot take before anything is enqueued,
and name the offending frame."""
import ctypes

import pytest

from paper_1906_04576_amd import mr

FAKE = 0x10000  # aligned non-null stand-in addresses: validation never dereferences them
_KEEP = []  # effect parameter structs the descriptors point to


def desc(W=256, H=128, effect=mr.MR_EFFECT_SSAO, params=None, mp=None):
    d = mr.mr_frame_desc()
    d.effect = effect
    d.multires = 1
    d.g = mr.mr_gbuffer(FAKE, FAKE * 2, mr.MR_F32, FAKE * 3 if effect == mr.MR_EFFECT_SSGI else None, mr.MR_F32)
    d.cam = mr.mr_camera(W, H, 0.8 * W)
    d.mp = (mp or mr.MaskParams(num_levels=4)).c()
    if params is None:
        params = mr.mr_ssao_params(FAKE * 4, 16, 1.0, 0.02)
    if effect == mr.MR_EFFECT_SSAO:
        d.ssao = ctypes.pointer(params)
    elif effect == mr.MR_EFFECT_SSGI:
        d.ssgi = ctypes.pointer(params)
    d.out = FAKE * 5
    _KEEP.append(params)
    return d


def arr(*ds):
    a = (mr.mr_frame_desc * len(ds))()
    for k, d in enumerate(ds):
        a[k] = d
    return a


def ws_bytes(a, n=None):
    return mr.lib().mr_batch_workspace_bytes(a, len(a) if n is None else n)


def test_uneven_frames_are_accepted_and_laid_out():
    a = arr(desc(256, 128), desc(640, 360), desc(1280, 720), desc(128, 8))
    total = ws_bytes(a)
    assert total > 0
    # each frame adds its own region
    assert ws_bytes(arr(desc(256, 128), desc(640, 360), desc(1280, 720))) < total
    assert ws_bytes(arr(desc(256, 128))) < ws_bytes(arr(desc(256, 128), desc(128, 8)))
    assert total % 256 == 0


@pytest.mark.parametrize("mutate,code,text", [
    (lambda a: setattr(a[1], "effect", mr.MR_EFFECT_SSGI), mr.MR_E_PARAM, "effect differs"),
    (lambda a: setattr(a[2], "multires", 0), mr.MR_E_PARAM, "multi-resolution only"),
    (lambda a: setattr(a[1], "level_map", FAKE), mr.MR_E_PARAM, "level_map"),
    (lambda a: setattr(a[2], "out", None), mr.MR_E_NULL, "out is NULL"),
    (lambda a: setattr(a[1], "out", FAKE + 4), mr.MR_E_PARAM, "aligned"),
    (lambda a: setattr(a[1], "level_dtype", mr.MR_F16), mr.MR_E_DTYPE, "level_dtype"),
    (lambda a: setattr(a[2].g, "normal_dtype", mr.MR_F16), mr.MR_E_DTYPE, "input types"),
    (lambda a: setattr(a[1].cam, "width", 320), mr.MR_E_PARAM, "compact frame path"),
    (lambda a: setattr(a[1].mp, "depth_ratio", 0.2), mr.MR_E_PARAM, "mask parameters differ"),
    (lambda a: setattr(a[2].g, "depth", None), mr.MR_E_NULL, "frame 2"),
])
def test_batch_rejects(mutate, code, text):
    a = arr(desc(256, 128), desc(384, 200), desc(512, 96))
    mutate(a)
    L = mr.lib()
    assert ws_bytes(a) == 0
    assert text in mr.mr_last_error(), mr.mr_last_error()
    plan = (ctypes.c_uint8 * mr.MR_BATCH_PLAN_BYTES)()
    st = L.mr_batch_setup(a, len(a), FAKE, 1 << 30, ctypes.cast(plan, ctypes.c_void_p), mr.MR_BATCH_PLAN_BYTES,
                          None)
    assert st == code, (st, mr.mr_last_error())
    assert text in mr.mr_last_error()


def test_batch_rejects_different_effect_parameters():
    p2 = mr.mr_ssao_params(FAKE * 4, 16, 2.0, 0.02)
    a = arr(desc(256, 128), desc(256, 128, params=p2))
    assert ws_bytes(a) == 0 and "effect parameters differ" in mr.mr_last_error()


def test_batch_sizes_and_effects():
    assert ws_bytes(arr(desc()), 0) == 0 and "batch size" in mr.mr_last_error()
    big = arr(*[desc() for _ in range(mr.MR_MAX_BATCH)])
    assert ws_bytes(big) > 0
    assert ws_bytes(big, mr.MR_MAX_BATCH + 1) == 0 and "batch size" in mr.mr_last_error()
    sh = desc(effect=mr.MR_EFFECT_SHADOW)
    assert ws_bytes(arr(sh)) == 0 and "MR_EFFECT_SSAO or MR_EFFECT_SSGI" in mr.mr_last_error()
    assert mr.lib().mr_batch_workspace_bytes(None, 1) == 0 and "NULL" in mr.mr_last_error()
    gi = arr(desc(effect=mr.MR_EFFECT_SSGI, mp=mr.MaskParams(num_levels=4, level_enable=0b1101)),
             desc(384, 64, effect=mr.MR_EFFECT_SSGI, mp=mr.MaskParams(num_levels=4, level_enable=0b1101)))
    assert ws_bytes(gi) > 0


def test_setup_checks_workspace_and_plan_before_any_copy():
    a = arr(desc(256, 128), desc(384, 200))
    need = ws_bytes(a)
    L = mr.lib()
    plan = (ctypes.c_uint8 * mr.MR_BATCH_PLAN_BYTES)()
    pp = ctypes.cast(plan, ctypes.c_void_p)
    assert L.mr_batch_setup(a, 2, FAKE, need - 1, pp, mr.MR_BATCH_PLAN_BYTES, None) == mr.MR_E_WORKSPACE
    assert L.mr_batch_setup(a, 2, None, need, pp, mr.MR_BATCH_PLAN_BYTES, None) == mr.MR_E_WORKSPACE
    assert L.mr_batch_setup(a, 2, FAKE, need, None, mr.MR_BATCH_PLAN_BYTES, None) == mr.MR_E_NULL
    assert L.mr_batch_setup(a, 2, FAKE, need, pp, mr.MR_BATCH_PLAN_BYTES - 1, None) == mr.MR_E_PARAM
    # a plan that mr_batch_setup did not fill is refused without a launch
    assert L.mr_batch_run(pp, None) == mr.MR_E_PARAM and "mr_batch_setup" in mr.mr_last_error()
    assert L.mr_batch_run(None, None) == mr.MR_E_NULL


def test_config_calls_need_a_filled_plan():
    L = mr.lib()
    plan = (ctypes.c_uint8 * mr.MR_BATCH_PLAN_BYTES)()
    pp = ctypes.cast(plan, ctypes.c_void_p)
    c = mr.mr_batch_config()
    assert L.mr_batch_get_config(pp, ctypes.byref(c)) == mr.MR_E_PARAM
    assert L.mr_batch_set_config(pp, ctypes.byref(c)) == mr.MR_E_PARAM
    assert L.mr_batch_tune(pp, 3, ctypes.byref(c), None) == mr.MR_E_PARAM
    assert L.mr_batch_get_config(None, ctypes.byref(c)) == mr.MR_E_NULL
    assert L.mr_batch_get_config(pp, None) == mr.MR_E_NULL
    assert L.mr_batch_set_config(pp, None) == mr.MR_E_NULL
    assert L.mr_batch_tune(None, 3, None, None) == mr.MR_E_NULL


@pytest.mark.parametrize("mutate,text", [
    (lambda d: setattr(d, "effect", mr.MR_EFFECT_SSGI), "MR_EFFECT_SSAO only"),
    (lambda d: setattr(d.cam, "width", 320), "compact frame path"),
    (lambda d: setattr(d.bilateral, "levels", 0b10001), "not enabled"),
    (lambda d: setattr(d.bilateral, "radius", 3), "radius"),
    (lambda d: setattr(d.bilateral, "depth_rel", 0.0), "depth_rel"),
    (lambda d: setattr(d.bilateral, "depth_rel", float("nan")), "depth_rel"),
    (lambda d: setattr(d, "multires", 0), "multires"),
])
def test_frame_rejects_bilateral_misuse(mutate, text):
    """Validation of the bilateral blur happens before anything is enqueued
    (the stand-in addresses are never touched)."""
    d = desc(256, 128)
    d.bilateral = mr.Bilateral(levels=0b1110, radius=2).c()
    if "SSGI" in text or "MR_EFFECT_SSAO" in text:
        d.ssgi = d.ssao
        d.g.color = FAKE * 3
    mutate(d)
    st = mr.lib().mr_frame(ctypes.byref(d), FAKE, 1 << 40, None)
    assert st == mr.MR_E_PARAM, (st, mr.mr_last_error())
    assert text in mr.mr_last_error(), mr.mr_last_error()


def test_batch_rejects_bilateral():
    d = desc(256, 128)
    d.bilateral = mr.Bilateral().c()
    assert ws_bytes(arr(desc(), d)) == 0 and "bilateral" in mr.mr_last_error()


def test_fullres_levels_validation():
    """mr_eval_ssao_fullres checks its level sample sets before any launch."""
    L = mr.lib()
    g = mr.mr_gbuffer(FAKE, FAKE * 2, mr.MR_F32, None, mr.MR_F32)
    cam = mr.mr_camera(256, 128, 200.0)
    mp = mr.MaskParams(num_levels=4).c()
    m = mr.mr_masks()
    for i in range(3):
        m.alpha[i] = FAKE * (8 + i)
        m.stencil[i] = FAKE * (12 + i)
    ps = [mr.mr_ssao_params(FAKE * 4, 300, 1.0, 0.02) for _ in range(4)]
    lp = (ctypes.POINTER(mr.mr_ssao_params) * mr.MR_MAX_LEVELS)()
    for i in range(3):
        lp[i] = ctypes.pointer(ps[i])
    args = lambda: (ctypes.byref(g), ctypes.byref(cam), ctypes.byref(mp), ctypes.byref(m), ctypes.byref(lp),
                    FAKE * 16, None)
    assert L.mr_eval_ssao_fullres(*args()) == mr.MR_E_NULL and "level_params[3]" in mr.mr_last_error()
    lp[3] = ctypes.pointer(ps[3])
    assert L.mr_eval_ssao_fullres(*args()) == mr.MR_E_PARAM and "1024" in mr.mr_last_error()
    m.alpha[1] = None
    assert L.mr_eval_ssao_fullres(*args()) == mr.MR_E_NULL and "alpha[1]" in mr.mr_last_error()
