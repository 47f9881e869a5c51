"""The C ABI without a GPU: libmr.so loads, exports every function that
include/mr.h declares, and rejects invalid arguments on the host before
anything is enqueued (these calls never reach the HIP runtime)."""
import ctypes
import math
import os
import re
import shutil
import subprocess

import pytest

from paper_1906_04576_amd import mr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mr.h")).read()
    return re.findall(r"MR_API\s+[\w\s\*]+?\b(mr_\w+)\s*\(", src)


def test_header_declares_the_boundary():
    names = set(declared_functions())
    assert {"mr_build_masks", "mr_eval_ssao", "mr_eval_shadow", "mr_eval_ssgi", "mr_upsample_merge",
            "mr_frame", "mr_workspace_bytes", "mr_shadow_hard", "mr_status_string", "mr_last_error",
            "mr_version"} <= names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mr.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in mr.SIGNATURES, name


def test_struct_sizes_match_header_layout():
    # mirrors of include/mr.h (x86-64 SysV alignment)
    assert ctypes.sizeof(mr.mr_camera) == 12
    assert ctypes.sizeof(mr.mr_mask_params) == 4 + 4 + 4 + 4 + 24 + 24 + 24 + 20
    assert ctypes.sizeof(mr.mr_masks) == 8 * (2 + 4 * 6 + 1)
    assert ctypes.sizeof(mr.mr_gbuffer) == 40


STRUCTS = ["mr_gbuffer", "mr_camera", "mr_fovea", "mr_mask_params", "mr_masks", "mr_ssao_params", "mr_shadow_params",
           "mr_ssgi_params", "mr_frame_desc", "mr_batch_config", "mr_bilateral_params", "mr_frame_layout"]


@pytest.mark.skipif(not shutil.which("gcc"), reason="needs a C compiler")
def test_struct_layout_matches_the_c_compiler(tmp_path):
    # sizeof / offsetof of every header struct as the C compiler lays them
    # out, against the ctypes mirrors the binding passes across the boundary
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mr.h"', 'int main(void) {']
    for st in STRUCTS:
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for name, _ in getattr(mr, st)._fields_:
            lines.append(f'printf("{st} {name} %zu\\n", offsetof({st}, {name}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        st, name, v = line.split()
        got[(st, name)] = int(v)
    for st in STRUCTS:
        cls = getattr(mr, st)
        assert got[(st, "size")] == ctypes.sizeof(cls), st
        for name, _ in cls._fields_:
            assert got[(st, name)] == getattr(cls, name).offset, (st, name)


def test_version_and_status_strings():
    assert mr.mr_version() == mr.MR_VERSION == 101
    assert mr.mr_status_string(0) == "MR_OK"
    for s in range(-6, 0):
        assert mr.mr_status_string(s).startswith("MR_E_")


def test_binding_refuses_a_library_of_another_version(monkeypatch):
    """A libmr.so built from another header version (other struct layouts)
    is refused when it is loaded, not misread later."""
    mr.lib()
    monkeypatch.setattr(mr, "_lib", None)
    monkeypatch.setattr(mr, "MR_VERSION", mr.MR_VERSION + 1)
    with pytest.raises(RuntimeError, match="version"):
        mr.lib()


def test_workspace_bytes_validation():
    mp = mr.MaskParams()
    assert mr.mr_workspace_bytes(3840, 2160, 1870.6, mp, mr.MR_EFFECT_SSAO) > 3840 * 2160 * 10
    assert mr.mr_workspace_bytes(3840, 2160, 1870.6, mp, mr.MR_WS_MASKS) > 0
    bad = [
        dict(W=3841, H=2160, mp=mp, code="divisible"),
        dict(W=0, H=2160, mp=mp, code="outside"),
        dict(W=64, H=64, mp=mr.MaskParams(num_levels=7, level_enable=0x7F), code="num_levels"),
        dict(W=64, H=64, mp=mr.MaskParams(level_enable=0b0111), code="level_enable"),
        dict(W=64, H=64, mp=mr.MaskParams(level_enable=0b11110), code="level_enable"),
        dict(W=64, H=64, mp=mr.MaskParams(sigma2=(-1.0, 1.848, 3.696, 0.0)), code="sigma2"),
        dict(W=64, H=64, mp=mr.MaskParams(sigma2=(40.0, 1.848, 3.696, 0.0)), code="radius"),
        dict(W=64, H=64, mp=mr.MaskParams(weight=(0.0, 50.0, 20.0, 1.0)), code="weight"),
        dict(W=64, H=64, mp=mr.MaskParams(normal_cos=1.5), code="normal_cos"),
        dict(W=64, H=64, mp=mr.MaskParams(depth_ratio=float("nan")), code="depth_ratio"),
    ]
    for b in bad:
        with pytest.raises(mr.MRError) as e:
            mr.mr_workspace_bytes(b["W"], b["H"], 100.0, b["mp"], mr.MR_EFFECT_SSAO)
        assert b["code"] in str(e.value), (b, str(e.value))


def test_entry_points_reject_null_and_bad_shapes_without_enqueueing():
    L = mr.lib()
    cam = mr.mr_camera(64, 64, 50.0)
    mp = mr.MaskParams().c()
    m = mr.mr_masks()
    assert L.mr_build_masks(None, ctypes.byref(cam), ctypes.byref(mp), None, ctypes.byref(m), None, 0,
                            None) == mr.MR_E_NULL
    assert "gbuffer" in mr.mr_last_error()
    g = mr.mr_gbuffer(ctypes.c_void_p(4096), ctypes.c_void_p(8192), mr.MR_F32, None, mr.MR_F32)
    # masks without stencil pointers
    assert L.mr_build_masks(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(mp), None, ctypes.byref(m), None,
                            0, None) == mr.MR_E_NULL
    # misaligned depth
    g2 = mr.mr_gbuffer(ctypes.c_void_p(4100), ctypes.c_void_p(8192), mr.MR_F32, None, mr.MR_F32)
    out = mr.c_ptr6()
    p = mr.mr_ssao_params(ctypes.c_void_p(4096), 16, 0.5, 0.02)
    assert L.mr_eval_ssao(ctypes.byref(g2), ctypes.byref(cam), None, None, ctypes.byref(p), ctypes.byref(out),
                          None) == mr.MR_E_PARAM
    # bad normal dtype
    g3 = mr.mr_gbuffer(ctypes.c_void_p(4096), ctypes.c_void_p(8192), 7, None, mr.MR_F32)
    out[0] = 4096
    assert L.mr_eval_ssao(ctypes.byref(g3), ctypes.byref(cam), None, None, ctypes.byref(p), ctypes.byref(out),
                          None) == mr.MR_E_DTYPE
    # sample count out of range, radius not positive
    for S, r, b in [(0, 0.5, 0.02), (8193, 0.5, 0.02), (16, 0.0, 0.02), (16, 0.5, -1.0), (16, math.inf, 0.0)]:
        p = mr.mr_ssao_params(ctypes.c_void_p(4096), S, r, b)
        assert L.mr_eval_ssao(ctypes.byref(g), ctypes.byref(cam), None, None, ctypes.byref(p),
                              ctypes.byref(out), None) == mr.MR_E_PARAM
    # frame: workspace too small
    d = mr.mr_frame_desc()
    d.effect = mr.MR_EFFECT_SSAO
    d.multires = 1
    d.g = g
    d.cam = cam
    d.mp = mp
    sp = mr.mr_ssao_params(ctypes.c_void_p(4096), 16, 0.5, 0.02)
    d.ssao = ctypes.pointer(sp)
    d.out = ctypes.c_void_p(4096)
    assert L.mr_frame(ctypes.byref(d), ctypes.c_void_p(4096), 100, None) == mr.MR_E_WORKSPACE
    d.effect = 9
    assert L.mr_frame(ctypes.byref(d), ctypes.c_void_p(4096), 100, None) == mr.MR_E_PARAM
    # eval_halo: not one of 0, 8, 16, 24; too many samples; off the compact path
    d.effect = mr.MR_EFFECT_SSAO
    for h in (4, 32, -8):
        d.eval_halo = h
        assert L.mr_frame(ctypes.byref(d), ctypes.c_void_p(4096), 1 << 30, None) == mr.MR_E_PARAM
        assert "eval_halo" in mr.mr_last_error()
    d.eval_halo = 16
    sp300 = mr.mr_ssao_params(ctypes.c_void_p(4096), 300, 0.5, 0.02)
    d.ssao = ctypes.pointer(sp300)
    assert L.mr_frame(ctypes.byref(d), ctypes.c_void_p(4096), 1 << 30, None) == mr.MR_E_PARAM
    d.ssao = ctypes.pointer(sp)
    assert L.mr_frame(ctypes.byref(d), ctypes.c_void_p(4096), 1 << 30, None) == mr.MR_E_PARAM  # width 64
    assert "compact" in mr.mr_last_error()
    d.eval_halo = 0
    # the frame tuner validates the frame before it creates its events
    assert L.mr_frame_tune(None, ctypes.c_void_p(4096), 1 << 30, 3, None, None) == mr.MR_E_NULL
    for reps in (0, 1001):
        assert L.mr_frame_tune(ctypes.byref(d), ctypes.c_void_p(4096), 1 << 30, reps, None, None) == mr.MR_E_PARAM
    assert L.mr_frame_tune(ctypes.byref(d), ctypes.c_void_p(4096), 100, 3, None, None) == mr.MR_E_WORKSPACE
    d.eval_halo = 4
    assert L.mr_frame_tune(ctypes.byref(d), ctypes.c_void_p(4096), 1 << 30, 3, None, None) == mr.MR_E_PARAM
    assert d.eval_halo == 4  # unchanged on an error
    d.eval_halo = 0
    # merge: bad channel count
    mm = mr.mr_masks()
    arr = mr.c_ptr6()
    mp1 = mr.MaskParams(num_levels=1, level_enable=1).c()
    assert L.mr_upsample_merge(ctypes.byref(cam), ctypes.byref(mp1), ctypes.byref(mm), ctypes.byref(arr), 2,
                               ctypes.c_void_p(4096), None) == mr.MR_E_PARAM


def test_shadow_params_validation():
    L = mr.lib()
    cam = mr.mr_camera(64, 64, 50.0)
    g = mr.mr_gbuffer(ctypes.c_void_p(4096), None, mr.MR_F32, None, mr.MR_F32)
    sp = mr.mr_shadow_params()
    sp.shadow_map = 4096
    sp.sm_size = 0
    sp.light_focal_px = 100.0
    sp.light_near = 1.0
    sp.blocker_disk = 4096
    sp.pcf_disk = 4096
    sp.n_blocker = 16
    sp.n_pcf = 32
    assert L.mr_shadow_hard(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(sp), ctypes.c_void_p(4096),
                            None) == mr.MR_E_SHAPE
    sp.sm_size = 64
    sp.light_near = 0.0
    assert L.mr_shadow_hard(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(sp), ctypes.c_void_p(4096),
                            None) == mr.MR_E_PARAM


def test_frame_workspace_layout_on_the_host():
    """The compact path's mask layout (host call, no GPU): list, stencil-bit
    and rank regions of every list level lie inside the workspace without
    overlap, after the counter words; other parameters report compact = 0."""
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=(0.924, 1.848, 3.696, 0.0),
                       weight=(100.0, 50.0, 20.0, 1.0))
    for W, H in ((3840, 2160), (1920, 1080), (256, 256)):
        cam = mr.camera(W, H, 100.0)
        lay = mr.mr_frame_workspace_layout(cam, mp.c(), mr.MR_EFFECT_SSAO)
        assert lay.compact == 1 and (lay.tile_words, lay.tile_rows) == (16, 32)
        nws = mr.mr_workspace_bytes(W, H, 100.0, mp, mr.MR_EFFECT_SSAO)
        assert lay.count == 0
        spans = []
        for i in (1, 2, 3):
            Wi, Hi = W >> (i - 1), H >> (i - 1)
            words = (Wi // 32) * Hi
            spans += [(lay.worklist[i - 1], 4 * Wi * Hi), (lay.stencil_bits[i - 1], 4 * words),
                      (lay.rank[i - 1], 4 * words)]
        assert lay.worklist[3] == 0
        spans.sort()
        assert spans[0][0] >= 4 * 6
        for (a, n), (b, _) in zip(spans, spans[1:]):
            assert a + n <= b
        assert spans[-1][0] + spans[-1][1] <= nws
    lay = mr.mr_frame_workspace_layout(mr.camera(200, 120, 100.0), mp.c(), mr.MR_EFFECT_SSAO)
    assert lay.compact == 0 and lay.worklist[0] == 0
    with pytest.raises(mr.MRError):
        mr.mr_frame_workspace_layout(mr.camera(0, 120, 100.0), mp.c(), mr.MR_EFFECT_SSAO)


def test_pyramid_and_scratch_sizes_on_the_host():
    """mr_pyramid_bytes (host call, no GPU): the resident pyramid holds every
    list, stencil-bit and rank region of the compact layout, pyramid plus
    scratch fit the frame's workspace, soft shadows need more scratch (the
    hard-shadow bytes), and parameters off the compact path are refused."""
    mp = mr.MaskParams(num_levels=4, level_enable=0xF, sigma2=(0.924, 1.848, 3.696, 0.0),
                       weight=(100.0, 50.0, 20.0, 1.0))
    for W, H in ((3840, 2160), (384, 256)):
        cam = mr.camera(W, H, 100.0)
        npyr, nscr = mr.mr_pyramid_bytes(W, H, 100.0, mp, mr.MR_EFFECT_SSAO)
        assert npyr > 0 and nscr > 0
        assert npyr + nscr <= mr.mr_workspace_bytes(W, H, 100.0, mp, mr.MR_EFFECT_SSAO)
        lay = mr.mr_frame_workspace_layout(cam, mp.c(), mr.MR_EFFECT_SSAO)
        for i in (1, 2, 3):
            Wi, Hi = W >> (i - 1), H >> (i - 1)
            assert lay.worklist[i - 1] + 4 * Wi * Hi <= npyr
            assert lay.stencil_bits[i - 1] + 4 * (Wi // 32) * Hi <= npyr
            assert lay.rank[i - 1] + 4 * (Wi // 32) * Hi <= npyr
        sp, ss = mr.mr_pyramid_bytes(W, H, 100.0, mp, mr.MR_EFFECT_SHADOW)
        assert sp == npyr and ss >= W * H
    with pytest.raises(mr.MRError):
        mr.mr_pyramid_bytes(200, 120, 100.0, mp, mr.MR_EFFECT_SSAO)  # width not divisible by 128
    with pytest.raises(mr.MRError):
        mr.mr_pyramid_bytes(384, 256, 100.0, mp, 7)


def test_frame_on_another_stream_holds_its_memory(monkeypatch):
    """A frame enqueued on a stream other than the current one records that
    stream on its workspace and output (torch's caching allocator then keeps
    the memory until the stream has passed that point); on the current
    stream, or with no stream, nothing is recorded."""
    class FakeTensor:
        def __init__(self):
            self.streams = []

        def record_stream(self, s):
            self.streams.append(s)

    current, other = object(), object()
    monkeypatch.setattr(mr.torch.cuda, "current_stream", lambda: current)
    fr = object.__new__(mr.FrameRunner)
    fr.workspace, fr.out = FakeTensor(), FakeTensor()
    fr._hold_for(None)
    fr._hold_for(current)
    assert fr.workspace.streams == [] and fr.out.streams == []
    fr._hold_for(other)
    assert fr.workspace.streams == [other] and fr.out.streams == [other]


def test_step_calls_on_another_stream_hold_what_they_use(monkeypatch):
    """The step entry points record a foreign stream on every tensor they
    write (the mask pyramid with its workspace, the level outputs, the merged
    image), and on none for the current stream or no stream."""
    class FakeTensor:
        def __init__(self):
            self.streams = []

        def record_stream(self, s):
            self.streams.append(s)

    current, other = object(), object()
    monkeypatch.setattr(mr.torch.cuda, "current_stream", lambda: current)
    m = mr.Masks(W=64, H=64, mp=mr.MaskParams(), edge=FakeTensor(), count=FakeTensor(), level_map=FakeTensor(),
                 alpha={2: FakeTensor()}, stencil={2: FakeTensor()}, worklist={2: FakeTensor()},
                 level_depth={2: FakeTensor(), 4: FakeTensor()}, workspace=FakeTensor())
    ts = m.tensors()
    assert len(ts) == 9 and len({id(t) for t in ts}) == 9
    mr._hold(None, *ts)
    mr._hold(current, *ts)
    assert all(t.streams == [] for t in ts)
    mr._hold(other, *ts, None)
    assert all(t.streams == [other] for t in ts)


def test_binding_constants_mirror_the_header():
    """Every MR_* integer constant the binding defines equals the header's
    #define of the same name (and the header defines it)."""
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mr.h")).read()
    defs = {}
    for name, val in re.findall(r"^#define (MR_[A-Z0-9_]+)\s+\(?(-?\d+)\)?\s*(?:/\*|$)", hdr, re.M):
        defs[name] = int(val)
    for name, a, b in re.findall(r"^#define (MR_[A-Z0-9_]+)\s+\((\d+)u?\s*<<\s*(\d+)\)", hdr, re.M):
        defs[name] = int(a) << int(b)
    names = [n for n in dir(mr) if n.startswith("MR_") and isinstance(getattr(mr, n), int)]
    assert len(names) > 15
    for n in names:
        assert n in defs, f"{n} is not defined in mr.h"
        assert getattr(mr, n) == defs[n], n


def test_a_c_client_builds_and_runs():
    """tests/native/abi_host.c includes mr.h as a C11 header, links libmr.so
    and calls the host-side entry points (sizes, layouts, validation)."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    libdir = os.path.join(root, "paper_1906_04576_amd")
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "abi_host")
        r = subprocess.run([gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(root, "include"),
                            os.path.join(root, "tests", "native", "abi_host.c"), "-L", libdir, "-lmr",
                            "-Wl,-rpath," + libdir, "-o", exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "0 failure(s)" in r.stdout and "FAIL" not in r.stdout
