"""Python binding of libmr (include/mr.h): argument marshalling only.

Every function here has the name of the C entry point it calls and takes
torch tensors that already live on the GPU; each step of the lighting path
runs in the HIP kernels of libmr.so.  PyTorch supplies device memory and the
current stream.  If libmr.so is missing or fails to load, every call raises:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmr.so")

# the header version whose structs this module mirrors
MR_VERSION = 101
MR_MAX_LEVELS = 6
MR_MAX_DIM = 16384
MR_OK, MR_E_NULL, MR_E_SHAPE, MR_E_PARAM, MR_E_WORKSPACE, MR_E_DTYPE, MR_E_DEVICE = 0, -1, -2, -3, -4, -5, -6
MR_F32, MR_F16 = 0, 1
MR_EFFECT_SSAO, MR_EFFECT_SHADOW, MR_EFFECT_SSGI = 0, 1, 2
MR_WS_MASKS = -1
MR_FRAME_EVENTS = 5
MR_MAX_BATCH = 64
MR_BATCH_PLAN_BYTES = 512
MR_STATIC_SCRATCH_BYTES = 64 << 20
EFFECTS = {"ssao": MR_EFFECT_SSAO, "shadow": MR_EFFECT_SHADOW, "ssgi": MR_EFFECT_SSGI}

c_float6 = ctypes.c_float * MR_MAX_LEVELS
c_int6 = ctypes.c_int * MR_MAX_LEVELS
c_ptr6 = ctypes.c_void_p * MR_MAX_LEVELS


class mr_gbuffer(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("normal", ctypes.c_void_p), ("normal_dtype", ctypes.c_int),
                ("color", ctypes.c_void_p), ("color_dtype", ctypes.c_int)]


class mr_camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("height", ctypes.c_int), ("focal_px", ctypes.c_float)]


class mr_fovea(ctypes.Structure):
    _fields_ = [("enable", ctypes.c_int), ("gaze_x", ctypes.c_float), ("gaze_y", ctypes.c_float),
                ("r_inner", ctypes.c_float), ("r_outer", ctypes.c_float)]


class mr_mask_params(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int), ("level_enable", ctypes.c_uint32),
                ("depth_ratio", ctypes.c_float), ("normal_cos", ctypes.c_float),
                ("sigma2", c_float6), ("weight", c_float6), ("radius", c_int6), ("fovea", mr_fovea)]


class mr_masks(ctypes.Structure):
    _fields_ = [("edge", ctypes.c_void_p), ("level_map", ctypes.c_void_p), ("alpha", c_ptr6),
                ("stencil", c_ptr6), ("worklist", c_ptr6), ("level_depth", c_ptr6),
                ("count", ctypes.c_void_p)]


class mr_ssao_params(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_void_p), ("samples", ctypes.c_int), ("radius", ctypes.c_float),
                ("bias_rel", ctypes.c_float)]


mr_ssgi_params = mr_ssao_params


class mr_shadow_params(ctypes.Structure):
    _fields_ = [("shadow_map", ctypes.c_void_p), ("sm_size", ctypes.c_int),
                ("view_to_light", ctypes.c_float * 12), ("light_focal_px", ctypes.c_float),
                ("light_size", ctypes.c_float), ("light_near", ctypes.c_float), ("bias", ctypes.c_float),
                ("blocker_disk", ctypes.c_void_p), ("pcf_disk", ctypes.c_void_p),
                ("n_blocker", ctypes.c_int), ("n_pcf", ctypes.c_int)]


class mr_bilateral_params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_uint32), ("radius", ctypes.c_int), ("depth_rel", ctypes.c_float)]


@dataclass
class Bilateral:
    """Bilateral blur of SSAO sub-images before the merge: bit i-1 of
    `levels` blurs level i; (2 radius + 1)^2 window; depth tolerance
    depth_rel relative to the centre depth."""
    levels: int = 0b1110
    radius: int = 2
    depth_rel: float = 0.05

    def c(self) -> mr_bilateral_params:
        return mr_bilateral_params(int(self.levels), int(self.radius), float(self.depth_rel))


class mr_frame_desc(ctypes.Structure):
    _fields_ = [("effect", ctypes.c_int), ("multires", ctypes.c_int), ("g", mr_gbuffer),
                ("cam", mr_camera), ("mp", mr_mask_params),
                ("ssao", ctypes.POINTER(mr_ssao_params)), ("shadow", ctypes.POINTER(mr_shadow_params)),
                ("ssgi", ctypes.POINTER(mr_ssgi_params)), ("out", ctypes.c_void_p),
                ("level_map", ctypes.c_void_p), ("level_dtype", ctypes.c_int),
                ("stage_events", ctypes.c_void_p * MR_FRAME_EVENTS), ("bilateral", mr_bilateral_params),
                ("eval_halo", ctypes.c_int)]


class mr_batch_config(ctypes.Structure):
    _fields_ = [("edge_tile", ctypes.c_int), ("eval_queue", ctypes.c_int), ("eval_blocks_per_cu", ctypes.c_int),
                ("merge_generic", ctypes.c_int), ("persistent", ctypes.c_int), ("eval_items", ctypes.c_int),
                ("worker_pixels", ctypes.c_int), ("tiles_per_ticket", ctypes.c_int), ("eval_halo", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mr_frame_layout(ctypes.Structure):
    _fields_ = [("compact", ctypes.c_int), ("tile_words", ctypes.c_int), ("tile_rows", ctypes.c_int),
                ("count", ctypes.c_size_t),
                ("worklist", ctypes.c_size_t * MR_MAX_LEVELS), ("stencil_bits", ctypes.c_size_t * MR_MAX_LEVELS),
                ("rank", ctypes.c_size_t * MR_MAX_LEVELS)]


# entry points and their ctypes signatures (also used by the export test)
_P = ctypes.c_void_p
SIGNATURES = {
    "mr_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(mr_camera), ctypes.POINTER(mr_mask_params), ctypes.c_int]),
    "mr_build_masks": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                      ctypes.POINTER(mr_mask_params), _P, ctypes.POINTER(mr_masks), _P,
                                      ctypes.c_size_t, _P]),
    "mr_eval_ssao": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                    ctypes.POINTER(mr_mask_params), ctypes.POINTER(mr_masks),
                                    ctypes.POINTER(mr_ssao_params), ctypes.POINTER(c_ptr6), _P]),
    "mr_shadow_hard": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                      ctypes.POINTER(mr_shadow_params), _P, _P]),
    "mr_eval_shadow": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                      ctypes.POINTER(mr_mask_params), ctypes.POINTER(mr_masks),
                                      ctypes.POINTER(mr_shadow_params), ctypes.POINTER(c_ptr6), _P]),
    "mr_eval_ssgi": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                    ctypes.POINTER(mr_mask_params), ctypes.POINTER(mr_masks),
                                    ctypes.POINTER(mr_ssgi_params), ctypes.POINTER(c_ptr6), _P]),
    "mr_upsample_merge": (ctypes.c_int, [ctypes.POINTER(mr_camera), ctypes.POINTER(mr_mask_params),
                                         ctypes.POINTER(mr_masks), ctypes.POINTER(c_ptr6), ctypes.c_int, _P, _P]),
    "mr_frame": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), _P, ctypes.c_size_t, _P]),
    "mr_frame_tune": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), _P, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_float), _P]),
    "mr_eval_ssao_fullres": (ctypes.c_int, [ctypes.POINTER(mr_gbuffer), ctypes.POINTER(mr_camera),
                                            ctypes.POINTER(mr_mask_params), ctypes.POINTER(mr_masks),
                                            ctypes.POINTER(ctypes.POINTER(mr_ssao_params) * MR_MAX_LEVELS),
                                            _P, _P]),
    "mr_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(mr_frame_desc), ctypes.c_int]),
    "mr_batch_setup": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), ctypes.c_int, _P, ctypes.c_size_t, _P,
                                      ctypes.c_size_t, _P]),
    "mr_batch_run": (ctypes.c_int, [_P, _P]),
    "mr_batch_get_config": (ctypes.c_int, [_P, ctypes.POINTER(mr_batch_config)]),
    "mr_batch_set_config": (ctypes.c_int, [_P, ctypes.POINTER(mr_batch_config)]),
    "mr_batch_tune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(mr_batch_config), _P]),
    "mr_batch_check": (ctypes.c_int, [_P, _P]),
    "mr_batch_staging_bytes": (ctypes.c_size_t, [ctypes.POINTER(mr_frame_desc), ctypes.c_int]),
    "mr_batch_cached_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(mr_frame_desc), ctypes.c_int]),
    "mr_batch_setup_cached": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.c_int, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P,
                                             ctypes.c_size_t, _P]),
    "mr_batch_setup_async": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), ctypes.c_int, _P, ctypes.c_size_t, _P,
                                            ctypes.c_size_t, _P, ctypes.c_size_t, _P]),
    "mr_frame_workspace_layout": (ctypes.c_int, [ctypes.POINTER(mr_camera), ctypes.POINTER(mr_mask_params),
                                                 ctypes.c_int, ctypes.POINTER(mr_frame_layout)]),
    "mr_frame_static": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), _P]),
    "mr_pyramid_bytes": (ctypes.c_int, [ctypes.POINTER(mr_camera), ctypes.POINTER(mr_mask_params), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "mr_frame_cached": (ctypes.c_int, [ctypes.POINTER(mr_frame_desc), _P, ctypes.c_size_t, ctypes.c_int, _P,
                                       ctypes.c_size_t, _P]),
    "mr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mr_last_error": (ctypes.c_char_p, []),
    "mr_version": (ctypes.c_int, []),
}

_lib = None


class MRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """The loaded libmr.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libmr.so not built at {LIB_PATH}; run paper_1906_04576_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.mr_version() != MR_VERSION:
            raise RuntimeError(f"{LIB_PATH} is version {L.mr_version()}, this binding mirrors version {MR_VERSION}; "
                               "rebuild it with paper_1906_04576_amd/build.py")
        _lib = L
    return _lib


def _check(status: int):
    if status != MR_OK:
        raise MRError(status, lib().mr_last_error().decode())


# ---------------------------------------------------------------------------
# parameter marshalling
# ---------------------------------------------------------------------------
@dataclass
class MaskParams:
    """Sec. 3.1 / Table 1 mask parameters (see mr_mask_params in mr.h)."""
    num_levels: int = 4
    level_enable: int = 0xF
    depth_ratio: float = 0.05
    normal_cos: float = math.cos(math.radians(25.0))
    sigma2: tuple = (0.924, 1.848, 3.696, 0.0)
    weight: tuple = (100.0, 50.0, 20.0, 1.0)
    radius: tuple = (-1, -1, -1, -1)
    fovea: tuple = None  # (gaze_x, gaze_y, r_inner, r_outer) or None

    def levels(self):
        return [i for i in range(1, self.num_levels + 1) if (self.level_enable >> (i - 1)) & 1]

    def c(self) -> mr_mask_params:
        p = mr_mask_params()
        p.num_levels = self.num_levels
        p.level_enable = self.level_enable
        p.depth_ratio = self.depth_ratio
        p.normal_cos = self.normal_cos
        for i in range(MR_MAX_LEVELS):
            p.sigma2[i] = self.sigma2[i] if i < len(self.sigma2) else 0.0
            p.weight[i] = self.weight[i] if i < len(self.weight) else 1.0
            p.radius[i] = self.radius[i] if i < len(self.radius) else -1
        if self.fovea is not None:
            p.fovea.enable = 1
            p.fovea.gaze_x, p.fovea.gaze_y, p.fovea.r_inner, p.fovea.r_outer = (float(v) for v in self.fovea)
        return p


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dt(t):
    if t is None:
        return MR_F32
    if t.dtype == torch.float32:
        return MR_F32
    if t.dtype == torch.float16:
        return MR_F16
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, what, dtypes=(torch.float32,)):
    if t is None:
        return
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.dtype not in dtypes:
        raise TypeError(f"{what} has dtype {t.dtype}")


def gbuffer(depth, normal=None, color=None) -> mr_gbuffer:
    _dev(depth, "depth")
    _dev(normal, "normal", (torch.float32, torch.float16))
    _dev(color, "color", (torch.float32, torch.float16))
    return mr_gbuffer(_ptr(depth), _ptr(normal), _dt(normal), _ptr(color), _dt(color))


def camera(width, height, focal) -> mr_camera:
    return mr_camera(int(width), int(height), float(focal))


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _hold(stream, *tensors):
    """Work enqueued on a stream other than torch's current one keeps the
    memory it uses alive for that stream: torch's caching allocator would
    otherwise hand that memory to the next allocation on the current stream
    while the work still runs."""
    if stream is not None and stream != torch.cuda.current_stream():
        for t in tensors:
            if t is not None:
                t.record_stream(stream)


def level_dims(W, H, i):
    return W >> (i - 1), H >> (i - 1)


@dataclass
class Masks:
    """Device tensors of one mask pyramid (see mr_masks in mr.h)."""
    W: int
    H: int
    mp: MaskParams
    edge: torch.Tensor
    count: torch.Tensor
    level_map: torch.Tensor = None
    alpha: dict = field(default_factory=dict)
    stencil: dict = field(default_factory=dict)
    worklist: dict = field(default_factory=dict)
    level_depth: dict = field(default_factory=dict)
    workspace: torch.Tensor = None

    def tensors(self) -> list:
        """Every device tensor of the pyramid, its workspace included."""
        t = [self.edge, self.count, self.level_map, self.workspace]
        for d in (self.alpha, self.stencil, self.worklist, self.level_depth):
            t.extend(d.values())
        return [x for x in t if x is not None]

    def c(self) -> mr_masks:
        m = mr_masks()
        m.edge = _ptr(self.edge)
        m.level_map = _ptr(self.level_map)
        m.count = _ptr(self.count)
        for i, t in self.alpha.items():
            m.alpha[i - 1] = t.data_ptr()
        for i, t in self.stencil.items():
            m.stencil[i - 1] = t.data_ptr()
        for i, t in self.worklist.items():
            m.worklist[i - 1] = t.data_ptr()
        for i, t in self.level_depth.items():
            m.level_depth[i - 1] = t.data_ptr()
        return m


def mr_workspace_bytes(W, H, focal, mp: MaskParams, purpose) -> int:
    cam = camera(W, H, focal)
    cmp = mp.c()
    n = lib().mr_workspace_bytes(ctypes.byref(cam), ctypes.byref(cmp), int(purpose))
    if n == 0:
        raise MRError(MR_E_PARAM, lib().mr_last_error().decode())
    return int(n)


def alloc_masks(W, H, focal, mp: MaskParams, device="cuda", level_map=True, level_depth=True) -> Masks:
    levels = mp.levels()
    L = levels[-1]
    u8 = dict(dtype=torch.uint8, device=device)
    f32 = dict(dtype=torch.float32, device=device)
    m = Masks(W, H, mp, edge=torch.empty((H, W), **u8), count=torch.zeros(8, dtype=torch.int32, device=device))
    if level_map:
        m.level_map = torch.empty((H, W), **u8)
    for i in levels:
        Wi, Hi = level_dims(W, H, i)
        if i != L:
            m.alpha[i] = torch.empty((Hi, Wi), **f32)
            m.stencil[i] = torch.empty((Hi, Wi), **u8)
            m.worklist[i] = torch.empty(Hi * Wi, dtype=torch.int32, device=device)
        if i >= 2 and level_depth:
            m.level_depth[i] = torch.empty((Hi, Wi), **f32)
    nws = mr_workspace_bytes(W, H, focal, mp, MR_WS_MASKS)
    m.workspace = torch.empty(nws, **u8)
    return m


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def mr_build_masks(depth, normal, focal, mp: MaskParams, hard_shadow=None, masks: Masks = None,
                   level_map=True, level_depth=True, stream=None) -> Masks:
    H, W = depth.shape
    if masks is None:
        masks = alloc_masks(W, H, focal, mp, depth.device, level_map, level_depth)
    _dev(hard_shadow, "hard_shadow", (torch.uint8,))
    g = gbuffer(depth, normal)
    cam = camera(W, H, focal)
    cmp = mp.c()
    cm = masks.c()
    _hold(stream, *masks.tensors())
    _check(lib().mr_build_masks(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cmp), _ptr(hard_shadow),
                                ctypes.byref(cm), _ptr(masks.workspace), masks.workspace.numel(),
                                _stream(stream)))
    return masks


def _level_outputs(W, H, levels, C, device, plain):
    out = {}
    for i in ([1] if plain else levels):
        Wi, Hi = level_dims(W, H, i)
        shape = (C, Hi, Wi) if C > 1 else (Hi, Wi)
        out[i] = torch.full(shape, float("nan"), dtype=torch.float32, device=device)
    return out


def _eval(name, g, W, H, focal, mp, masks, params_c, C, out, stream):
    levels = mp.levels() if masks is not None else [1]
    if out is None:
        out = _level_outputs(W, H, levels, C, g_device(g), masks is None)
    arr = c_ptr6()
    for i, t in out.items():
        arr[i - 1] = t.data_ptr()
    cam = camera(W, H, focal)
    cmp = mp.c() if mp is not None else None
    cm = masks.c() if masks is not None else None
    fn = getattr(lib(), name)
    _hold(stream, *out.values())
    _check(fn(ctypes.byref(g[0]), ctypes.byref(cam), ctypes.byref(cmp) if cmp is not None else None,
              ctypes.byref(cm) if cm is not None else None, ctypes.byref(params_c), ctypes.byref(arr),
              _stream(stream)))
    return out


class FullresRunner:
    """Pre-marshalled mr_eval_ssao_fullres call: SSAO with every level's
    sub-image at full resolution with its own sample set.  level_params:
    {level: mr_ssao_params} for every enabled level; masks from
    mr_build_masks of the same frame."""

    def __init__(self, depth, normal, focal, mp: MaskParams, masks: "Masks", level_params: dict, out=None):
        H, W = depth.shape
        self.out = out if out is not None else torch.empty((H, W), dtype=torch.float32, device=depth.device)
        self.g = gbuffer(depth, normal)
        self.cam = camera(W, H, focal)
        self.cmp = mp.c()
        self.cm = masks.c()
        self.lp = (ctypes.POINTER(mr_ssao_params) * MR_MAX_LEVELS)()
        for i, p in level_params.items():
            self.lp[i - 1] = ctypes.pointer(p)
        self._keep = (depth, normal, masks, level_params)
        self._fn = lib().mr_eval_ssao_fullres

    def __call__(self, stream=None):
        _hold(stream, self.out)
        _check(self._fn(ctypes.byref(self.g), ctypes.byref(self.cam), ctypes.byref(self.cmp), ctypes.byref(self.cm),
                        ctypes.byref(self.lp), _ptr(self.out), _stream(stream)))
        return self.out


def mr_eval_ssao_fullres(depth, normal, focal, mp: MaskParams, masks: "Masks", level_params: dict, out=None,
                         stream=None):
    return FullresRunner(depth, normal, focal, mp, masks, level_params, out)(stream)


def g_device(g):
    return g[1]


def ssao_params(kernel, radius, bias_rel) -> mr_ssao_params:
    """SSAO / SSGI sampling parameters.  The returned struct holds a reference
    to `kernel`, so the device memory it points to lives as long as it does."""
    _dev(kernel, "kernel")
    p = mr_ssao_params(_ptr(kernel), int(kernel.shape[0]), float(radius), float(bias_rel))
    p._tensors = (kernel,)
    return p


def mr_eval_ssao(depth, normal, focal, kernel, radius, bias_rel, mp: MaskParams = None, masks: Masks = None,
                 out=None, stream=None):
    """Per-level SSAO (masks given) or the naive full-resolution pass."""
    H, W = depth.shape
    p = ssao_params(kernel, radius, bias_rel)
    return _eval("mr_eval_ssao", (gbuffer(depth, normal), depth.device), W, H, focal, mp, masks, p, 1, out,
                 stream)


def shadow_params(shadow_map, view_to_light, light_focal, light_size, light_near, bias, blocker_disk,
                  pcf_disk) -> mr_shadow_params:
    _dev(shadow_map, "shadow_map")
    _dev(blocker_disk, "blocker_disk")
    _dev(pcf_disk, "pcf_disk")
    p = mr_shadow_params()
    p.shadow_map = _ptr(shadow_map)
    p.sm_size = int(shadow_map.shape[0])
    m = [float(v) for v in list(view_to_light.reshape(-1))]
    for k in range(12):
        p.view_to_light[k] = m[k]
    p.light_focal_px = float(light_focal)
    p.light_size = float(light_size)
    p.light_near = float(light_near)
    p.bias = float(bias)
    p.blocker_disk = _ptr(blocker_disk)
    p.pcf_disk = _ptr(pcf_disk)
    p.n_blocker = int(blocker_disk.shape[0])
    p.n_pcf = int(pcf_disk.shape[0])
    # keep the device arrays alive as long as the struct that points to them
    p._tensors = (shadow_map, blocker_disk, pcf_disk)
    return p


def mr_shadow_hard(depth, focal, sp: mr_shadow_params, hard=None, stream=None):
    H, W = depth.shape
    if hard is None:
        hard = torch.empty((H, W), dtype=torch.uint8, device=depth.device)
    g = gbuffer(depth)
    cam = camera(W, H, focal)
    _hold(stream, hard)
    _check(lib().mr_shadow_hard(ctypes.byref(g), ctypes.byref(cam), ctypes.byref(sp), _ptr(hard), _stream(stream)))
    return hard


def mr_eval_shadow(depth, focal, sp: mr_shadow_params, mp: MaskParams = None, masks: Masks = None, out=None,
                   stream=None):
    H, W = depth.shape
    return _eval("mr_eval_shadow", (gbuffer(depth), depth.device), W, H, focal, mp, masks, sp, 1, out, stream)


def mr_eval_ssgi(depth, normal, color, focal, kernel, radius, bias_rel, mp: MaskParams = None,
                 masks: Masks = None, out=None, stream=None):
    H, W = depth.shape
    p = ssao_params(kernel, radius, bias_rel)
    return _eval("mr_eval_ssgi", (gbuffer(depth, normal, color), depth.device), W, H, focal, mp, masks, p, 3,
                 out, stream)


def mr_upsample_merge(focal, mp: MaskParams, masks: Masks, level_out: dict, channels=1, out=None, stream=None):
    W, H = masks.W, masks.H
    if out is None:
        shape = (channels, H, W) if channels > 1 else (H, W)
        out = torch.empty(shape, dtype=torch.float32, device=masks.edge.device)
    arr = c_ptr6()
    for i, t in level_out.items():
        arr[i - 1] = t.data_ptr()
    cam = camera(W, H, focal)
    cmp = mp.c()
    cm = masks.c()
    _hold(stream, out)
    _check(lib().mr_upsample_merge(ctypes.byref(cam), ctypes.byref(cmp), ctypes.byref(cm), ctypes.byref(arr),
                                   int(channels), _ptr(out), _stream(stream)))
    return out


_hip = None


def _hip_runtime():
    """The HIP runtime torch has loaded (one runtime per process)."""
    global _hip
    if _hip is None:
        path = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
        _hip = ctypes.CDLL(path if os.path.exists(path) else "libamdhip64.so")
        _hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        _hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        _hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        _hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    return _hip


HIP_EVENT_RELEASE_TO_DEVICE = 0x40000000  # hipEventReleaseToDevice


class DeviceEvent:
    """A timing event recorded with a device-scope release, so that marking a
    stage boundary does not write caches back to the system between two
    kernels (torch's events use the default, system-scope release)."""

    def __init__(self):
        torch.cuda.init()
        h = ctypes.c_void_p()
        err = _hip_runtime().hipEventCreateWithFlags(ctypes.byref(h), HIP_EVENT_RELEASE_TO_DEVICE)
        if err != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({err})")
        self.handle = h.value

    def elapsed_ms(self, later: "DeviceEvent") -> float:
        ms = ctypes.c_float()
        err = _hip_runtime().hipEventElapsedTime(ctypes.byref(ms), self.handle, later.handle)
        if err != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({err})")
        return ms.value

    def __del__(self):
        if getattr(self, "handle", None) and _hip is not None:
            _hip.hipEventDestroy(self.handle)


def record(event: DeviceEvent, stream=None):
    """Record a DeviceEvent on `stream` (default: torch's current stream)."""
    err = _hip_runtime().hipEventRecord(event.handle, _stream(stream))
    if err != 0:
        raise RuntimeError(f"hipEventRecord failed ({err})")


class FrameRunner:
    """Pre-marshalled mr_frame call: the descriptor and workspace are built
    once so that repeated calls cost one ctypes call each."""

    def __init__(self, effect, depth, normal, focal, mp: MaskParams, multires=True, color=None, params=None,
                 out=None, level_map=None, workspace=None, level_dtype=torch.float32, bilateral: Bilateral = None,
                 ws_bytes=None, eval_halo=0):
        self.effect = EFFECTS[effect] if isinstance(effect, str) else int(effect)
        H, W = depth.shape
        C = 3 if self.effect == MR_EFFECT_SSGI else 1
        self.out = out if out is not None else torch.empty((C, H, W) if C > 1 else (H, W), dtype=torch.float32,
                                                           device=depth.device)
        d = mr_frame_desc()
        d.effect = self.effect
        d.multires = 1 if multires else 0
        d.g = gbuffer(depth, normal, color)
        d.cam = camera(W, H, focal)
        d.mp = mp.c()
        self._params = params
        if self.effect == MR_EFFECT_SSAO:
            d.ssao = ctypes.pointer(params)
        elif self.effect == MR_EFFECT_SHADOW:
            d.shadow = ctypes.pointer(params)
        else:
            d.ssgi = ctypes.pointer(params)
        d.out = _ptr(self.out)
        d.level_map = _ptr(level_map)
        d.level_dtype = MR_F16 if level_dtype == torch.float16 else MR_F32
        if bilateral is not None:
            d.bilateral = bilateral.c()
        d.eval_halo = int(eval_halo)
        self.desc = d
        self._keep = (depth, normal, color, level_map)
        nws = ws_bytes if ws_bytes is not None else (mr_workspace_bytes(W, H, focal, mp, self.effect) if multires else 0)
        if workspace is not None and workspace.numel() >= nws:
            self.workspace = workspace
        else:
            self.workspace = torch.empty(max(nws, 256), dtype=torch.uint8, device=depth.device)
        self._fn = lib().mr_frame
        self._ws = _ptr(self.workspace)
        self._nws = self.workspace.numel()

    def set_stage_events(self, events):
        """Have mr_frame record `events` (MR_FRAME_EVENTS DeviceEvent or
        torch.cuda.Event objects with timing, or None to stop) at its stage
        boundaries."""
        if events is None:
            for k in range(MR_FRAME_EVENTS):
                self.desc.stage_events[k] = None
            self._events = None
            return
        if len(events) != MR_FRAME_EVENTS:
            raise ValueError(f"need {MR_FRAME_EVENTS} events")
        for k, e in enumerate(events):
            if isinstance(e, DeviceEvent):
                self.desc.stage_events[k] = e.handle
                continue
            if not e.cuda_event:  # torch creates the HIP event at its first record
                e.record()
            self.desc.stage_events[k] = e.cuda_event
        self._events = tuple(events)

    def _hold_for(self, stream):
        """A frame enqueued on a stream other than torch's current one
        keeps its workspace and output alive for that stream: torch's caching
        allocator would otherwise hand their memory to the next allocation on
        the current stream while the frame still runs."""
        _hold(stream, self.workspace, self.out)

    def __call__(self, stream=None):
        self._hold_for(stream)
        _check(self._fn(ctypes.byref(self.desc), self._ws, self._nws, _stream(stream)))
        return self.out

    def tune(self, reps=10, stream=None):
        """mr_frame_tune: time the frame with every depth-halo size it admits
        and keep the fastest in the descriptor.  Returns (eval_halo, {halo:
        ms per frame}) for the sizes that were timed."""
        self._hold_for(stream)
        ms = (ctypes.c_float * 4)()
        _check(lib().mr_frame_tune(ctypes.byref(self.desc), self._ws, self._nws, int(reps), ms, _stream(stream)))
        return self.desc.eval_halo, {h: float(t) for h, t in zip((0, 8, 16, 24), ms) if t >= 0.0}

    def layout(self) -> mr_frame_layout:
        return mr_frame_workspace_layout(self.desc.cam, self.desc.mp, self.effect)

    def lists(self) -> dict:
        """After the frame has completed: {level: (worklist, stencil bits,
        ranks)} of the compact path's list levels as CPU int64 / uint32
        arrays, read from the workspace."""
        import numpy as np
        lay = self.layout()
        if not lay.compact:
            raise ValueError("the frame does not take the compact path")
        ws = self.workspace
        W, H = self.desc.cam.width, self.desc.cam.height

        def words(off, n):
            return ws[off:off + 4 * n].cpu().numpy().view(np.uint32)

        counts = words(lay.count, MR_MAX_LEVELS)
        res = {}
        for i in range(1, MR_MAX_LEVELS + 1):
            if not lay.worklist[i - 1]:
                continue
            Wi, Hi = W >> (i - 1), H >> (i - 1)
            n = int(counts[i - 1])
            res[i] = (words(lay.worklist[i - 1], n).astype(np.int64),
                      words(lay.stencil_bits[i - 1], Hi * (Wi // 32)).reshape(Hi, Wi // 32),
                      words(lay.rank[i - 1], Hi * (Wi // 32)).reshape(Hi, Wi // 32))
        return res


def mr_frame_workspace_layout(cam: mr_camera, cmp: mr_mask_params, effect) -> mr_frame_layout:
    lay = mr_frame_layout()
    _check(lib().mr_frame_workspace_layout(ctypes.byref(cam), ctypes.byref(cmp), int(effect), ctypes.byref(lay)))
    return lay


def mr_pyramid_bytes(W, H, focal, mp: MaskParams, effect) -> tuple:
    """(pyramid bytes, scratch bytes) of a frame with a resident pyramid."""
    cam, cmp = camera(W, H, focal), mp.c()
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mr_pyramid_bytes(ctypes.byref(cam), ctypes.byref(cmp), int(effect), ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


class CachedFrameRunner(FrameRunner):
    """mr_frame_cached: the frame with its mask pyramid in `pyramid` (a
    device tensor of at least the pyramid size, kept by the caller across
    frames of the same inputs).  call(build=True) computes the masks into
    it, call(build=False) reuses them."""

    def __init__(self, effect, depth, normal, focal, mp: MaskParams, pyramid, color=None, params=None, out=None,
                 level_map=None, workspace=None, level_dtype=torch.float32, bilateral: Bilateral = None):
        eff = EFFECTS[effect] if isinstance(effect, str) else int(effect)
        H, W = depth.shape
        npyr, nscr = mr_pyramid_bytes(W, H, focal, mp, eff)
        if pyramid.numel() < npyr:
            raise ValueError(f"pyramid needs {npyr} bytes")
        super().__init__(effect, depth, normal, focal, mp, True, color, params, out, level_map, workspace=workspace,
                         level_dtype=level_dtype, bilateral=bilateral, ws_bytes=nscr)
        self.pyramid = pyramid
        self._pyr = _ptr(pyramid)
        self._npyr = pyramid.numel()
        self._cfn = lib().mr_frame_cached

    def __call__(self, stream=None, build=True):
        _hold(stream, self.workspace, self.out, self.pyramid)
        _check(self._cfn(ctypes.byref(self.desc), self._pyr, self._npyr, 1 if build else 0, self._ws, self._nws,
                         _stream(stream)))
        return self.out


class StaticFrameRunner(FrameRunner):
    """mr_frame_static: the frame with the library's static device scratch
    instead of a workspace (for callers that cannot allocate).  Frames on
    one device share that scratch, so they must not overlap."""

    def __init__(self, effect, depth, normal, focal, mp: MaskParams, multires=True, color=None, params=None,
                 out=None, level_map=None, level_dtype=torch.float32, bilateral: Bilateral = None):
        super().__init__(effect, depth, normal, focal, mp, multires, color, params, out, level_map,
                         workspace=torch.empty(256, dtype=torch.uint8, device=depth.device),
                         level_dtype=level_dtype, bilateral=bilateral)
        self._fn = lib().mr_frame_static

    def __call__(self, stream=None):
        _hold(stream, self.out)
        _check(self._fn(ctypes.byref(self.desc), _stream(stream)))
        return self.out


def mr_frame(effect, depth, normal, focal, mp: MaskParams, params, multires=True, color=None, out=None,
             level_map=None, stream=None, level_dtype=torch.float32, bilateral: Bilateral = None, eval_halo=0):
    return FrameRunner(effect, depth, normal, focal, mp, multires, color, params, out, level_map,
                       level_dtype=level_dtype, bilateral=bilateral, eval_halo=eval_halo)(stream)


def _batch_descs(effect: int, frames, mp: MaskParams, params, level_dtype):
    """Frame descriptors of a batch, the output tensors (allocated where a
    frame brings none) and the tensors the descriptors point into."""
    n = len(frames)
    descs = (mr_frame_desc * n)()
    outs, keep = [], [params]
    C = 3 if effect == MR_EFFECT_SSGI else 1
    for k, f in enumerate(frames):
        depth, normal, color = f["depth"], f["normal"], f.get("color")
        H, W = depth.shape
        out = f.get("out")
        if out is None:
            out = torch.empty((C, H, W) if C > 1 else (H, W), dtype=torch.float32, device=depth.device)
        d = descs[k]
        d.effect = effect
        d.multires = 1
        d.g = gbuffer(depth, normal, color)
        d.cam = camera(W, H, f["focal"])
        d.mp = mp.c()
        if effect == MR_EFFECT_SSAO:
            d.ssao = ctypes.pointer(params)
        else:
            d.ssgi = ctypes.pointer(params)
        d.out = _ptr(out)
        d.level_dtype = MR_F16 if level_dtype == torch.float16 else MR_F32
        outs.append(out)
        keep += [depth, normal, color]
    return descs, outs, keep


class Batch:
    """Frames of one effect (same mask and effect parameters, any sizes)
    run with one launch per stage, or in one persistent launch
    (config["persistent"] = 1), through mr_batch_setup / mr_batch_run.
    frames: list of FrameRunner-style argument dicts:
        dict(depth=, normal=, focal=, color=None, out=None)
    The frame tensors must stay alive and at the same addresses."""

    def __init__(self, effect, frames, mp: MaskParams, params, level_dtype=torch.float32, stream=None):
        self.effect = EFFECTS[effect] if isinstance(effect, str) else int(effect)
        n = len(frames)
        descs, self.outs, self._keep = _batch_descs(self.effect, frames, mp, params, level_dtype)
        self.descs = descs
        nws = lib().mr_batch_workspace_bytes(descs, n)
        if nws == 0:
            _check(MR_E_PARAM)
        self.workspace = torch.empty(nws, dtype=torch.uint8, device=frames[0]["depth"].device)
        self.plan = (ctypes.c_uint8 * MR_BATCH_PLAN_BYTES)()
        _check(lib().mr_batch_setup(descs, n, _ptr(self.workspace), nws, ctypes.cast(self.plan, ctypes.c_void_p),
                                    MR_BATCH_PLAN_BYTES, _stream(stream)))
        self._run = lib().mr_batch_run

    def __call__(self, stream=None):
        _hold(stream, self.workspace, *self.outs)
        _check(self._run(ctypes.cast(self.plan, ctypes.c_void_p), _stream(stream)))
        return self.outs

    @property
    def config(self) -> dict:
        c = mr_batch_config()
        _check(lib().mr_batch_get_config(ctypes.cast(self.plan, ctypes.c_void_p), ctypes.byref(c)))
        return c.as_dict()

    @config.setter
    def config(self, cfg: dict):
        c = mr_batch_config()
        lib().mr_batch_get_config(ctypes.cast(self.plan, ctypes.c_void_p), ctypes.byref(c))
        for k, v in cfg.items():
            setattr(c, k, int(v))
        _check(lib().mr_batch_set_config(ctypes.cast(self.plan, ctypes.c_void_p), ctypes.byref(c)))

    def check(self, stream=None):
        """mr_batch_check: waits for the stream and raises MRError if a
        persistent run gave up waiting for a stage since the last check."""
        _check(lib().mr_batch_check(ctypes.cast(self.plan, ctypes.c_void_p), _stream(stream)))

    def tune(self, reps=5, stream=None) -> dict:
        """Autotune the plan's launch configuration on the current inputs
        (mr_batch_tune); returns the configuration kept."""
        c = mr_batch_config()
        _check(lib().mr_batch_tune(ctypes.cast(self.plan, ctypes.c_void_p), int(reps), ctypes.byref(c),
                                   _stream(stream)))
        return c.as_dict()


class BatchSlot:
    """Memory for batches formed on the fly (mr_batch_setup_async): a device
    workspace and a page-locked staging buffer of fixed sizes.  run() sets up
    a batch of the given frames and enqueues it on the stream without
    waiting; the slot may take its next batch once the stream has passed
    this one (the caller orders that, e.g. with an event)."""

    def __init__(self, ws_bytes: int, staging_bytes: int, device="cuda"):
        self.workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=device)
        self.staging = torch.empty(staging_bytes, dtype=torch.uint8, pin_memory=True)
        self.plan = (ctypes.c_uint8 * MR_BATCH_PLAN_BYTES)()
        self._keep = None

    @staticmethod
    def sizes(effect, frames, mp: MaskParams, params, level_dtype=torch.float32, cached=False) -> tuple:
        """(workspace bytes, staging bytes) of a batch of these frames
        (cached: on resident pyramids, scratch only)."""
        eff = EFFECTS[effect] if isinstance(effect, str) else int(effect)
        descs, _, _ = _batch_descs(eff, frames, mp, params, level_dtype)
        fn = lib().mr_batch_cached_workspace_bytes if cached else lib().mr_batch_workspace_bytes
        nws = fn(descs, len(frames))
        nst = lib().mr_batch_staging_bytes(descs, len(frames))
        if nws == 0 or nst == 0:
            _check(MR_E_PARAM)
        return int(nws), int(nst)

    def run(self, effect, frames, mp: MaskParams, params, stream=None, level_dtype=torch.float32, pyramids=None):
        """pyramids: per frame a device tensor holding that frame's built
        mask pyramid (mr_batch_setup_cached: evaluation and merge only)."""
        eff = EFFECTS[effect] if isinstance(effect, str) else int(effect)
        descs, outs, keep = _batch_descs(eff, frames, mp, params, level_dtype)
        _hold(stream, self.workspace, *outs, *(pyramids or ()))
        if pyramids is not None:
            pp = (ctypes.c_void_p * len(frames))(*[t.data_ptr() for t in pyramids])
            keep = keep + [pyramids, pp]
            _check(lib().mr_batch_setup_cached(descs, pp, len(frames), _ptr(self.workspace), self.workspace.numel(),
                                               ctypes.cast(self.plan, ctypes.c_void_p), MR_BATCH_PLAN_BYTES,
                                               _ptr(self.staging), self.staging.numel(), _stream(stream)))
        else:
            _check(lib().mr_batch_setup_async(descs, len(frames), _ptr(self.workspace), self.workspace.numel(),
                                              ctypes.cast(self.plan, ctypes.c_void_p), MR_BATCH_PLAN_BYTES,
                                              _ptr(self.staging), self.staging.numel(), _stream(stream)))
        _check(lib().mr_batch_run(ctypes.cast(self.plan, ctypes.c_void_p), _stream(stream)))
        self._keep = (descs, keep)  # the frame descriptors' targets stay alive until the next batch
        return outs


class Prepared:
    """One C entry point with its ctypes arguments built once; calling it
    costs a single foreign call (used where Python overhead would otherwise
    leave the GPU idle between short launches)."""

    def __init__(self, name, args, keep=()):
        self._fn = getattr(lib(), name)
        self._args = args
        self._keep = keep

    def __call__(self):
        _check(self._fn(*self._args))


def prepare_build_masks(depth, normal, focal, mp: MaskParams, masks: Masks, hard_shadow=None, stream=None):
    H, W = depth.shape
    g, cam, cmp, cm = gbuffer(depth, normal), camera(W, H, focal), mp.c(), masks.c()
    args = (ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cmp), _ptr(hard_shadow), ctypes.byref(cm),
            _ptr(masks.workspace), masks.workspace.numel(), _stream(stream))
    return Prepared("mr_build_masks", args, (g, cam, cmp, cm, masks, depth, normal, hard_shadow))


def prepare_eval_ssao(depth, normal, focal, params: mr_ssao_params, out: dict, mp: MaskParams = None,
                      masks: Masks = None, stream=None):
    H, W = depth.shape
    g, cam = gbuffer(depth, normal), camera(W, H, focal)
    cmp = mp.c() if mp is not None else None
    cm = masks.c() if masks is not None else None
    arr = c_ptr6()
    for i, t in out.items():
        arr[i - 1] = t.data_ptr()
    args = (ctypes.byref(g), ctypes.byref(cam), ctypes.byref(cmp) if cmp is not None else None,
            ctypes.byref(cm) if cm is not None else None, ctypes.byref(params), ctypes.byref(arr), _stream(stream))
    return Prepared("mr_eval_ssao", args, (g, cam, cmp, cm, arr, params, out, masks, depth, normal))


def prepare_upsample_merge(focal, mp: MaskParams, masks: Masks, level_out: dict, out, channels=1, stream=None):
    cam, cmp, cm = camera(masks.W, masks.H, focal), mp.c(), masks.c()
    arr = c_ptr6()
    for i, t in level_out.items():
        arr[i - 1] = t.data_ptr()
    args = (ctypes.byref(cam), ctypes.byref(cmp), ctypes.byref(cm), ctypes.byref(arr), int(channels), _ptr(out),
            _stream(stream))
    return Prepared("mr_upsample_merge", args, (cam, cmp, cm, arr, masks, level_out, out))


def mr_version() -> int:
    return lib().mr_version()


def mr_status_string(status: int) -> str:
    return lib().mr_status_string(int(status)).decode()


def mr_last_error() -> str:
    return lib().mr_last_error().decode()
