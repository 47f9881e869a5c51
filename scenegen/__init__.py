"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This module holds no arithmetic of the multi-resolution method.  It produces
only *inputs*: G-buffers ray-cast in FP64 from seeded box/sphere scenes, the
light-view depth map and view-to-light transform for soft shadows, a
Lambert-lit colour buffer, and the random sample sets (SSAO hemisphere
kernel, PCSS disks) that the lighting estimators take as arguments.

Scenes stand in for the paper's Office / Hall / Breakfast Room scenes, which
are not available: a ground plane plus axis-aligned boxes (sides uniform in
[0.5, 2], centres uniform in a 10 x 10 area) and optionally spheres (radii
uniform in [0.2, 1.5]), seen from 8 orbit cameras (the paper averages over
3 scenes x 8 cameras, Sec. 5).  Random numbers come from splitmix64
(Steele, Lea and Flood, OOPSLA 2014).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raycast.c")
_LIB = os.path.join(_HERE, "_raycast.so")
_lib = None

MASK64 = (1 << 64) - 1


def build(force: bool = True) -> str:
    """Compile the FP64 ray caster (plain C, gcc) in-tree."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.rc_gbuffer.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp,
                                   ctypes.c_int, dp, ctypes.c_int, fp, fp, ip]
        lib.rc_gbuffer.restype = None
        lib.rc_depthmap.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_int, dp,
                                    ctypes.c_int, fp]
        lib.rc_depthmap.restype = None
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class SplitMix64:
    """splitmix64 generator; ``uniform`` returns (next() >> 11) * 2**-53."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------
# scenes and cameras
# --------------------------------------------------------------------------
@dataclass
class Scene:
    seed: int
    boxes: np.ndarray    # (nb, 6) xmin, ymin, zmin, xmax, ymax, zmax
    spheres: np.ndarray  # (ns, 4) cx, cy, cz, r
    albedo: np.ndarray = field(default=None)  # (1 + nb + ns, 3) plane first


def make_scene(seed: int, n_boxes: int, n_spheres: int = 0, ground_only: bool = False) -> Scene:
    """Ground plane y = 0 plus n_boxes boxes then n_spheres spheres.

    Draw order: per box (x, z, sx, sy, sz), then per sphere (x, z, r)."""
    rng = SplitMix64(seed)
    boxes = np.zeros((n_boxes, 6), np.float64)
    for b in range(n_boxes):
        x = -5.0 + 10.0 * rng.uniform()
        z = -5.0 + 10.0 * rng.uniform()
        sx = 0.5 + 1.5 * rng.uniform()
        sy = 0.5 + 1.5 * rng.uniform()
        sz = 0.5 + 1.5 * rng.uniform()
        boxes[b] = (x - 0.5 * sx, 0.0, z - 0.5 * sz, x + 0.5 * sx, sy, z + 0.5 * sz)
    spheres = np.zeros((n_spheres, 4), np.float64)
    for s in range(n_spheres):
        x = -5.0 + 10.0 * rng.uniform()
        z = -5.0 + 10.0 * rng.uniform()
        r = 0.2 + 1.3 * rng.uniform()
        spheres[s] = (x, r, z, r)
    if ground_only:
        boxes = boxes[:0]
        spheres = spheres[:0]
    arng = SplitMix64(seed ^ 0x5DEECE66D)
    n_obj = 1 + len(boxes) + len(spheres)
    albedo = np.empty((n_obj, 3), np.float64)
    albedo[0] = (0.8, 0.8, 0.8)
    for o in range(1, n_obj):
        albedo[o] = [0.2 + 0.8 * arng.uniform() for _ in range(3)]
    return Scene(seed, boxes, spheres, albedo)


def look_at(eye, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """View basis as 12 doubles: eye, right, up, back (world space)."""
    eye = np.asarray(eye, np.float64)
    back = eye - np.asarray(target, np.float64)
    back /= np.linalg.norm(back)
    right = np.cross(np.asarray(up, np.float64), back)
    right /= np.linalg.norm(right)
    upv = np.cross(back, right)
    return np.concatenate([eye, right, upv, back])


def orbit_view(k: int) -> np.ndarray:
    """Orbit camera k = 0..7: eye (11 sin t, 9, 11 cos t), t = k * 45 deg, at the origin."""
    t = math.radians(45.0 * k)
    return look_at((11.0 * math.sin(t), 9.0, 11.0 * math.cos(t)), (0.0, 0.0, 0.0))


def focal_px(height: int, fov_deg: float = 60.0) -> np.float32:
    """Focal length in pixels for a vertical field of view, rounded to FP32."""
    return np.float32((0.5 * height) / math.tan(math.radians(0.5 * fov_deg)))


@dataclass
class GBuffer:
    width: int
    height: int
    focal: np.float32
    depth: np.ndarray    # f32 [H][W] linear view depth, +inf = background
    normal: np.ndarray   # f32 [3][H][W] view-space unit normals (planar)
    objid: np.ndarray    # i32 [H][W], -1 background, 0 ground, then boxes, spheres
    view: np.ndarray     # 12 doubles


def render_gbuffer(scene: Scene, view: np.ndarray, width: int, height: int,
                   focal: np.float32 | None = None) -> GBuffer:
    lib = _load()
    if focal is None:
        focal = focal_px(height)
    depth = np.empty((height, width), np.float32)
    normal = np.empty((3, height, width), np.float32)
    objid = np.empty((height, width), np.int32)
    boxes = np.ascontiguousarray(scene.boxes, np.float64)
    spheres = np.ascontiguousarray(scene.spheres, np.float64)
    if boxes.size == 0:
        boxes = np.zeros((1, 6))
    if spheres.size == 0:
        spheres = np.zeros((1, 4))
    view = np.ascontiguousarray(view, np.float64)
    lib.rc_gbuffer(_ptr(view, ctypes.c_double), width, height, float(focal),
                   _ptr(boxes, ctypes.c_double), len(scene.boxes),
                   _ptr(spheres, ctypes.c_double), len(scene.spheres),
                   _ptr(depth, ctypes.c_float), _ptr(normal, ctypes.c_float),
                   _ptr(objid, ctypes.c_int32))
    return GBuffer(width, height, np.float32(focal), depth, normal, objid, view)


# --------------------------------------------------------------------------
# soft-shadow inputs
# --------------------------------------------------------------------------
LIGHT_EYE = (6.0, 14.0, 4.0)
LIGHT_TARGET = (0.0, 0.0, 0.0)


@dataclass
class ShadowInputs:
    shadow_map: np.ndarray      # f32 [size][size] linear light depth (+inf on miss)
    size: int
    light_focal: np.float32     # texels
    view_to_light: np.ndarray   # f32 [3][4]: camera view space -> light view space
    light_size: np.float32      # side of the square area light
    light_near: np.float32


def light_view() -> np.ndarray:
    return look_at(LIGHT_EYE, LIGHT_TARGET)


def render_shadow_inputs(scene: Scene, cam_view: np.ndarray, size: int = 2048,
                         fov_deg: float = 60.0, light_size: float = 0.5,
                         light_near: float = 1.0) -> ShadowInputs:
    lib = _load()
    lv = light_view()
    focal = focal_px(size, fov_deg)
    sm = np.empty((size, size), np.float32)
    boxes = np.ascontiguousarray(scene.boxes if len(scene.boxes) else np.zeros((1, 6)), np.float64)
    spheres = np.ascontiguousarray(scene.spheres if len(scene.spheres) else np.zeros((1, 4)), np.float64)
    lv = np.ascontiguousarray(lv)
    lib.rc_depthmap(_ptr(lv, ctypes.c_double), size, float(focal),
                    _ptr(boxes, ctypes.c_double), len(scene.boxes),
                    _ptr(spheres, ctypes.c_double), len(scene.spheres), _ptr(sm, ctypes.c_float))
    # camera view -> world: p_w = eye_c + [right up back]_c p ; world -> light view
    rc = np.stack([cam_view[3:6], cam_view[6:9], cam_view[9:12]], axis=1)  # columns
    rl = np.stack([lv[3:6], lv[6:9], lv[9:12]], axis=0)                     # rows
    m = np.zeros((3, 4))
    m[:, :3] = rl @ rc
    m[:, 3] = rl @ (cam_view[0:3] - lv[0:3])
    return ShadowInputs(sm, size, focal, m.astype(np.float32), np.float32(light_size),
                        np.float32(light_near))


def ground_only_shadow_map(size: int, fov_deg: float = 60.0) -> np.ndarray:
    """Light-view depth of the bare ground plane (no occluders)."""
    lib = _load()
    lv = np.ascontiguousarray(light_view())
    sm = np.empty((size, size), np.float32)
    z6, z4 = np.zeros((1, 6)), np.zeros((1, 4))
    lib.rc_depthmap(_ptr(lv, ctypes.c_double), size, float(focal_px(size, fov_deg)),
                    _ptr(z6, ctypes.c_double), 0, _ptr(z4, ctypes.c_double), 0,
                    _ptr(sm, ctypes.c_float))
    return sm


# --------------------------------------------------------------------------
# colour buffer for one-bounce indirect light
# --------------------------------------------------------------------------
def lambert_color(scene: Scene, gb: GBuffer) -> np.ndarray:
    """f16 [3][H][W]: albedo * (0.1 + 0.9 max(0, n.l)), l towards the light position."""
    l_w = np.asarray(LIGHT_EYE) - np.asarray(LIGHT_TARGET)
    l_w = l_w / np.linalg.norm(l_w)
    v = gb.view
    l_v = np.array([np.dot(l_w, v[3:6]), np.dot(l_w, v[6:9]), np.dot(l_w, v[9:12])])
    n = gb.normal.astype(np.float64)
    ndl = np.maximum(0.0, n[0] * l_v[0] + n[1] * l_v[1] + n[2] * l_v[2])
    ids = np.where(gb.objid < 0, 0, gb.objid)
    alb = scene.albedo[ids]  # H, W, 3
    col = alb * (0.1 + 0.9 * ndl)[..., None]
    col[gb.objid < 0] = 0.0
    return np.ascontiguousarray(np.moveaxis(col, -1, 0)).astype(np.float16)


# --------------------------------------------------------------------------
# sample sets (random inputs of the estimators)
# --------------------------------------------------------------------------
def ssao_kernel(samples: int, seed: int | None = None) -> np.ndarray:
    """f32 [S][3] hemisphere samples (z >= 0.01), lengths growing quadratically.

    Sample j: cz = 0.1 + 0.9 u1, phi = 2 pi u2, l = 0.1 + 0.9 ((j + u3)/S)^2,
    k = l (sqrt(1 - cz^2) cos phi, sqrt(1 - cz^2) sin phi, cz)."""
    rng = SplitMix64(1000 + samples if seed is None else seed)
    k = np.empty((samples, 3), np.float64)
    for j in range(samples):
        cz = 0.1 + 0.9 * rng.uniform()
        phi = 2.0 * math.pi * rng.uniform()
        ln = 0.1 + 0.9 * ((j + rng.uniform()) / samples) ** 2
        sz = math.sqrt(1.0 - cz * cz)
        k[j] = (ln * sz * math.cos(phi), ln * sz * math.sin(phi), ln * cz)
    return k.astype(np.float32)


def disk_samples(n: int, seed: int) -> np.ndarray:
    """f32 [n][2] points uniform in the unit disk: (sqrt(u1) cos 2pi u2, sqrt(u1) sin 2pi u2)."""
    rng = SplitMix64(seed)
    d = np.empty((n, 2), np.float64)
    for j in range(n):
        r = math.sqrt(rng.uniform())
        a = 2.0 * math.pi * rng.uniform()
        d[j] = (r * math.cos(a), r * math.sin(a))
    return d.astype(np.float32)


# --------------------------------------------------------------------------
# workload presets (sizes and parameters of the seeded workloads)
# --------------------------------------------------------------------------
# Table 1 of the paper: per-level blur variance and blend weight per effect.
TABLE1 = {
    "ssao":   {"sigma2": (0.924, 1.848, 3.696, 0.0), "weight": (100.0, 50.0, 20.0, 1.0)},
    "shadow": {"sigma2": (0.924, 1.848, 3.696, 0.0), "weight": (1000.0, 1000.0, 1000.0, 1.0)},
    "ssgi":   {"sigma2": (0.924, 0.0, 0.924, 0.0), "weight": (1000.0, 1.0, 100.0, 1.0)},
}

WORKLOADS = {
    # 256x256, 8 boxes, 3 levels, 16 samples, radius 0.5
    "ssao_256": dict(width=256, height=256, boxes=8, spheres=0, levels=3, samples=16, radius=0.5),
    # 1920x1080, 200 boxes + 50 spheres, 4 levels, 32 samples, radius 1.0
    "ssao_1080p": dict(width=1920, height=1080, boxes=200, spheres=50, levels=4, samples=32, radius=1.0),
    # the same generator at 3840x2160
    "ssao_4k": dict(width=3840, height=2160, boxes=200, spheres=50, levels=4, samples=32, radius=1.0),
    # soft shadows at 3840x2160, 2048^2 shadow map, 16 blocker + 32 PCF samples
    "pcss_4k": dict(width=3840, height=2160, boxes=200, spheres=50, levels=4, n_blocker=16, n_pcf=32,
                    sm_size=2048, light_size=0.5),
    # one-bounce indirect light, 64 samples, radius 2.0
    "ssgi": dict(boxes=200, spheres=50, levels=4, samples=64, radius=2.0),
}

SSGI_SIZES = ((640, 360), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160))
