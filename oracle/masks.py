"""Mask creation: edge image, mask pyramid, stencils, partition, work lists.

Paper passages: Sec. 3.1 (Mask Creation) and Table 1 for the edge image, the
downsampling, the blur variances and the inclusive decomposition; Sec. 4
(Implementation) for the four levels of successively halved width and the
SSGI choice of skipping the half-resolution level; Sec. 4.1 for stencil =
mask > 0.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class MaskParams:
    """Per-frame mask parameters.

    num_levels   N: level i (1-based) has scale s_i = 2**(i-1).
    level_enable bit (i-1) set = level i used.  Bits 0 and N-1 must be set.
    depth_ratio  threshold on the relative depth second difference.
    normal_cos   threshold on the dot product of neighbouring normals.
    sigma2       blur variance per level, in level-i texels (Table 1).
    weight       blend weight per level (Table 1).
    radius       blur radius per level; -1 means ceil(3 sigma).
    fovea        (gaze_x, gaze_y, r_inner, r_outer) or None: see foveate().
    """
    num_levels: int = 4
    level_enable: int = 0xF
    depth_ratio: float = 0.05
    normal_cos: float = float(np.float32(math.cos(math.radians(25.0))))
    sigma2: tuple = (0.924, 1.848, 3.696, 0.0)
    weight: tuple = (100.0, 50.0, 20.0, 1.0)
    radius: tuple = (-1, -1, -1, -1)
    fovea: tuple = None

    def enabled(self):
        return [i for i in range(1, self.num_levels + 1) if (self.level_enable >> (i - 1)) & 1]


def level_dims(width: int, height: int, level: int):
    s = 1 << (level - 1)
    return width // s, height // s


def _valid(z):
    # reading: a pixel is geometry iff its linear depth is finite and > 0;
    # anything else is background (the paper does not discuss background).
    return np.isfinite(z) & (z > 0)


# --------------------------------------------------------------------------
# Sec. 3.1: edge image
# --------------------------------------------------------------------------
def edge_image(depth, normal, depth_ratio, normal_cos, dtype=np.float32):
    """E[H][W] in {0, 1} (uint8).

    Sec. 3.1 finds the geometry edges by numerically differentiating the
    G-buffer: first derivative of the normal in x and y, second derivative of
    the depth.  Readings (thresholds are not printed in the paper):

    * depth: along each axis with both neighbours inside the image,
      |(z[-1] + z[+1]) - 2 z| > t_d * z  (relative second difference);
    * normal: some in-image 4-neighbour q has dot(n_p, n_q) < c_n, with
      dot = ((nx nx') + (ny ny')) + (nz nz');
    * strict inequalities; the second difference is skipped along an axis at
      the image border; background pixels are never edges, geometry next to
      background always is.
    """
    z = depth.astype(dtype)
    n = normal.astype(dtype)
    td = dtype(depth_ratio)
    cn = dtype(normal_cos)
    H, W = z.shape
    valid = _valid(z)
    E = np.zeros((H, W), dtype=bool)
    with np.errstate(invalid="ignore", over="ignore"):
        two = dtype(2.0)
        thr = td * z
        # horizontal second difference, interior columns
        sx = np.zeros((H, W), bool)
        if W >= 3:
            d2 = np.abs((z[:, :-2] + z[:, 2:]) - two * z[:, 1:-1])
            sx[:, 1:-1] = d2 > thr[:, 1:-1]
        sy = np.zeros((H, W), bool)
        if H >= 3:
            d2 = np.abs((z[:-2, :] + z[2:, :]) - two * z[1:-1, :])
            sy[1:-1, :] = d2 > thr[1:-1, :]

        def dot(a, b):
            return ((a[0] * b[0]) + (a[1] * b[1])) + (a[2] * b[2])

        nedge = np.zeros((H, W), bool)
        bgnb = np.zeros((H, W), bool)
        # left/right neighbours
        if W >= 2:
            d = dot(n[:, :, :-1], n[:, :, 1:]) < cn   # pair (x, x+1)
            nedge[:, :-1] |= d
            nedge[:, 1:] |= d
            bgnb[:, :-1] |= ~valid[:, 1:]
            bgnb[:, 1:] |= ~valid[:, :-1]
        if H >= 2:
            d = dot(n[:, :-1, :], n[:, 1:, :]) < cn   # pair (y, y+1)
            nedge[:-1, :] |= d
            nedge[1:, :] |= d
            bgnb[:-1, :] |= ~valid[1:, :]
            bgnb[1:, :] |= ~valid[:-1, :]
        E = bgnb | sx | sy | nedge
    E &= valid
    return E.astype(np.uint8)


# --------------------------------------------------------------------------
# Sec. 3.1: downsampling of the mask to each sub-image resolution
# --------------------------------------------------------------------------
def foveate(E, fovea):
    """Sec. 6 (foveated rendering: the mask modulated by an importance mask
    from an eye tracker) with Sec. 3.1's combination of masks by minimum and
    maximum.  Reading: the importance mask of a gaze point g is 1 within
    r_inner of g (full resolution there), 0 beyond r_outer (coarsest level
    there) and leaves the edges alone in between:
        E' = max(min(E, [d2 <= r_outer^2]), [d2 <= r_inner^2]),
    d2 = dx^2 + dy^2 from the pixel centre, all in FP32."""
    if fovea is None:
        return E
    gx, gy, ri, ro = (np.float32(v) for v in fovea)
    H, W = E.shape
    dx = (np.arange(W, dtype=np.float32) + np.float32(0.5)) - gx
    dy = (np.arange(H, dtype=np.float32) + np.float32(0.5)) - gy
    d2 = (dx * dx)[None, :] + (dy * dy)[:, None]
    outer = d2 <= ro * ro
    inner = d2 <= ri * ri
    return ((E.astype(bool) & outer) | inner).astype(np.uint8)


def or_pool(E, s):
    """E_i(x, y) = OR of E over the s x s full-resolution block of texel (x, y).

    reading: the paper says only "downsample"; OR (max) keeps every edge
    (Sec. 3.1 allows combining masks by maximum)."""
    if s == 1:
        return E.copy()
    H, W = E.shape
    return E.reshape(H // s, s, W // s, s).max(axis=(1, 3)).astype(np.uint8)


# --------------------------------------------------------------------------
# Sec. 3.1 + Table 1: blur with variance sigma_i^2
# --------------------------------------------------------------------------
def blur_radius(sigma2, radius=-1):
    """reading: support radius ceil(3 sigma), computed in double."""
    if radius is not None and radius >= 0:
        return int(radius)
    s2 = float(np.float32(sigma2))
    if s2 <= 0.0:
        return 0
    return int(math.ceil(3.0 * math.sqrt(s2)))


def gaussian_weights(sigma2, radius=-1):
    """Normalised 1-D Gaussian taps g[k], k = -r..r, as float32.

    g[k] = float32(exp(-k^2 / (2 sigma^2)) / sum_j exp(-j^2 / (2 sigma^2))),
    evaluated in double (math.exp), then rounded.  sigma^2 = 0 gives [1]."""
    r = blur_radius(sigma2, radius)
    s2 = float(np.float32(sigma2))
    if s2 <= 0.0:
        w = [1.0 if k == 0 else 0.0 for k in range(-r, r + 1)]
        return np.array(w, np.float32)
    e = [math.exp(-(k * k) / (2.0 * s2)) for k in range(-r, r + 1)]
    tot = 0.0
    for v in e:
        tot += v
    return np.array([v / tot for v in e], np.float32)


def _shift(a, k, axis):
    """b[..., p, ...] = a[..., p + k, ...], zero outside (zero padding)."""
    out = np.zeros_like(a)
    n = a.shape[axis]
    if abs(k) >= n:
        return out
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if k >= 0:
        src[axis] = slice(k, n)
        dst[axis] = slice(0, n - k)
    else:
        src[axis] = slice(0, n + k)
        dst[axis] = slice(-k, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


def blur(Ei, g, dtype=np.float32):
    """Separable blur, horizontal then vertical, taps in ascending k.

    h(x, y) = sum_k g[k] * E(x + k, y), accumulator starting at +0, one
    rounding per product and per sum; out-of-image taps are 0.
    a(x, y) = sum_k g[k] * h(x, y + k) likewise."""
    g = g.astype(dtype)
    r = (len(g) - 1) // 2
    e = Ei.astype(dtype)
    h = np.zeros_like(e)
    for k in range(-r, r + 1):
        h = h + g[k + r] * _shift(e, k, 1)
    a = np.zeros_like(e)
    for k in range(-r, r + 1):
        a = a + g[k + r] * _shift(h, k, 0)
    return a


# --------------------------------------------------------------------------
# the pyramid
# --------------------------------------------------------------------------
@dataclass
class Pyramid:
    levels: list                  # enabled levels, ascending (1-based)
    E: np.ndarray                 # full-res edge image (after any extra edges)
    Ei: dict = field(default_factory=dict)      # level -> OR-pooled edges
    alpha: dict = field(default_factory=dict)   # level (< L) -> blurred mask a_i
    stencil: dict = field(default_factory=dict) # level -> S_i (uint8); S_L == 1
    level_map: np.ndarray = None  # full-res owner level (uint8, 1-based)
    worklist: dict = field(default_factory=dict)  # level (< L) -> uint32 indices
    radius: dict = field(default_factory=dict)
    weights: dict = field(default_factory=dict)


def build_pyramid(E, mp: MaskParams, dtype=np.float32) -> Pyramid:
    """From the full-resolution edge image to the nested stencils.

    Sec. 3.1: downsample the mask to every sub-image resolution, blur it with
    the level's variance (Table 1), and keep the levels inclusive: every
    higher-resolution area is contained in all lower ones and the lowest
    level covers the whole image.  Sec. 4.1: stencil = blurred mask > 0.
    """
    H, W = E.shape
    levels = mp.enabled()
    L = levels[-1]
    pyr = Pyramid(levels=levels, E=E)
    for i in levels:
        s = 1 << (i - 1)
        pyr.Ei[i] = or_pool(E, s)
    for i in levels:
        Wi, Hi = level_dims(W, H, i)
        if i == L:
            pyr.stencil[i] = np.ones((Hi, Wi), np.uint8)
            continue
        r = blur_radius(mp.sigma2[i - 1], mp.radius[i - 1])
        g = gaussian_weights(mp.sigma2[i - 1], mp.radius[i - 1])
        a = blur(pyr.Ei[i], g, dtype)
        pyr.alpha[i] = a
        pyr.radius[i] = r
        pyr.weights[i] = g
        pyr.stencil[i] = (a > 0).astype(np.uint8)
    # nesting: for consecutive enabled levels i < j, every texel of level j
    # whose footprint holds a level-i stencil texel is in S_j as well.
    for a_, b_ in zip(levels[:-1], levels[1:]):
        if b_ == L:
            break
        k = 1 << (b_ - a_)
        pyr.stencil[b_] = pyr.stencil[b_] | or_pool(pyr.stencil[a_], k)
    # owner-level partition: the finest enabled level whose stencil covers p.
    lm = np.zeros((H, W), np.uint8)
    for i in reversed(levels):
        s = 1 << (i - 1)
        up = np.repeat(np.repeat(pyr.stencil[i], s, axis=0), s, axis=1)
        lm = np.where(up.astype(bool), np.uint8(i), lm)
    pyr.level_map = lm
    pyr.worklist = work_lists(pyr)
    return pyr


def work_lists(pyr: Pyramid):
    """Row-major ascending linear indices y * W_i + x of the stencil texels of
    every enabled level below the coarsest (the coarsest is dense).

    reading: the set is what Sec. 4.1's stencil test lets through; the order
    is fixed to row-major ascending so lists compare exactly."""
    out = {}
    L = pyr.levels[-1]
    for i in pyr.levels:
        if i == L:
            continue
        out[i] = np.flatnonzero(pyr.stencil[i]).astype(np.uint32)
    return out


# --------------------------------------------------------------------------
# G-buffer of a sub-image
# --------------------------------------------------------------------------
def level_sample(plane, level):
    """Point sample of a full-resolution plane (last two axes H, W) for level i:
    v_i(x, y) = v(s x + s/2, s y + s/2), s = 2**(i-1); level 1 is the plane.

    reading: the paper renders each sub-image "in lower resolution" without
    saying how the G-buffer is reduced; this takes the G-buffer sample nearest
    to the texel centre (lower-right of the four central samples)."""
    s = 1 << (level - 1)
    if s == 1:
        return plane
    h = s // 2
    return np.ascontiguousarray(plane[..., h::s, h::s])
