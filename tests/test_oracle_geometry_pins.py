"""Pins of the two estimator parts whose values depend on scene geometry
(Sec. 2.4): the SSGI transfer term and the view-to-light transform of the
soft-shadow estimator.  The expected values come from the scene itself
(planes and boxes intersected in float64 world space), not from the oracle's
view-space code.

SSGI: a floor and a back wall meet in a crease.  A receiver on the floor
next to the wall gathers light from chosen wall texels, and a receiver on the
wall gathers light from chosen floor texels.  Between two perpendicular
planes the transfer term of one hit reduces to

    g = (h_e * h_r) / (|v|^2 * max(|v|^2, (0.1 r)^2))

where h_e is the height of the emitting point above the receiver's plane and
h_r the distance of the receiver from the emitter's plane (both cosines are
"distance to the other plane over |v|").  The test compares the oracle's
r^2/S-scaled sum of C_t g with this closed form.

Soft shadows: the light sits away from the camera, rotated and translated.
The oracle's light coordinates (d_r, su, sv) are compared with a direct
projection of known world points through the light's own axes, and its
one-sample shadow bits with a segment-versus-box test towards the light.

Either test fails if the sign of one cosine flips, the r^2/S factor is
dropped, the distance clamp is wrong, the transform is transposed or the
map's v axis is flipped.
"""
import math

import numpy as np
import pytest

import oracle
import scenegen

F64 = np.float64
F32 = np.float32

# ---------------------------------------------------------------------------
# SSGI: floor y = -h and back wall z = -D in view space, camera at the origin
# ---------------------------------------------------------------------------
W, H, FOCAL = 96, 64, 80.0
CX, CY = 0.5 * W, 0.5 * H
FLOOR_H = 0.5
RADIUS = 2.0
ROW_R = 50                                       # receiver row on the floor
T_R = FLOOR_H * FOCAL / ((ROW_R + 0.5) - CY)     # its depth (first floor row)
WALL_D = T_R + 0.12                              # wall 0.12 behind it


def _ray(x, y):
    return np.array([(x + 0.5 - CX) / FOCAL, (CY - (y + 0.5)) / FOCAL, -1.0], F64)


def _hit(x, y):
    """Nearest of floor and wall along the centre ray of pixel (x, y):
    (depth, normal, 'floor' | 'wall')."""
    d = _ray(x, y)
    t_wall = WALL_D
    t_floor = -FLOOR_H / d[1] if d[1] < 0 else math.inf
    if t_floor < t_wall:
        return t_floor, np.array([0.0, 1.0, 0.0]), "floor"
    return t_wall, np.array([0.0, 0.0, 1.0]), "wall"


def _corner_gbuffer():
    depth = np.empty((H, W), F64)
    normal = np.empty((3, H, W), F64)
    kind = np.empty((H, W), object)
    colour = np.empty((3, H, W), F64)
    for y in range(H):
        for x in range(W):
            t, n, k = _hit(x, y)
            depth[y, x] = t
            normal[:, y, x] = n
            kind[y, x] = k
            # a distinct colour per texel (exact in FP16), so a wrong texel shows
            colour[:, y, x] = ((x % 16) / 16.0, (y % 16) / 16.0, 0.25 + ((x + y) % 4) / 8.0)
    return depth, normal, kind, colour


def _world(x, y, depth):
    return _ray(x, y) * depth


# Duff et al. tangent frames of the two plane normals (the estimator's basis)
FRAME_FLOOR = (np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, -1.0]), np.array([0.0, 1.0, 0.0]))
FRAME_WALL = (np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0]))


def _sample_towards(P, frame, target, scale):
    """Kernel entry whose sample point lies on the camera ray of `target`
    (a world point), `scale` times as far from the camera: it projects to the
    centre of target's texel and lies behind the surface there."""
    Q = target * scale
    T, B, N = frame
    return np.array([np.dot(Q - P, T), np.dot(Q - P, B), np.dot(Q - P, N)]) / RADIUS


def _design(depth, kind):
    """Two receivers with hand-placed samples.  Returns per receiver
    (x, y, kernel f32[S][3], list of hit texels)."""
    out = []
    # receiver 1: floor texel right in front of the wall
    xr, yr = 41, ROW_R
    assert kind[yr, xr] == "floor" and kind[yr - 1, xr] == "wall"
    P = _world(xr, yr, depth[yr, xr])
    hits = [(41, 45), (44, 40), (55, 30), (36, 20), (47, 48)]  # wall texels
    for tx, ty in hits:
        assert kind[ty, tx] == "wall"
    ks = [_sample_towards(P, FRAME_FLOOR, _world(tx, ty, depth[ty, tx]), 1.04) for tx, ty in hits]
    ks += [
        np.array([0.0, 0.0, 0.3]),     # straight up: lands on the wall in front of its depth
        np.array([0.9, 0.0, 0.05]),    # far to the right: off screen
        np.array([0.0, -1.3, 0.1]),    # towards the camera past it: d <= 0
    ]
    out.append((xr, yr, np.array(ks), hits))
    # receiver 2: wall texel above the crease, lit by floor texels in front
    xr, yr = 60, 40
    assert kind[yr, xr] == "wall"
    P = _world(xr, yr, depth[yr, xr])
    hits = [(60, 50), (66, 51), (52, 53), (71, 56)]
    for tx, ty in hits:
        assert kind[ty, tx] == "floor"
    ks = [_sample_towards(P, FRAME_WALL, _world(tx, ty, depth[ty, tx]), 1.03) for tx, ty in hits]
    ks += [np.array([0.1, 0.2, 0.05])]  # in front of the wall, above the floor: free
    out.append((xr, yr, np.array(ks), hits))
    return out


def _closed_form(P, kind_r, hits, depth, colour, S):
    """(r^2 / S) * sum over hits of C_t (h_e h_r) / (|v|^2 max(|v|^2, (0.1 r)^2))."""
    acc = np.zeros(3)
    for tx, ty in hits:
        X = _world(tx, ty, depth[ty, tx])
        v2 = float(np.sum((X - P) ** 2))
        if kind_r == "floor":   # emitter on the wall
            h_e = X[1] + FLOOR_H          # emitter height above the floor
            h_r = P[2] + WALL_D           # receiver distance from the wall plane
        else:                   # receiver on the wall, emitter on the floor
            h_e = X[2] + WALL_D           # emitter distance in front of the wall
            h_r = P[1] + FLOOR_H          # receiver height above the floor
        assert h_e > 0 and h_r > 0
        acc += colour[:, ty, tx] * (h_e * h_r) / (v2 * max(v2, (0.1 * RADIUS) ** 2))
    return acc * (RADIUS * RADIUS / S)


def test_ssgi_transfer_term_closed_form_between_perpendicular_planes():
    depth, normal, kind, colour = _corner_gbuffer()
    col16 = colour.astype(np.float16)
    assert np.array_equal(col16.astype(F64), colour)
    clamped = 0
    for xr, yr, K64, hits in _design(depth, kind):
        K = K64.astype(F32)
        S = K.shape[0]
        P = _world(xr, yr, depth[yr, xr])
        exp = _closed_form(P, kind[yr, xr], hits, depth, colour, S)
        for tx, ty in hits:
            v2 = float(np.sum((_world(tx, ty, depth[ty, tx]) - P) ** 2))
            clamped += v2 < (0.1 * RADIUS) ** 2
        xs, ys = np.array([xr]), np.array([yr])
        p = oracle.SSGIParams(K, RADIUS, 0.02)
        got64 = oracle.ssgi_texels(depth, normal, colour, F64(FOCAL), 1, xs, ys, p, dtype=F64)[:, 0]
        np.testing.assert_allclose(got64, exp, rtol=1e-9, atol=0)
        # the FP32 estimator on the FP32-rounded G-buffer finds the same hits
        got32 = oracle.ssgi_texels(depth.astype(F32), normal.astype(F32), col16, F32(FOCAL), 1, xs, ys,
                                   p, dtype=F32)[:, 0]
        np.testing.assert_allclose(got32.astype(F64), exp, rtol=2e-4, atol=0)
        # and the same samples count as occluders for SSAO
        occ = oracle.ssao_texels(depth, normal, F64(FOCAL), 1, xs, ys,
                                 oracle.SSAOParams(K, RADIUS, 0.02), dtype=F64)[0]
        assert occ == len(hits) / S
    assert clamped >= 1, "one hit must lie inside the distance clamp"


def test_ssgi_transfer_is_zero_between_coplanar_points():
    """A receiver on the wall gets no light from other wall texels: both
    cosines are 0 for points in one plane, although the samples (pushed
    behind those texels) pass the SSAO occlusion test."""
    depth, normal, kind, colour = _corner_gbuffer()
    xr, yr = 30, 20
    P = _world(xr, yr, depth[yr, xr])
    # samples pushed behind neighbouring wall texels
    ks = [_sample_towards(P, FRAME_WALL, _world(tx, ty, depth[ty, tx]), 1.04) for tx, ty in ((33, 22), (26, 18))]
    K = np.array(ks).astype(F32)
    p = oracle.SSGIParams(K, RADIUS, 0.02)
    got = oracle.ssgi_texels(depth, normal, colour, F64(FOCAL), 1, np.array([xr]), np.array([yr]), p, dtype=F64)
    occ = oracle.ssao_texels(depth, normal, F64(FOCAL), 1, np.array([xr]), np.array([yr]),
                             oracle.SSAOParams(K, RADIUS, 0.02), dtype=F64)[0]
    assert occ == 1.0
    assert (got == 0).all()


# ---------------------------------------------------------------------------
# soft shadows: a rotated, translated light
# ---------------------------------------------------------------------------
def _basis(eye, target):
    """Light axes from first principles: forward towards the target, right
    perpendicular to forward and world up, up completing the frame."""
    eye = np.asarray(eye, F64)
    fwd = np.asarray(target, F64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.array([-fwd[2], 0.0, fwd[0]])  # fwd x (0, 1, 0)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    return eye, right, up, fwd


def _view_to_light(cam_view, light):
    """3 x 4 affine map from camera view space to light view space
    (x right, y up, z backwards), composed through world space."""
    e_c = cam_view[0:3]
    rc = np.stack([cam_view[3:6], cam_view[6:9], cam_view[9:12]], axis=1)  # view -> world rotation
    e_l, right, up, fwd = light
    rl = np.stack([right, up, -fwd], axis=0)                                # world -> light rotation
    M = np.zeros((3, 4))
    M[:, :3] = rl @ rc
    M[:, 3] = rl @ (e_c - e_l)
    return M


def _to_view(cam_view, Xw):
    e_c = cam_view[0:3]
    d = Xw - e_c
    return d @ cam_view[3:6], d @ cam_view[6:9], d @ cam_view[9:12]


LIGHT_EYE = (-7.0, 11.0, 5.0)
LIGHT_AT = (1.5, 0.0, -2.0)


def test_light_coords_equal_direct_projection_through_the_light_axes():
    cam = scenegen.orbit_view(3)
    light = _basis(LIGHT_EYE, LIGHT_AT)
    M = _view_to_light(cam, light)
    size, fL = 1024, 700.0
    rng = np.random.default_rng(5)
    Xw = rng.uniform([-6, 0, -6], [6, 3, 6], size=(200, 3))
    Px, Py, Pz = _to_view(cam, Xw)
    p = oracle.ShadowParams(np.zeros((size, size), F64), M, fL, 0.5, 1.0, 0.05,
                            np.zeros((16, 2)), np.zeros((32, 2)))
    dr, su, sv, inside = oracle.light_coords(Px, Py, Pz, p, F64)
    e_l, right, up, fwd = light
    rel = Xw - e_l
    depth = rel @ fwd                              # distance along the light's axis
    exp_su = 0.5 * size + fL * (rel @ right) / depth
    exp_sv = 0.5 * size - fL * (rel @ up) / depth  # map row 0 at the top
    np.testing.assert_allclose(dr, depth, rtol=1e-12)
    np.testing.assert_allclose(su, exp_su, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(sv, exp_sv, rtol=1e-12, atol=1e-9)
    exp_in = (depth > 0) & (exp_su >= 0) & (exp_su < size) & (exp_sv >= 0) & (exp_sv < size)
    assert np.array_equal(inside, exp_in)
    assert exp_in.sum() > 150 and not exp_in.all()
    # the same points through the transposed rotation land far away
    Mt = M.copy()
    Mt[:, :3] = M[:, :3].T
    pt = oracle.ShadowParams(p.shadow_map, Mt, fL, 0.5, 1.0, 0.05, p.blocker_disk, p.pcf_disk)
    _, su_t, sv_t, _ = oracle.light_coords(Px, Py, Pz, pt, F64)
    assert np.median(np.hypot(su_t - exp_su, sv_t - exp_sv)) > 20


def _render_light_map(scene, light, size, fov_deg):
    """Linear light depth map of `scene` through the FP64 ray caster, with the
    light's axes given as the caster's view basis (eye, right, up, back)."""
    e_l, right, up, fwd = light
    lv = np.concatenate([e_l, right, up, -fwd])
    lib = scenegen._load()
    sm = np.empty((size, size), F32)
    boxes = np.ascontiguousarray(scene.boxes, F64)
    spheres = np.zeros((1, 4))
    focal = scenegen.focal_px(size, fov_deg)
    lib.rc_depthmap(scenegen._ptr(np.ascontiguousarray(lv), scenegen.ctypes.c_double), size, float(focal),
                    scenegen._ptr(boxes, scenegen.ctypes.c_double), len(scene.boxes),
                    scenegen._ptr(spheres, scenegen.ctypes.c_double), 0, scenegen._ptr(sm, scenegen.ctypes.c_float))
    return sm, focal


def _segment_hits_box(P, L, boxes):
    """Smallest parameter t in (0, 1) where the segment P -> L enters a box
    (inf if none); slab test, all boxes at once."""
    d = L - P
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (boxes[:, :3] - P) / d
        t2 = (boxes[:, 3:] - P) / d
    tmin = np.nanmax(np.minimum(t1, t2), axis=1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=1)
    ok = (tmin < tmax) & (tmax > 0) & (tmin > 0) & (tmin < 1)
    return float(tmin[ok].min()) if ok.any() else math.inf


def test_hard_shadow_bits_equal_segment_test_towards_the_light():
    scene = scenegen.make_scene(7, 14, 0)
    cam = scenegen.orbit_view(5)
    Wg, Hg = 128, 80
    gb = scenegen.render_gbuffer(scene, cam, Wg, Hg)
    light = _basis(LIGHT_EYE, LIGHT_AT)
    size, bias = 1024, 0.05
    sm, fL = _render_light_map(scene, light, size, 70.0)
    M = _view_to_light(cam, light)
    p = oracle.ShadowParams(sm, M.astype(F32), fL, F32(0.5), F32(1.0), F32(bias),
                            scenegen.disk_samples(16, 11), scenegen.disk_samples(32, 12))
    hard = oracle.hard_shadow(gb.depth, gb.focal, 1, p)
    e_l, right, up, fwd = light
    f = float(gb.focal)
    checked = shadowed = 0
    for y in range(Hg):
        for x in range(Wg):
            if gb.objid[y, x] != 0:  # receivers on the ground
                continue
            z = float(gb.depth[y, x])
            pv = np.array([(x + 0.5 - 0.5 * Wg) / f * z, (0.5 * Hg - (y + 0.5)) / f * z, -z])
            Xw = cam[0:3] + pv[0] * cam[3:6] + pv[1] * cam[6:9] + pv[2] * cam[9:12]
            rel = Xw - e_l
            dr = rel @ fwd
            su = 0.5 * size + fL * (rel @ right) / dr
            sv = 0.5 * size - fL * (rel @ up) / dr
            if not (4 <= su < size - 4 and 4 <= sv < size - 4):
                continue
            # light depth of the bare ground along the centre ray of the map
            # texel: where it differs from d_r by more than half the bias, a
            # constant bias cannot separate the receiver from its own surface
            # (shadow acne, a property of the estimator, not of the transform)
            dl = fwd + ((math.floor(su) + 0.5 - 0.5 * size) / fL) * right - ((math.floor(sv) + 0.5 - 0.5 * size) / fL) * up
            if abs(-e_l[1] / dl[1] - dr) > 0.5 * bias:
                continue
            # the geometric answer, and the same at points 2.5 map texels away
            # in the light's image plane: skip pixels near a shadow boundary
            step = 2.5 * dr / fL
            states = []
            for ox, oy in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)):
                q = Xw + step * (ox * right + oy * up)
                t = _segment_hits_box(q, e_l, scene.boxes)
                states.append(t)
            sh = [t < math.inf for t in states]
            if len(set(sh)) != 1:
                continue
            if sh[0] and min(states) * dr < 0.3:  # contact shadow: blocker depth near the receiver's
                continue
            assert bool(hard[y, x]) == sh[0], (x, y)
            checked += 1
            shadowed += sh[0]
    n_ground = int((gb.objid == 0).sum())
    assert checked > 0.5 * n_ground
    assert shadowed > 50 and checked - shadowed > 50
