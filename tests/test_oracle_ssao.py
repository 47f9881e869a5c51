"""Pins of the oracle's SSAO estimator: a fronto-parallel plane is unoccluded
exactly; the ground-only scene is unoccluded under the chosen bias; on a
two-plane step the occluded count of every texel equals a float64 count of
the projected samples that land on the nearer plane (pins projection, tangent
frame orientation, level camera and counting)."""
import math

import numpy as np
import pytest

import oracle
import scenegen

F32 = np.float32


def planes(H, W, z=10.0):
    d = np.full((H, W), z, F32)
    n = np.zeros((3, H, W), F32)
    n[2] = 1.0
    return d, n


def test_duff_frame_is_orthonormal():
    rng = np.random.default_rng(0)
    v = rng.normal(size=(3, 1000))
    v /= np.linalg.norm(v, axis=0)
    v = v.astype(np.float64)
    T, B = oracle.ssao.tangent_frame(v[0], v[1], v[2], np.float64)
    T, B = np.array(T), np.array(B)
    assert np.allclose((T * T).sum(0), 1) and np.allclose((B * B).sum(0), 1)
    assert np.allclose((T * B).sum(0), 0, atol=1e-12)
    assert np.allclose((T * v).sum(0), 0, atol=1e-12) and np.allclose((B * v).sum(0), 0, atol=1e-12)
    # right-handed: T x B = n
    assert np.allclose(np.cross(T.T, B.T).T, v, atol=1e-12)


@pytest.mark.parametrize("level", [1, 2, 3])
def test_fronto_parallel_plane_unoccluded(level):
    d, n = planes(24, 40)
    p = oracle.SSAOParams(scenegen.ssao_kernel(32), 1.0, 0.02)
    out = oracle.ssao_level(d, n, F32(30.0), level, p)
    assert (out == 0).all()


@pytest.mark.parametrize("W,H,S", [(256, 256, 16), (640, 360, 32)])
def test_ground_only_scene_unoccluded(W, H, S):
    s = scenegen.make_scene(1, 0, 0)
    for k in (0, 5):
        gb = scenegen.render_gbuffer(s, scenegen.orbit_view(k), W, H)
        p = oracle.SSAOParams(scenegen.ssao_kernel(S), 0.5 if S == 16 else 1.0, 0.02)
        for level in (1, 2, 3):
            zi = oracle.level_sample(gb.depth, level)
            ni = oracle.level_sample(gb.normal, level)
            assert (oracle.ssao_level(zi, ni, gb.focal, level, p) == 0).all()


def step_expectation(W, H, f, z_far, z_near, near_mask_fn, kernel, r, b, xs, ys):
    """float64 count of samples landing on the nearer plane; None if a
    decision is within 1e-6 of its boundary."""
    cx, cy = W / 2, H / 2
    out = []
    for x, y in zip(xs, ys):
        X = (x + 0.5 - cx) / f
        Y = (cy - (y + 0.5)) / f
        P = np.array([X * z_far, Y * z_far, -z_far])
        cnt = 0
        amb = False
        for kx, ky, kz in kernel.astype(np.float64):
            Q = P + r * np.array([kx, ky, kz])
            dq = -Q[2]
            u = cx + Q[0] / dq * f
            v = cy - Q[1] / dq * f
            if min(abs(u - round(u)), abs(v - round(v))) < 1e-6 or abs(z_near - (dq - b * dq)) < 1e-6:
                amb = True
            if not (0 <= u < W and 0 <= v < H):
                continue
            if near_mask_fn(int(math.floor(u)), int(math.floor(v))) and z_near < dq - b * dq:
                cnt += 1
        out.append(None if amb else cnt)
    return out


@pytest.mark.parametrize("level", [1, 2, 3])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_two_plane_step_counts(level, axis):
    W, H, f = 128, 96, 160.0
    s = 1 << (level - 1)
    Wi, Hi, fi = W // s, H // s, f / s
    zf, zn = 10.0, 9.6
    d, n = planes(Hi, Wi, zf)
    if axis == "x":
        near = lambda tx, ty: tx < Wi // 2
        d[:, : Wi // 2] = zn
    else:
        near = lambda tx, ty: ty < Hi // 2
        d[: Hi // 2, :] = zn
    K = scenegen.ssao_kernel(32)
    r, b = 1.0, 0.005
    p = oracle.SSAOParams(K, r, b)
    out = oracle.ssao_level(d, n, F32(f), level, p)
    ys, xs = np.nonzero(d == zf)
    exp = step_expectation(Wi, Hi, fi, zf, zn, near, K, r, float(F32(b)), xs, ys)
    checked = 0
    for x, y, e in zip(xs, ys, exp):
        if e is None:
            continue
        assert out[y, x] * 32 == e, (x, y, out[y, x] * 32, e)
        checked += 1
    assert checked > 0.8 * len(xs)
    assert (out[d == zn] == 0).all()
    assert out.max() > 0


def test_values_are_multiples_of_one_over_S(scene256):
    s, gb = scene256
    p = oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02)
    out = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, p)
    assert np.array_equal(out * 16, np.round(out * 16))
    assert out.min() >= 0 and out.max() <= 1 and out.max() > 0


def test_background_gives_zero():
    d, n = planes(16, 16)
    d[4:8, 4:8] = np.inf
    p = oracle.SSAOParams(scenegen.ssao_kernel(16), 1.0, 0.02)
    out = oracle.ssao_plain(d, n, F32(20.0), p)
    assert (out[4:8, 4:8] == 0).all()


def test_fp64_twin_close_to_fp32(scene256):
    s, gb = scene256
    p = oracle.SSAOParams(scenegen.ssao_kernel(16), 0.5, 0.02)
    a = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, p)
    b = oracle.ssao_plain(gb.depth, gb.normal, gb.focal, p, np.float64)
    assert np.abs(a - b).mean() < 1e-3
