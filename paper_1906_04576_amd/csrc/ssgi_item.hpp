// One-bounce screen-space indirect light (Sec. 2.4, after Ritschel et al.
// 2009).  The SSAO sampling and occlusion test are reused; every occluding
// sample adds the directly lit colour of the texel it hit, weighted as a
// small patch sending light to the receiver:
//   v = X_t - P, dd = dot(v, v), dist2 = max(dd, (0.1 r)^2),
//   v_hat = v / sqrt(dd), g = (max(0, n.v_hat) max(0, -n_t.v_hat)) / dist2,
//   acc += C_t g;  out = acc (r^2 / S).
#pragma once
#include "eval_common.hpp"

namespace mr {

// depth gathers in flight per sample group of the naive pass (measured)
constexpr int kSsgiGroup = 8;

// one item (a listed texel, or a texel of a dense level)
template <typename NT, typename CT, bool AL, typename KP>
__device__ __forceinline__ void ssgi_item(const SsgiArgs& a, const ItemMap& m, unsigned item, KP K,
                                          const float* eg) {
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const CT* col = static_cast<const CT*>(a.c.color);
    const long long plane = a.c.plane;
    const float r = a.r, b = a.b;
    const int S = a.S;
    const float rmin = 0.1f * r;
    const float rmin2 = rmin * rmin;
    const float scale = (r * r) / (float)S;
    {
        const int j = item_level(m, item);
        const EvalLevel& L = a.c.lv[j];
        const unsigned local = item_local(m, item, j);
        if (local == ~0u) return;  // padding of the level's item range
        const unsigned t = L.list ? L.list[local] : local;
        if (t >= L.dense_n) return;  // malformed list entry
        const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
        if (AL && L.ac) L.ac[local] = alpha_dispatch(L, eg + j * kEgStride, x, y);
        const float z = L.z[(unsigned)y * L.zpy + (unsigned)x * L.zpx];
        float acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
        if (valid_depth(z)) {
            const long long g = L.goff + (long long)y * L.gpy + (long long)x * L.gpx;
            const float nx = ld(nrm, g), ny = ld(nrm, plane + g), nz = ld(nrm, 2 * plane + g);
            float px, py, pz;
            view_pos(x, y, z, L.f, L.cx, L.cy, px, py, pz);
            float tx, ty, tz, bx, by, bz;
            onb(nx, ny, nz, tx, ty, tz, bx, by, bz);
            const float rtx = r * tx, rty = r * ty, rtz = r * tz;
            const float rbx = r * bx, rby = r * by, rbz = r * bz;
            const float rnx = r * nx, rny = r * ny, rnz = r * nz;
            if constexpr (AL) {
                // multi-resolution launches: one pass over the samples (their
                // texels sit near edges, where many samples occlude)
                const float Wf = (float)L.W, Hf = (float)L.H;
                for (int s = 0; s < S; ++s) {
                    const float kx = K[3 * s], ky = K[3 * s + 1], kz = K[3 * s + 2];
                    const float qx = ((px + kx * rtx) + ky * rbx) + kz * rnx;
                    const float qy = ((py + kx * rty) + ky * rby) + kz * rny;
                    const float qz = ((pz + kx * rtz) + ky * rbz) + kz * rnz;
                    const float d = -qz;
                    if (!(d > 0.0f)) continue;
                    const float inv = recip_pos(d);  // = 1.0f / d (d > 0)
                    const float u = L.cx + (qx * inv) * L.f;
                    const float v = L.cy - (qy * inv) * L.f;
                    // 0 <= u < W and 0 <= v < H as unsigned compares of the
                    // bit patterns: exact, as u = cx + t and v = cy - t' are
                    // never -0 (cx, cy > 0)
                    if (!((__float_as_uint(u) < __float_as_uint(Wf)) & (__float_as_uint(v) < __float_as_uint(Hf))))
                        continue;
                    const int sx = (int)u, sy = (int)v;  // u, v >= 0: truncation is floor
                    const float zs = L.z[(unsigned)sy * L.zpy + (unsigned)sx * L.zpx];
                    if (!valid_depth(zs)) continue;
                    if (!(zs < d - (b * d) && fabsf(z - zs) < r)) continue;
                    float hx, hy, hz;
                    view_pos(sx, sy, zs, L.f, L.cx, L.cy, hx, hy, hz);
                    const float vx = hx - px, vy = hy - py, vz = hz - pz;
                    const float dd = ((vx * vx) + (vy * vy)) + (vz * vz);
                    if (!(dd > 0.0f)) continue;
                    const float dist2 = fmaxf(dd, rmin2);
                    const float il = rsqrt_pos(dd);  // = 1.0f / sqrtf(dd) (dd > 0)
                    const float vhx = vx * il, vhy = vy * il, vhz = vz * il;
                    const long long gt = L.goff + (long long)sy * L.gpy + (long long)sx * L.gpx;
                    const float mx = ld(nrm, gt), my = ld(nrm, plane + gt), mz = ld(nrm, 2 * plane + gt);
                    const float cr = fmaxf(0.0f, ((nx * vhx) + (ny * vhy)) + (nz * vhz));
                    const float ce = fmaxf(0.0f, -(((mx * vhx) + (my * vhy)) + (mz * vhz)));
                    const float w = (cr * ce) / dist2;
                    acc0 = acc0 + ld(col, gt) * w;
                    acc1 = acc1 + ld(col, plane + gt) * w;
                    acc2 = acc2 + ld(col, 2 * plane + gt) * w;
                }
            } else {
                const float Wf = (float)L.W, Hf = (float)L.H;
                // sample s: its point, depth d, and the texel it projects to
                auto project = [&](int s, float& d, bool& on, int& sx, int& sy) {
                    const float kx = K[3 * s], ky = K[3 * s + 1], kz = K[3 * s + 2];
                    const float qx = ((px + kx * rtx) + ky * rbx) + kz * rnx;
                    const float qy = ((py + kx * rty) + ky * rby) + kz * rny;
                    const float qz = ((pz + kx * rtz) + ky * rbz) + kz * rnz;
                    d = -qz;
                    const float inv = recip_pos(d);  // = 1.0f / d when d > 0 (else unused)
                    const float u = L.cx + (qx * inv) * L.f;
                    const float v = L.cy - (qy * inv) * L.f;
                    on = (d > 0.0f) & (u >= 0.0f) & (u < Wf) & (v >= 0.0f) & (v < Hf);
                    sx = (int)(on ? u : 0.0f);  // u, v >= 0 when on: truncation is floor
                    sy = (int)(on ? v : 0.0f);
                };
                // L is wave-uniform: the depth plane as a buffer resource
                const unsigned zpy = (unsigned)L.zpy, zpx = (unsigned)L.zpx;
                const __amdgpu_buffer_rsrc_t rz =
                    buf_rsrc(L.z, ((unsigned)(L.H - 1) * zpy + (unsigned)(L.W - 1) * zpx + 1u) * 4u);
                // a sample adds light iff it occludes: on screen, valid depth
                // z_s below the biased sample depth and within the radius
                auto occludes = [&](bool on, float d, float zs) {
                    return on & (zs > 0.0f) & (zs < d - (b * d)) & (fabsf(z - zs) < r);
                };
                // Per block of 32 samples: first which samples occlude (the
                // depth gathers of kSsgiGroup samples in flight together), then
                // the light of exactly those samples in sample order, so that
                // the sums are the ones of one pass over the samples.
                for (int s0 = 0; s0 < S; s0 += 32) {
                    const int ns = min(32, S - s0);
                    unsigned hits = 0u;
                    int k0 = 0;
                    for (; k0 + kSsgiGroup <= ns; k0 += kSsgiGroup) {
                        float d[kSsgiGroup], zs[kSsgiGroup];
                        bool on[kSsgiGroup];
                        unsigned off[kSsgiGroup];
    #pragma unroll
                        for (int k = 0; k < kSsgiGroup; ++k) {
                            int sx, sy;
                            project(s0 + k0 + k, d[k], on[k], sx, sy);
                            off[k] = __umul24((unsigned)sy, zpy) + __umul24((unsigned)sx, zpx);
                            __builtin_amdgcn_sched_barrier(0);
                        }
    #pragma unroll
                        for (int k = 0; k < kSsgiGroup; ++k) zs[k] = buf_f1(rz, off[k] * 4u);
    #pragma unroll
                        for (int k = 0; k < kSsgiGroup; ++k) hits |= occludes(on[k], d[k], zs[k]) ? 1u << (k0 + k) : 0u;
                    }
                    for (; k0 < ns; ++k0) {
                        float d;
                        bool on;
                        int sx, sy;
                        project(s0 + k0, d, on, sx, sy);
                        const float zs = buf_f1(rz, (__umul24((unsigned)sy, zpy) + __umul24((unsigned)sx, zpx)) * 4u);
                        hits |= occludes(on, d, zs) ? 1u << k0 : 0u;
                    }
                    while (hits) {
                        const int k = __builtin_ctz(hits);
                        hits &= hits - 1;
                        float d;
                        bool on;
                        int sx, sy;
                        project(s0 + k, d, on, sx, sy);
                        const float zs = L.z[(unsigned)sy * zpy + (unsigned)sx * zpx];
                        float hx, hy, hz;
                        view_pos(sx, sy, zs, L.f, L.cx, L.cy, hx, hy, hz);
                        const float vx = hx - px, vy = hy - py, vz = hz - pz;
                        const float dd = ((vx * vx) + (vy * vy)) + (vz * vz);
                        if (!(dd > 0.0f)) continue;
                        const float dist2 = fmaxf(dd, rmin2);
                        const float il = rsqrt_pos(dd);  // = 1.0f / sqrtf(dd) (dd > 0)
                        const float vhx = vx * il, vhy = vy * il, vhz = vz * il;
                        const long long gt = L.goff + (long long)sy * L.gpy + (long long)sx * L.gpx;
                        const float mx = ld(nrm, gt), my = ld(nrm, plane + gt), mz = ld(nrm, 2 * plane + gt);
                        const float cr = fmaxf(0.0f, ((nx * vhx) + (ny * vhy)) + (nz * vhz));
                        const float ce = fmaxf(0.0f, -(((mx * vhx) + (my * vhy)) + (mz * vhz)));
                        const float w = (cr * ce) / dist2;
                        acc0 = acc0 + ld(col, gt) * w;
                        acc1 = acc1 + ld(col, plane + gt) * w;
                        acc2 = acc2 + ld(col, 2 * plane + gt) * w;
                    }
                }
            }
        }
        const long long o = L.compact ? (long long)local : (long long)y * L.W + x;
        store_out(L, (unsigned)o, acc0 * scale);
        store_out(L, (unsigned)L.out_plane + (unsigned)o, acc1 * scale);
        store_out(L, 2u * (unsigned)L.out_plane + (unsigned)o, acc2 * scale);
    }
}

template <typename NT, typename CT, bool AL, typename KP>
__device__ __forceinline__ void ssgi_items(const SsgiArgs& a, KP K, const float* eg) {
    const ItemMap m = make_item_map(a.c);
    const unsigned total = item_total(m);
    const ChunkRange cr = chunk_range((total + 255) / 256);
    for (unsigned c = cr.first; c < cr.end; c += cr.step) {
        const unsigned item = c * 256u + threadIdx.x;
        if (item < total) ssgi_item<NT, CT, AL>(a, m, item, K, eg);
    }
}

// per block: blur taps (AL) and, KLDS, the samples (S <= kLdsSamples)
template <bool AL, bool KLDS>
__device__ __forceinline__ void ssgi_stage(const SsgiArgs& a, float* ks, float* eg) {
    if (AL) stage_taps(a.c, eg);
    if (KLDS)
        for (int i = threadIdx.x; i < 3 * a.S; i += 256) ks[i] = a.kernel[i];
    __syncthreads();
}

}  // namespace mr
