// Soft shadows (Sec. 2.4: shadow map after Williams 1978, percentage-closer
// filtering after Reeves et al. 1987, PCSS penumbra after Fernando 2005) and
// the one-sample shadow test whose differences add shadow edges to the mask
// (Sec. 3.1).
//
// Light coordinates: P_l = M P (3 x 4 affine, rows summed left to right),
// d_r = -P_l.z, su = c_L + (P_l.x / d_r) f_L, sv = c_L - (P_l.y / d_r) f_L,
// c_L = size / 2.  Outside the light frustum = lit.  Blocker search over a
// disk of half-width R_s = (l (d_r - n_L)) / (d_r n_L), l = f_L (w_L / 2);
// penumbra R_f = (l (d_r - d_b)) / (d_b d_r) from the mean blocker depth d_b;
// visibility = share of PCF taps that are not in front of d_r - bias.
#include "eval_common.hpp"

namespace mr {

struct LightCoord {
    float dr, su, sv;
    bool inside;
};

__device__ __forceinline__ LightCoord to_light(const float* M, int size, float fL, float px,
                                               float py, float pz) {
    const float lx = ((M[0] * px + M[1] * py) + M[2] * pz) + M[3];
    const float ly = ((M[4] * px + M[5] * py) + M[6] * pz) + M[7];
    const float lz = ((M[8] * px + M[9] * py) + M[10] * pz) + M[11];
    LightCoord c;
    const float cL = 0.5f * (float)size;
    c.dr = -lz;
    const float inv = 1.0f / c.dr;
    c.su = cL + (lx * inv) * fL;
    c.sv = cL - (ly * inv) * fL;
    const float sz = (float)size;
    c.inside = c.dr > 0.0f && c.su >= 0.0f && c.su < sz && c.sv >= 0.0f && c.sv < sz;
    return c;
}

__device__ __forceinline__ float sm_tap(const float* sm, int size, float su, float sv, float R,
                                        float ox, float oy) {
    const float hi = (float)(size - 1);
    const float fx = fminf(fmaxf(floorf(su + R * ox), 0.0f), hi);
    const float fy = fminf(fmaxf(floorf(sv + R * oy), 0.0f), hi);
    return sm[(long long)(int)fy * size + (int)fx];
}

__global__ __launch_bounds__(256) void k_hard(HardArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    const long long p = (long long)y * a.W + x;
    const float z = a.depth[p];
    uint8_t h = 0;
    if (valid_depth(z)) {
        float px, py, pz;
        view_pos(x, y, z, a.f, 0.5f * (float)a.W, 0.5f * (float)a.H, px, py, pz);
        const LightCoord c = to_light(a.M, a.size, a.fL, px, py, pz);
        if (c.inside) {
            const float thr = c.dr - a.bias;
            h = a.sm[(long long)(int)floorf(c.sv) * a.size + (int)floorf(c.su)] < thr ? 1 : 0;
        }
    }
    a.hard[p] = h;
}

hipError_t launch_hard(const HardArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_hard, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

// visibility of one texel; BD / PD point to LDS (staged disks) or global memory
template <typename DP>
__device__ __forceinline__ float pcss_texel(const ShadowArgs& a, const EvalLevel& L, DP bd, DP pd, int x, int y,
                                            float z) {
    float px, py, pz;
    view_pos(x, y, z, L.f, L.cx, L.cy, px, py, pz);
    const LightCoord c = to_light(a.M, a.size, a.fL, px, py, pz);
    if (!c.inside) return 1.0f;
    const float lsz = a.fL * (0.5f * a.lsize);
    const float thr = c.dr - a.bias;
    const float Rs = (lsz * (c.dr - a.nL)) / (c.dr * a.nL);
    float bsum = 0.0f;
    int bcnt = 0;
    for (int k = 0; k < a.nb; ++k) {
        const float s = sm_tap(a.sm, a.size, c.su, c.sv, Rs, bd[2 * k], bd[2 * k + 1]);
        if (s < thr) {
            bsum = bsum + s;
            ++bcnt;
        }
    }
    if (bcnt == 0) return 1.0f;
    const float db = bsum / (float)bcnt;
    const float Rf = (lsz * (c.dr - db)) / (db * c.dr);
    int lit = 0;
    for (int k = 0; k < a.np; ++k) {
        const float s = sm_tap(a.sm, a.size, c.su, c.sv, Rf, pd[2 * k], pd[2 * k + 1]);
        if (!(s < thr)) ++lit;
    }
    return (float)lit / (float)a.np;
}

template <bool LDS, bool AL>
__device__ __forceinline__ void pcss_items(const ShadowArgs& a, const float* bds, const float* pds, const float* eg) {
    const ItemMap m = make_item_map(a.c);
    const unsigned total = item_total(m);
    const ChunkRange cr = chunk_range((total + 255) / 256);
    for (unsigned c = cr.first; c < cr.end; c += cr.step) {
        const unsigned item = c * 256u + threadIdx.x;
        if (item >= total) continue;
        const int j = item_level(m, item);
        const EvalLevel& L = a.c.lv[j];
        const unsigned local = item_local(m, item, j);
        if (local == ~0u) continue;  // padding of the level's item range
        const unsigned t = L.list ? L.list[local] : local;
        if (t >= L.dense_n) continue;  // malformed list entry
        const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
        if (AL && L.ac) L.ac[local] = alpha_dispatch(L, eg + j * kEgStride, x, y);
        const float z = L.z[(unsigned)y * L.zpy + (unsigned)x * L.zpx];
        float vis = 1.0f;
        if (valid_depth(z)) {
            if (LDS)
                vis = pcss_texel(a, L, bds, pds, x, y, z);
            else
                vis = pcss_texel(a, L, a.bd, a.pd, x, y, z);
        }
        store_out(L, L.compact ? local : (unsigned)y * (unsigned)L.W + (unsigned)x, vis);
    }
}

template <bool AL>
__global__ __launch_bounds__(256) void k_pcss(ShadowArgs a) {
    __shared__ float bds[2 * kLdsSamples], pds[2 * kLdsSamples];
    __shared__ float eg[kMaxLevels * kEgStride];
    if (AL) stage_taps(a.c, eg);
    const bool staged = a.nb <= kLdsSamples && a.np <= kLdsSamples;  // uniform
    if (staged) {
        for (int i = threadIdx.x; i < 2 * a.nb; i += 256) bds[i] = a.bd[i];
        for (int i = threadIdx.x; i < 2 * a.np; i += 256) pds[i] = a.pd[i];
        __syncthreads();
        pcss_items<true, AL>(a, bds, pds, eg);
    } else {
        __syncthreads();
        pcss_items<false, AL>(a, bds, pds, eg);
    }
}

hipError_t launch_shadow(const ShadowArgs& a, unsigned total_hint, hipStream_t s) {
    if (fused_alpha(a.c))
        hipLaunchKernelGGL(k_pcss<true>, dim3(eval_blocks<k_pcss<true>>(total_hint)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_pcss<false>, dim3(eval_blocks<k_pcss<false>>(total_hint)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mr
