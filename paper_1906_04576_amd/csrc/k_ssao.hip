// SSAO evaluated per sub-image (Sec. 3.2 / 4.1) and as the naive full-res
// pass (Sec. 5).  The paper cites Mittring 2007 and Bavoil et al. 2008 for
// SSAO without printing an estimator; this one is a normal-oriented
// hemisphere with a fixed caller-supplied kernel, a hard range check and a
// relative depth bias; output = occluded fraction.
#include "eval_common.hpp"

namespace mr {

// occlusion of one texel; K points to LDS (staged samples) or global memory
template <typename NT, typename KP>
__device__ __forceinline__ float ssao_texel(const SsaoArgs& a, const EvalLevel& L, const NT* nrm, unsigned plane,
                                            KP K, int x, int y, float z) {
    const float r = a.r, b = a.b;
    const int S = a.S;
    const float* zb = L.z;
    const int zpy = L.zpy, zpx = L.zpx;
    const unsigned g = (unsigned)L.goff + (unsigned)y * (unsigned)L.gpy + (unsigned)x * (unsigned)L.gpx;
    const float nx = ld(nrm, g), ny = ld(nrm, plane + g), nz = ld(nrm, 2 * plane + g);
    float px, py, pz;
    view_pos(x, y, z, L.f, L.cx, L.cy, px, py, pz);
    float tx, ty, tz, bx, by, bz;
    onb(nx, ny, nz, tx, ty, tz, bx, by, bz);
    const float rtx = r * tx, rty = r * ty, rtz = r * tz;
    const float rbx = r * bx, rby = r * by, rbz = r * bz;
    const float rnx = r * nx, rny = r * ny, rnz = r * nz;
    const float Wf = (float)L.W, Hf = (float)L.H;
    const float f = L.f, cx = L.cx, cy = L.cy;
    // Branch-free sample loop: every sample computes its projection and
    // gathers (texel 0 when it is off-screen or behind the eye), and counts
    // only if all tests pass; the count is the same as skipping the sample,
    // and the unrolled body keeps several gathers in flight per wave.
    int occ = 0;
#pragma unroll 4
    for (int s = 0; s < S; ++s) {
        const float kx = K[3 * s], ky = K[3 * s + 1], kz = K[3 * s + 2];
        const float qz = ((pz + kx * rtz) + ky * rbz) + kz * rnz;
        const float d = -qz;
        const float qx = ((px + kx * rtx) + ky * rbx) + kz * rnx;
        const float qy = ((py + kx * rty) + ky * rby) + kz * rny;
        const float inv = 1.0f / d;
        const float u = cx + (qx * inv) * f;
        const float v = cy - (qy * inv) * f;
        const bool on = (d > 0.0f) & (u >= 0.0f) & (u < Wf) & (v >= 0.0f) & (v < Hf);
        // u, v >= 0 when on, so truncation is floor
        const int sx = (int)(on ? u : 0.0f), sy = (int)(on ? v : 0.0f);
        const float zs = zb[(unsigned)sy * zpy + (unsigned)sx * zpx];
        // z_s <= 0 must not count; +inf and NaN fail the depth test
        occ += (on & (zs > 0.0f) & (zs < d - (b * d)) & (fabsf(z - zs) < r)) ? 1 : 0;
    }
    return (float)occ / (float)S;
}

template <typename NT, bool KLDS, bool AL>
__device__ __forceinline__ void ssao_items(const SsaoArgs& a, const float* ks, const float* eg) {
    const ItemMap m = make_item_map(a.c);
    const unsigned total = item_total(m);
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const unsigned plane = (unsigned)a.c.plane;
    const unsigned nchunks = (total + 255) / 256;
    for (unsigned base = 0; base < nchunks; base += gridDim.x) {
        const unsigned first = chunk_of(base, nchunks);
        if (first == ~0u) break;
        const unsigned item = first + threadIdx.x;
        if (item >= total) continue;
        const int j = item_level(m, item);
        const EvalLevel& L = a.c.lv[j];
        const unsigned local = item_local(m, item, j);
        const unsigned t = L.list ? L.list[local] : local;
        if (t >= L.dense_n) continue;  // malformed list entry
        const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
        if (AL && L.ac) L.ac[local] = alpha_dispatch(L, eg + j * kEgStride, x, y);
        const float z = L.z[(unsigned)y * L.zpy + (unsigned)x * L.zpx];
        float res = 0.0f;
        if (valid_depth(z)) {
            if (KLDS)
                res = ssao_texel<NT>(a, L, nrm, plane, ks, x, y, z);
            else
                res = ssao_texel<NT>(a, L, nrm, plane, a.kernel, x, y, z);
        }
        L.out[L.compact ? local : (unsigned)y * (unsigned)L.W + (unsigned)x] = res;
    }
}

template <typename NT, bool AL>
__global__ __launch_bounds__(256) void k_ssao(SsaoArgs a) {
    __shared__ float ks[3 * kLdsSamples];
    __shared__ float eg[kMaxLevels * kEgStride];
    if (AL) stage_taps(a.c, eg);
    if (a.S <= kLdsSamples) {
        for (int i = threadIdx.x; i < 3 * a.S; i += 256) ks[i] = a.kernel[i];
        __syncthreads();
        ssao_items<NT, true, AL>(a, ks, eg);
    } else {
        __syncthreads();
        ssao_items<NT, false, AL>(a, ks, eg);
    }
}

hipError_t launch_ssao(const SsaoArgs& a, int normal_dtype, unsigned total_hint, hipStream_t s) {
    const unsigned nb = eval_blocks(total_hint);
    const bool al = fused_alpha(a.c);
    if (normal_dtype == MR_F16) {
        if (al)
            hipLaunchKernelGGL((k_ssao<_Float16, true>), dim3(nb), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_ssao<_Float16, false>), dim3(nb), dim3(256), 0, s, a);
    } else {
        if (al)
            hipLaunchKernelGGL((k_ssao<float, true>), dim3(nb), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_ssao<float, false>), dim3(nb), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace mr
