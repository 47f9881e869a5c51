// SSAO evaluated per sub-image (Sec. 3.2 / 4.1) and as the naive full-res
// pass (Sec. 5).  The paper cites Mittring 2007 and Bavoil et al. 2008 for
// SSAO without printing an estimator; this one is a normal-oriented
// hemisphere with a fixed caller-supplied kernel, a hard range check and a
// relative depth bias; output = occluded fraction.
#include "eval_common.hpp"

namespace mr {

template <typename NT>
__global__ __launch_bounds__(256) void k_ssao(SsaoArgs a) {
    const ItemMap m = make_item_map(a.c);
    const unsigned total = m.cum[m.nlev];
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const long long plane = a.c.plane;
    const float r = a.r, b = a.b;
    const int S = a.S;
    for (unsigned item = blockIdx.x * 256 + threadIdx.x; item < total; item += gridDim.x * 256) {
        const int j = item_level(m, item);
        const EvalLevel& L = a.c.lv[j];
        const unsigned local = item - m.cum[j];
        const unsigned t = L.list ? L.list[local] : local;
        if (t >= L.dense_n) continue;  // malformed list entry
        const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
        const float z = L.z[(long long)y * L.zpy + (long long)x * L.zpx];
        float res = 0.0f;
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
            const float Wf = (float)L.W, Hf = (float)L.H;
            int occ = 0;
            for (int s = 0; s < S; ++s) {
                const float kx = a.kernel[3 * s], ky = a.kernel[3 * s + 1], kz = a.kernel[3 * s + 2];
                const float qx = ((px + kx * rtx) + ky * rbx) + kz * rnx;
                const float qy = ((py + kx * rty) + ky * rby) + kz * rny;
                const float qz = ((pz + kx * rtz) + ky * rbz) + kz * rnz;
                const float d = -qz;
                if (!(d > 0.0f)) continue;
                const float inv = 1.0f / d;
                const float u = L.cx + (qx * inv) * L.f;
                const float v = L.cy - (qy * inv) * L.f;
                if (!(u >= 0.0f && u < Wf && v >= 0.0f && v < Hf)) continue;
                const int sx = (int)floorf(u), sy = (int)floorf(v);
                const float zs = L.z[(long long)sy * L.zpy + (long long)sx * L.zpx];
                if (!valid_depth(zs)) continue;
                if (zs < d - (b * d) && fabsf(z - zs) < r) ++occ;
            }
            res = (float)occ / (float)S;
        }
        L.out[(long long)y * L.W + x] = res;
    }
}

hipError_t launch_ssao(const SsaoArgs& a, int normal_dtype, unsigned total_hint, hipStream_t s) {
    const unsigned nb = eval_blocks(total_hint);
    if (normal_dtype == MR_F16)
        hipLaunchKernelGGL(k_ssao<_Float16>, dim3(nb), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_ssao<float>, dim3(nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mr
