// Mask creation kernels: edge image with fused OR-downsampling (Sec. 3.1),
// separable Gaussian blur with the Table 1 variances and stencil = mask > 0
// (Sec. 3.1, Sec. 4.1), nesting of the inclusive levels and the owner-level
// map.
#include "mr_internal.hpp"

namespace mr {

// ---------------------------------------------------------------------------
// edge image + pooling.  One workgroup = 64 x 32 pixel tile (aligned to every
// pooling block up to s = 32), 256 threads, 8 pixels per thread.
// ---------------------------------------------------------------------------
constexpr int kEdgeTW = 64, kEdgeTH = 32;

template <typename NT>
__device__ __forceinline__ float ndot(const NT* n, long long plane, long long p, long long q) {
    // ((nx_p nx_q) + (ny_p ny_q)) + (nz_p nz_q)
    float a = ld(n, p) * ld(n, q);
    float b = ld(n, plane + p) * ld(n, plane + q);
    float c = ld(n, 2 * plane + p) * ld(n, 2 * plane + q);
    return (a + b) + c;
}

template <typename NT>
__device__ uint8_t edge_at(const EdgeArgs& a, int x, int y) {
    const int W = a.W, H = a.H;
    const long long p = (long long)y * W + x;
    const float z = a.depth[p];
    if (!valid_depth(z)) return 0;
    const bool hl = x > 0, hr = x < W - 1, hu = y > 0, hd = y < H - 1;
    const float zl = hl ? a.depth[p - 1] : 0.0f;
    const float zr = hr ? a.depth[p + 1] : 0.0f;
    const float zu = hu ? a.depth[p - W] : 0.0f;
    const float zd = hd ? a.depth[p + W] : 0.0f;
    // geometry next to background is an edge
    if ((hl && !valid_depth(zl)) || (hr && !valid_depth(zr)) || (hu && !valid_depth(zu)) ||
        (hd && !valid_depth(zd)))
        return 1;
    // depth: relative second difference per axis, skipped at the border
    const float thr = a.depth_ratio * z;
    const float two_z = 2.0f * z;
    if (hl && hr && fabsf((zl + zr) - two_z) > thr) return 1;
    if (hu && hd && fabsf((zu + zd) - two_z) > thr) return 1;
    // normal: first difference as an angle test against the 4-neighbours
    const NT* n = static_cast<const NT*>(a.normal);
    const long long plane = (long long)W * H;
    const float cn = a.normal_cos;
    if (hl && ndot(n, plane, p, p - 1) < cn) return 1;
    if (hr && ndot(n, plane, p, p + 1) < cn) return 1;
    if (hu && ndot(n, plane, p, p - W) < cn) return 1;
    if (hd && ndot(n, plane, p, p + W) < cn) return 1;
    // shadow edges (soft shadows): the one-sample shadow bit changes
    if (a.hard) {
        const uint8_t h = a.hard[p];
        if ((hl && a.hard[p - 1] != h) || (hr && a.hard[p + 1] != h) ||
            (hu && a.hard[p - W] != h) || (hd && a.hard[p + W] != h))
            return 1;
    }
    return 0;
}

template <typename NT>
__global__ __launch_bounds__(256) void k_edges(EdgeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ uint8_t t1[kEdgeTH][kEdgeTW];
    __shared__ uint8_t t2[kEdgeTH / 2][kEdgeTW / 2];
    __shared__ uint8_t t3[kEdgeTH / 4][kEdgeTW / 4];
    __shared__ uint8_t t4[kEdgeTH / 8][kEdgeTW / 8];
    __shared__ uint8_t t5[kEdgeTH / 16][kEdgeTW / 16];
    __shared__ uint8_t t6[kEdgeTH / 32][kEdgeTW / 32];

    const unsigned tile = xcd_remap(blockIdx.x, ntiles);
    const int x0 = (int)(tile % tiles_x) * kEdgeTW;
    const int y0 = (int)(tile / tiles_x) * kEdgeTH;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int W = a.W, H = a.H;
#pragma unroll
    for (int k = 0; k < kEdgeTH / 4; ++k) {
        const int ly = ty + 4 * k;
        const int x = x0 + tx, y = y0 + ly;
        uint8_t e = 0;
        if (x < W && y < H) {
            e = edge_at<NT>(a, x, y);
            a.E[(long long)y * W + x] = e;
            // point-sampled level depth: z_i(X, Y) = z(s X + s/2, s Y + s/2)
            for (int i = 2; i <= a.num_levels; ++i) {
                float* zi = a.zi[i - 1];
                const int s = 1 << (i - 1), h = s >> 1;
                if (zi && (x & (s - 1)) == h && (y & (s - 1)) == h)
                    zi[(long long)(y >> (i - 1)) * a.Wi[i - 1] + (x >> (i - 1))] =
                        a.depth[(long long)y * W + x];
            }
        }
        t1[ly][tx] = e;
    }
    __syncthreads();
    // hierarchical OR: level i texel = OR of its four level-(i-1) children
    const int t = threadIdx.x;
    for (int idx = t; idx < (kEdgeTH / 2) * (kEdgeTW / 2); idx += 256) {
        const int yy = idx / (kEdgeTW / 2), xx = idx % (kEdgeTW / 2);
        t2[yy][xx] = t1[2 * yy][2 * xx] | t1[2 * yy][2 * xx + 1] | t1[2 * yy + 1][2 * xx] |
                     t1[2 * yy + 1][2 * xx + 1];
    }
    __syncthreads();
    if (t < (kEdgeTH / 4) * (kEdgeTW / 4)) {
        const int yy = t / (kEdgeTW / 4), xx = t % (kEdgeTW / 4);
        t3[yy][xx] = t2[2 * yy][2 * xx] | t2[2 * yy][2 * xx + 1] | t2[2 * yy + 1][2 * xx] |
                     t2[2 * yy + 1][2 * xx + 1];
    }
    __syncthreads();
    if (t < (kEdgeTH / 8) * (kEdgeTW / 8)) {
        const int yy = t / (kEdgeTW / 8), xx = t % (kEdgeTW / 8);
        t4[yy][xx] = t3[2 * yy][2 * xx] | t3[2 * yy][2 * xx + 1] | t3[2 * yy + 1][2 * xx] |
                     t3[2 * yy + 1][2 * xx + 1];
    }
    __syncthreads();
    if (t < (kEdgeTH / 16) * (kEdgeTW / 16)) {
        const int yy = t / (kEdgeTW / 16), xx = t % (kEdgeTW / 16);
        t5[yy][xx] = t4[2 * yy][2 * xx] | t4[2 * yy][2 * xx + 1] | t4[2 * yy + 1][2 * xx] |
                     t4[2 * yy + 1][2 * xx + 1];
    }
    __syncthreads();
    if (t < (kEdgeTH / 32) * (kEdgeTW / 32)) {
        const int xx = t;
        t6[0][xx] = t5[0][2 * xx] | t5[0][2 * xx + 1] | t5[1][2 * xx] | t5[1][2 * xx + 1];
    }
    __syncthreads();
    // write the pooled levels that the blur needs
    for (int i = 2; i <= a.num_levels; ++i) {
        uint8_t* Ei = a.Ei[i - 1];
        if (!Ei) continue;
        const int sh = i - 1;
        const int tw = kEdgeTW >> sh, th = kEdgeTH >> sh;
        for (int idx = t; idx < tw * th; idx += 256) {
            const int yy = idx / tw, xx = idx % tw;
            const int X = (x0 >> sh) + xx, Y = (y0 >> sh) + yy;
            if (X >= a.Wi[i - 1] || Y >= a.Hi[i - 1]) continue;
            uint8_t v;
            switch (i) {
                case 2: v = t2[yy][xx]; break;
                case 3: v = t3[yy][xx]; break;
                case 4: v = t4[yy][xx]; break;
                case 5: v = t5[yy][xx]; break;
                default: v = t6[yy][xx]; break;
            }
            Ei[(long long)Y * a.Wi[i - 1] + X] = v;
        }
    }
}

hipError_t launch_edges(const EdgeArgs& a, int normal_dtype, hipStream_t s) {
    const unsigned tx = (a.W + kEdgeTW - 1) / kEdgeTW, ty = (a.H + kEdgeTH - 1) / kEdgeTH;
    const unsigned n = tx * ty;
    if (normal_dtype == MR_F16)
        hipLaunchKernelGGL(k_edges<_Float16>, dim3(n), dim3(256), 0, s, a, tx, n);
    else
        hipLaunchKernelGGL(k_edges<float>, dim3(n), dim3(256), 0, s, a, tx, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// separable blur of one level: tile of 64 x 16 output texels, 256 threads.
// h(x, y) = sum_k g[k] E(x + k, y) then a(x, y) = sum_k g[k] h(x, y + k), taps
// in ascending k, accumulators from +0, zero outside the image.
// ---------------------------------------------------------------------------
constexpr int kBlurTW = 64, kBlurTH = 16;

__global__ __launch_bounds__(256) void k_blur(BlurArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ float es[kBlurTH + 2 * kMaxRadius][kBlurTW + 2 * kMaxRadius];
    __shared__ float hs[kBlurTH + 2 * kMaxRadius][kBlurTW];
    const unsigned tile = xcd_remap(blockIdx.x, ntiles);
    const int x0 = (int)(tile % tiles_x) * kBlurTW;
    const int y0 = (int)(tile / tiles_x) * kBlurTH;
    const int r = a.r, W = a.W, H = a.H;
    const int ew = kBlurTW + 2 * r, eh = kBlurTH + 2 * r;
    for (int idx = threadIdx.x; idx < ew * eh; idx += 256) {
        const int yy = idx / ew, xx = idx % ew;
        const int X = x0 - r + xx, Y = y0 - r + yy;
        float v = 0.0f;
        if (X >= 0 && X < W && Y >= 0 && Y < H) v = a.Ei[(long long)Y * W + X] ? 1.0f : 0.0f;
        es[yy][xx] = v;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < kBlurTW * eh; idx += 256) {
        const int yy = idx / kBlurTW, xx = idx % kBlurTW;
        float acc = 0.0f;
        for (int k = 0; k <= 2 * r; ++k) acc = acc + a.g[k] * es[yy][xx + k];
        hs[yy][xx] = acc;
    }
    __syncthreads();
    const int xx = threadIdx.x & 63;
    for (int yy = threadIdx.x >> 6; yy < kBlurTH; yy += 4) {
        const int X = x0 + xx, Y = y0 + yy;
        if (X >= W || Y >= H) continue;
        float acc = 0.0f;
        for (int k = 0; k <= 2 * r; ++k) acc = acc + a.g[k] * hs[yy + k][xx];
        const long long p = (long long)Y * W + X;
        a.a[p] = acc;
        a.S[p] = acc > 0.0f ? 1 : 0;
    }
}

hipError_t launch_blur(const BlurArgs& a, hipStream_t s) {
    const unsigned tx = (a.W + kBlurTW - 1) / kBlurTW, ty = (a.H + kBlurTH - 1) / kBlurTH;
    hipLaunchKernelGGL(k_blur, dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// nesting: S_coarse(t) |= OR of S_fine over the k x k children of t
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nest(NestArgs a) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long long)a.Wc * a.Hc) return;
    const int Y = (int)(t / a.Wc), X = (int)(t - (long long)Y * a.Wc);
    uint8_t v = 0;
    for (int dy = 0; dy < a.k; ++dy)
        for (int dx = 0; dx < a.k; ++dx)
            v |= a.Sf[(long long)(Y * a.k + dy) * a.Wf + X * a.k + dx];
    if (v) a.Sc[t] = 1;
}

hipError_t launch_nest(const NestArgs& a, hipStream_t s) {
    const long long n = (long long)a.Wc * a.Hc;
    hipLaunchKernelGGL(k_nest, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// owner-level map: finest enabled level whose stencil covers the pixel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_level_map(LevelMapArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    uint8_t lvl = (uint8_t)a.levels[a.nlev - 1];
    for (int j = 0; j < a.nlev - 1; ++j) {
        const int i = a.levels[j], sh = i - 1;
        if (a.S[j][(long long)(y >> sh) * a.Wi[j] + (x >> sh)]) {
            lvl = (uint8_t)i;
            break;
        }
    }
    a.out[(long long)y * a.W + x] = lvl;
}

hipError_t launch_level_map(const LevelMapArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_level_map, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace mr
