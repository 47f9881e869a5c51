// Upsampling and blending of the sub-images (Sec. 3.3, Sec. 4.2, Eq. 1).
//
// Per full-resolution pixel and enabled level i: bilinear taps at
// u = (X + 0.5) / s - 0.5 (texel centres, clamp to edge), weights
// b = ((1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy).  Only taps inside the
// level's stencil carry the sub-image value and the sum is renormalised by
// their weight (undefined texels are selected away, never multiplied by 0);
// the blurred mask a_i is interpolated over all four taps.  Then, from the
// coarsest level: c' = C_N, and c' = C_i alpha_i + c' (1 - alpha_i) with
// alpha_i = min(A_i w_i, 1) for the enabled finer levels in descending order
// (the text's order; the printed index of Eq. 1 refers to c'_(i-1) but the
// recursion starts at the lowest resolution).  All sums run left to right
// from +0, which makes the level-1 case an exact select.
#include "mr_internal.hpp"

namespace mr {

struct Taps {
    long long i00, i01, i10, i11;
    float b0, b1, b2, b3;
};

__device__ __forceinline__ Taps make_taps(int X, int Y, const MergeLevel& L) {
    const float inv_s = 1.0f / (float)L.s;  // exact: s is a power of two
    const float u = ((float)X + 0.5f) * inv_s - 0.5f;
    const float v = ((float)Y + 0.5f) * inv_s - 0.5f;
    const float x0f = floorf(u), y0f = floorf(v);
    const float fx = u - x0f, fy = v - y0f;
    const int x0 = (int)x0f, y0 = (int)y0f;
    const int xa = min(max(x0, 0), L.W - 1), xb = min(max(x0 + 1, 0), L.W - 1);
    const int ya = min(max(y0, 0), L.H - 1), yb = min(max(y0 + 1, 0), L.H - 1);
    Taps t;
    t.i00 = (long long)ya * L.W + xa;
    t.i01 = (long long)ya * L.W + xb;
    t.i10 = (long long)yb * L.W + xa;
    t.i11 = (long long)yb * L.W + xb;
    const float gx = 1.0f - fx, gy = 1.0f - fy;
    t.b0 = gx * gy;
    t.b1 = fx * gy;
    t.b2 = gx * fy;
    t.b3 = fx * fy;
    return t;
}

template <int C>
__global__ __launch_bounds__(256) void k_merge(MergeArgs a, unsigned tiles_x, unsigned ntiles) {
    const unsigned tile = xcd_remap(blockIdx.x, ntiles);
    const int X = (int)(tile % tiles_x) * 64 + (threadIdx.x & 63);
    const int Y = (int)(tile / tiles_x) * 4 + (threadIdx.x >> 6);
    if (X >= a.W || Y >= a.H) return;
    const int nl = a.nlev;
    float out[C];
    // coarsest level: plain bilinear (its stencil covers everything)
    {
        const MergeLevel& L = a.lv[nl - 1];
        if (L.s == 1) {
            const long long p = (long long)Y * L.W + X;
            for (int c = 0; c < C; ++c) out[c] = L.c[c * L.c_plane + p];
        } else {
            const Taps t = make_taps(X, Y, L);
            for (int c = 0; c < C; ++c) {
                const float* cc = L.c + c * L.c_plane;
                float num = t.b0 * cc[t.i00];
                num = num + t.b1 * cc[t.i01];
                num = num + t.b2 * cc[t.i10];
                num = num + t.b3 * cc[t.i11];
                // den = b0 + b1 + b2 + b3 = 1 exactly
                out[c] = num / (((t.b0 + t.b1) + t.b2) + t.b3);
            }
        }
    }
    for (int j = nl - 2; j >= 0; --j) {
        const MergeLevel& L = a.lv[j];
        float Ci[C];
        float alpha;
        if (L.s == 1) {
            const long long p = (long long)Y * L.W + X;
            const bool in = L.S[p] != 0;
            for (int c = 0; c < C; ++c) Ci[c] = in ? L.c[c * L.c_plane + p] : 0.0f;
            alpha = in ? fminf(L.a[p] * L.w, 1.0f) : 0.0f;
        } else {
            const Taps t = make_taps(X, Y, L);
            const bool s0 = L.S[t.i00] != 0, s1 = L.S[t.i01] != 0;
            const bool s2 = L.S[t.i10] != 0, s3 = L.S[t.i11] != 0;
            float den = s0 ? t.b0 : 0.0f;
            den = den + (s1 ? t.b1 : 0.0f);
            den = den + (s2 ? t.b2 : 0.0f);
            den = den + (s3 ? t.b3 : 0.0f);
            float A = t.b0 * L.a[t.i00];
            A = A + t.b1 * L.a[t.i01];
            A = A + t.b2 * L.a[t.i10];
            A = A + t.b3 * L.a[t.i11];
            const bool any = den > 0.0f;
            alpha = any ? fminf(A * L.w, 1.0f) : 0.0f;
            for (int c = 0; c < C; ++c) {
                const float* cc = L.c + c * L.c_plane;
                float num = s0 ? t.b0 * cc[t.i00] : 0.0f;
                num = num + (s1 ? t.b1 * cc[t.i01] : 0.0f);
                num = num + (s2 ? t.b2 * cc[t.i10] : 0.0f);
                num = num + (s3 ? t.b3 * cc[t.i11] : 0.0f);
                Ci[c] = any ? num / den : 0.0f;
            }
        }
        const float om = 1.0f - alpha;
        for (int c = 0; c < C; ++c) out[c] = Ci[c] * alpha + out[c] * om;
    }
    const long long p = (long long)Y * a.W + X;
    const long long plane = (long long)a.W * a.H;
    for (int c = 0; c < C; ++c) a.out[c * plane + p] = out[c];
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
    const unsigned tx = (a.W + 63) / 64, ty = (a.H + 3) / 4;
    if (a.C == 3)
        hipLaunchKernelGGL(k_merge<3>, dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    else
        hipLaunchKernelGGL(k_merge<1>, dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    return hipGetLastError();
}

}  // namespace mr
