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
    int i00, i01, i10, i11;  // LDS indices of the four taps
    float b0, b1, b2, b3;
};

// One axis of the bilinear taps at full-res coordinate X for scale s = 2^sh:
// u = (X + 0.5) / s - 0.5 is the exact dyadic (m + 0.5) / s with m = X - s/2,
// so floor(u) = m >> sh (floor division) and u - floor(u) = ((m mod s) + 0.5) / s;
// both are computed exactly here with integers.  Taps are clamped to the
// level and returned relative to the staged region's origin `lo`.
__device__ __forceinline__ void axis_taps(int X, int sh, int n, int lo, int& ia, int& ib, float& f) {
    const int s = 1 << sh;
    const int m = X - (s >> 1);
    const int x0 = m >> sh;
    f = ((float)(m & (s - 1)) + 0.5f) * (1.0f / (float)s);
    ia = min(max(x0, 0), n - 1) - lo;
    ib = min(max(x0 + 1, 0), n - 1) - lo;
}

template <int C>
__global__ __launch_bounds__(256) void k_merge(MergeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ float la[kMergeLDS];
    __shared__ uint8_t ls[kMergeLDS];
    __shared__ float lc[C][kMergeLDS];
    const unsigned tile = xcd_remap(blockIdx.x, ntiles);
    const int x0 = (int)(tile % tiles_x) * kMergeTW;
    const int y0 = (int)(tile / tiles_x) * kMergeTH;
    const int nl = a.nlev, t = threadIdx.x;
    const bool fine1 = a.lv[0].s == 1 && nl > 1;  // level 1 is read per pixel from memory
    // ---- issue every load of the tile before the first LDS store ----
    constexpr int kSlots = (kMergeLDS + 255) / 256;
    uint8_t sv[kSlots];
    float av[kSlots], cv[kSlots][C];
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int idx = t + 256 * j;
        sv[j] = 0;
        av[j] = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) cv[j][c] = 0.0f;
        if (idx >= a.staged) continue;
        const uint8_t* Sp = nullptr;
        const float* ap = nullptr;
        const float* cp = nullptr;
        long long cpl = 0, p = 0;
        bool coarsest = false;
#pragma unroll
        for (int q = 0; q < kMaxLevels; ++q) {
            const MergeLevel& L = a.lv[q];
            if (q < nl && L.s != 1 && idx >= L.roff && idx < L.roff + L.rw * L.rh) {
                const int k = idx - L.roff;
                const int yy = (int)(((unsigned)k * L.rmagic) >> 16), xx = k - yy * L.rw;
                const int Xl = min(max((x0 >> L.sh) - 1 + xx, 0), L.W - 1);
                const int Yl = min(max((y0 >> L.sh) - 1 + yy, 0), L.H - 1);
                p = (long long)Yl * L.W + Xl;
                Sp = L.S;
                ap = L.a;
                cp = L.c;
                cpl = L.c_plane;
                coarsest = q == nl - 1;
            }
        }
        sv[j] = coarsest ? 1 : Sp[p];
        av[j] = coarsest ? 0.0f : ap[p];
#pragma unroll
        for (int c = 0; c < C; ++c) cv[j][c] = cp[c * cpl + p];
    }
    const int q = t & 15, row = t >> 4;
    const int Y = y0 + row;
    const int XQ = x0 + 4 * q;
    const bool active = Y < a.H && XQ < a.W;
    uint8_t s1[4] = {0, 0, 0, 0};
    float a1[4] = {0, 0, 0, 0}, c1[C][4];
#pragma unroll
    for (int c = 0; c < C; ++c) c1[c][0] = c1[c][1] = c1[c][2] = c1[c][3] = 0.0f;
    const bool vec = (a.W & 3) == 0;
    if (fine1 && active) {
        const MergeLevel& L = a.lv[0];
        const long long p = (long long)Y * L.W + XQ;
        if (vec) {
            const uchar4 s4 = *reinterpret_cast<const uchar4*>(L.S + p);
            s1[0] = s4.x;
            s1[1] = s4.y;
            s1[2] = s4.z;
            s1[3] = s4.w;
            const float4 a4 = *reinterpret_cast<const float4*>(L.a + p);
            a1[0] = a4.x;
            a1[1] = a4.y;
            a1[2] = a4.z;
            a1[3] = a4.w;
            if (s1[0] | s1[1] | s1[2] | s1[3]) {
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float4 c4 = *reinterpret_cast<const float4*>(L.c + c * L.c_plane + p);
                    c1[c][0] = c4.x;
                    c1[c][1] = c4.y;
                    c1[c][2] = c4.z;
                    c1[c][3] = c4.w;
                }
            }
        } else {
            for (int k = 0; k < 4; ++k) {
                const bool in = XQ + k < a.W;
                s1[k] = in ? L.S[p + k] : 0;
                a1[k] = in ? L.a[p + k] : 0.0f;
                for (int c = 0; c < C; ++c) c1[c][k] = (in && s1[k]) ? L.c[c * L.c_plane + p + k] : 0.0f;
            }
        }
    }
    // ---- stage the coarse levels ----
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int idx = t + 256 * j;
        if (idx >= a.staged) continue;
        ls[idx] = sv[j];
        la[idx] = av[j];
#pragma unroll
        for (int c = 0; c < C; ++c) lc[c][idx] = sv[j] ? cv[j][c] : 0.0f;
    }
    __syncthreads();
    if (!active) return;

    // ---- blend: levels outer (coarse to fine), the thread's 4 pixels inner ----
    float out[C][4];
    {
        // coarsest level: plain bilinear (its stencil covers everything, so
        // the normalising sum of the weights is exactly 1 and num / 1 = num)
        const MergeLevel& L = a.lv[nl - 1];
        if (L.s == 1) {
            const long long p = (long long)Y * L.W + XQ;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < C; ++c) out[c][k] = XQ + k < a.W ? L.c[c * L.c_plane + p + k] : 0.0f;
        } else {
            int ya, yb;
            float fy;
            axis_taps(Y, L.sh, L.H, (y0 >> L.sh) - 1, ya, yb, fy);
            const float gy = 1.0f - fy;
            const int r0 = L.roff + ya * L.rw, r1 = L.roff + yb * L.rw;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                int xa, xb;
                float fx;
                axis_taps(XQ + k, L.sh, L.W, (x0 >> L.sh) - 1, xa, xb, fx);
                const float gx = 1.0f - fx;
                const float b0 = gx * gy, b1 = fx * gy, b2 = gx * fy, b3 = fx * fy;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    float num = b0 * lc[c][r0 + xa];
                    num = num + b1 * lc[c][r0 + xb];
                    num = num + b2 * lc[c][r1 + xa];
                    num = num + b3 * lc[c][r1 + xb];
                    out[c][k] = num;
                }
            }
        }
    }
    // finer levels.  alpha = 0 leaves the composite unchanged bit for bit
    // (C * 0 + c' * 1 = c' for the finite C >= 0 of every level), so a level
    // with A = 0 at all four pixels is skipped; otherwise the four pixels are
    // blended branch-free with alpha = 0 where A = 0 or no tap is in the
    // stencil.  A full stencil has den = 1 and num / 1 = num.
    for (int j = nl - 2; j >= 0; --j) {
        const MergeLevel& L = a.lv[j];
        if (j == 0 && fine1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in = s1[k] != 0;
                const float alpha = in ? fminf(a1[k] * L.w, 1.0f) : 0.0f;
                const float om = 1.0f - alpha;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const float Ci = in ? c1[c][k] : 0.0f;
                    out[c][k] = Ci * alpha + out[c][k] * om;
                }
            }
            continue;
        }
        int ya, yb;
        float fy;
        axis_taps(Y, L.sh, L.H, (y0 >> L.sh) - 1, ya, yb, fy);
        const float gy = 1.0f - fy;
        const int r0 = L.roff + ya * L.rw, r1 = L.roff + yb * L.rw;
        float A[4], b[4][4];
        int ix[4][2];
        bool nz = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int xa, xb;
            float fx;
            axis_taps(XQ + k, L.sh, L.W, (x0 >> L.sh) - 1, xa, xb, fx);
            const float gx = 1.0f - fx;
            b[k][0] = gx * gy;
            b[k][1] = fx * gy;
            b[k][2] = gx * fy;
            b[k][3] = fx * fy;
            ix[k][0] = xa;
            ix[k][1] = xb;
            float s_ = b[k][0] * la[r0 + xa];
            s_ = s_ + b[k][1] * la[r0 + xb];
            s_ = s_ + b[k][2] * la[r1 + xa];
            s_ = s_ + b[k][3] * la[r1 + xb];
            A[k] = s_;
            nz |= s_ != 0.0f;
        }
        if (!nz) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i00 = r0 + ix[k][0], i01 = r0 + ix[k][1], i10 = r1 + ix[k][0], i11 = r1 + ix[k][1];
            const bool e0 = ls[i00] != 0, e1 = ls[i01] != 0, e2 = ls[i10] != 0, e3 = ls[i11] != 0;
            float den = e0 ? b[k][0] : 0.0f;
            den = den + (e1 ? b[k][1] : 0.0f);
            den = den + (e2 ? b[k][2] : 0.0f);
            den = den + (e3 ? b[k][3] : 0.0f);
            const bool use = A[k] != 0.0f && den > 0.0f;
            const float alpha = use ? fminf(A[k] * L.w, 1.0f) : 0.0f;
            const float om = 1.0f - alpha;
            const float dd = use ? den : 1.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                float num = e0 ? b[k][0] * lc[c][i00] : 0.0f;
                num = num + (e1 ? b[k][1] * lc[c][i01] : 0.0f);
                num = num + (e2 ? b[k][2] * lc[c][i10] : 0.0f);
                num = num + (e3 ? b[k][3] * lc[c][i11] : 0.0f);
                const float Ci = use ? (dd == 1.0f ? num : num / dd) : 0.0f;
                out[c][k] = Ci * alpha + out[c][k] * om;
            }
        }
    }
    // ---- store ----
    const long long p = (long long)Y * a.W + XQ;
    const long long plane = (long long)a.W * a.H;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        if (vec) {
            *reinterpret_cast<float4*>(a.out + c * plane + p) = make_float4(out[c][0], out[c][1], out[c][2], out[c][3]);
        } else {
            for (int k = 0; k < 4 && XQ + k < a.W; ++k) a.out[c * plane + p + k] = out[c][k];
        }
    }
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t s) {
    const unsigned tx = (a.W + kMergeTW - 1) / kMergeTW, ty = (a.H + kMergeTH - 1) / kMergeTH;
    if (a.C == 3)
        hipLaunchKernelGGL(k_merge<3>, dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    else
        hipLaunchKernelGGL(k_merge<1>, dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    return hipGetLastError();
}

}  // namespace mr
