// The edge image of one tile (Sec. 3.1) with fused OR-downsampling into the
// level edge bits and the point-sampled level depth: the fast path for
// widths divisible by 4, shared by the frame, batch and persistent launches.
#pragma once
#include "mr_internal.hpp"

namespace mr {

// edge tiles: 64 x 32 pixels (stacked waves), or 256 x 8 (WIDE)
constexpr int kEdgeTW = 64, kEdgeTH = 32;

// Importance mask of a gaze point combined with the edge bit e (minimum with
// the outer disk, maximum with the inner one), FP32 in the documented order.
__device__ __forceinline__ bool fovea(const EdgeArgs& a, int x, int y, bool e) {
    if (!a.fov) return e;
    const float dx = ((float)x + 0.5f) - a.fgx, dy = ((float)y + 0.5f) - a.fgy;
    const float d2 = (dx * dx) + (dy * dy);
    return (e & (d2 <= a.fro2)) | (d2 <= a.fri2);
}

__device__ __forceinline__ bool ndot_lt(const float* a, const float* b, float cn) {
    // ((nx nx') + (ny ny')) + (nz nz') < c_n
    return ((a[0] * b[0]) + (a[1] * b[1])) + (a[2] * b[2]) < cn;
}


// ---------------------------------------------------------------------------
// Fast path for W divisible by 4 (every image with N >= 3 levels): the same
// classification, branch-free, with buffer loads (descriptor + 32-bit offset)
// of clamped rows and columns.  Rows or columns outside the image are loaded
// from a clamped position and only ever used behind the border flags.
// ---------------------------------------------------------------------------
template <typename NT>
struct NormalRow;

template <>
struct NormalRow<float> {
    static constexpr unsigned kSize = 4;
    __device__ static void load4(__amdgpu_buffer_rsrc_t r, unsigned e, float* o) {
        const float4 v = buf_f4(r, e * 4u);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    __device__ static float load1(__amdgpu_buffer_rsrc_t r, unsigned e) { return buf_f1(r, e * 4u); }
};

template <>
struct NormalRow<_Float16> {
    static constexpr unsigned kSize = 2;
    __device__ static void load4(__amdgpu_buffer_rsrc_t r, unsigned e, float* o) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        const h4 v = __builtin_bit_cast(h4, __builtin_amdgcn_raw_buffer_load_b64(r, e * 2u, 0, 0));
        o[0] = (float)v.x;
        o[1] = (float)v.y;
        o[2] = (float)v.z;
        o[3] = (float)v.w;
    }
    __device__ static float load1(__amdgpu_buffer_rsrc_t r, unsigned e) {
        return (float)__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0));
    }
};

// Row shifts within the 16-lane DPP rows: lane i takes src of lane i - 1
// (shr) or i + 1 (shl); the lane with no source in its row keeps `own`.
__device__ __forceinline__ unsigned dpp_shr1u(unsigned own, unsigned src) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)own, (int)src, 0x111, 0xF, 0xF, false);
}
__device__ __forceinline__ unsigned dpp_shl1u(unsigned own, unsigned src) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)own, (int)src, 0x101, 0xF, 0xF, false);
}
__device__ __forceinline__ float dpp_shr1(float own, float src) {
    return __builtin_bit_cast(float, dpp_shr1u(__builtin_bit_cast(unsigned, own), __builtin_bit_cast(unsigned, src)));
}
__device__ __forceinline__ float dpp_shl1(float own, float src) {
    return __builtin_bit_cast(float, dpp_shl1u(__builtin_bit_cast(unsigned, own), __builtin_bit_cast(unsigned, src)));
}

// WIDE: the four waves of a block sit side by side (256 x 8 pixel tile), so
// that a block reads 1 KB runs of every row; levels up to 4 only (the 8 x 8
// pooling blocks stay inside one wave).  Otherwise they are stacked (64 x 32
// tile) and levels 5 and 6 are pooled across the waves through LDS.
// One tile of the edge image; tile k also zeroes counter words 256 k ..
// 256 k + 255 (those below zero_n).
template <typename NT, bool HARD, bool BITS, bool WIDE>
__device__ __forceinline__ void edges_tile(const EdgeArgs& a, unsigned tile, unsigned tiles_x) {
    __shared__ uint8_t p4[4][8];
    if (a.zero && tile * 256u + threadIdx.x < a.zero_n) a.zero[tile * 256u + threadIdx.x] = 0u;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int x0 = WIDE ? (int)(tile % tiles_x) * (4 * kEdgeTW) + wave * kEdgeTW : (int)(tile % tiles_x) * kEdgeTW;
    const int y0 = WIDE ? (int)(tile / tiles_x) * 8 : (int)(tile / tiles_x) * kEdgeTH;
    const int W = a.W, H = a.H;
    const int cg = lane & 15, rp = lane >> 4;
    const int xb = x0 + 4 * cg, yb = y0 + (WIDE ? 0 : 8 * wave) + 2 * rp;
    const bool any = xb < W && yb < H;
    const unsigned plane = (unsigned)W * (unsigned)H;
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(a.depth, plane * 4u);
    const NT* nrm = static_cast<const NT*>(a.normal);
    const unsigned nb = plane * NormalRow<NT>::kSize;
    const __amdgpu_buffer_rsrc_t rn0 = buf_rsrc(nrm, nb), rn1 = buf_rsrc(nrm + plane, nb),
                                 rn2 = buf_rsrc(nrm + 2 * plane, nb);
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(a.hard, HARD ? plane : 0u);
    // clamped element offsets of rows yb-1 .. yb+2 and the side columns
    const int xc = min(xb, W - 4);
    unsigned ro[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ro[r] = (unsigned)min(max(yb - 1 + r, 0), H - 1) * (unsigned)W;
    // Side columns xb - 1 and xb + 4 are the neighbouring lanes' pixels (the
    // 16 lanes of a DPP row cover the wave's 64 columns of one row pair);
    // only the wave's outer columns x0 - 1 and x0 + 64 come from elsewhere.
    const unsigned xl = (unsigned)max(x0 - 1, 0), xr = (unsigned)min(x0 + 64, W - 1);

    float z[4][4], n[4][4][3];
    float zs[2][2], ns[2][2][3];
    unsigned hrow[4] = {0, 0, 0, 0}, hside[2][2] = {{0, 0}, {0, 0}};
    // Rows yb - 1 .. yb + 2: a lane loads its own rows yb, yb + 1; the row
    // above is the second own row of the lane 16 below (the wave's row pairs
    // are consecutive) and the row below the first own row of the lane 16
    // above, except for the wave's first and last row pair, which load the
    // wave's halo rows.  Every row of the wave is read once.
#pragma unroll
    for (int r = 1; r <= 2; ++r) {
        const unsigned e = ro[r] + (unsigned)xc;
        const float4 zv = buf_f4(rz, e * 4u);
        z[r][0] = zv.x;
        z[r][1] = zv.y;
        z[r][2] = zv.z;
        z[r][3] = zv.w;
        float t0[4], t1[4], t2[4];
        NormalRow<NT>::load4(rn0, e, t0);
        NormalRow<NT>::load4(rn1, e, t1);
        NormalRow<NT>::load4(rn2, e, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            n[r][k][0] = t0[k];
            n[r][k][1] = t1[k];
            n[r][k][2] = t2[k];
        }
        if (HARD) hrow[r] = __builtin_amdgcn_raw_buffer_load_b32(rh, e, 0, 0);
    }
    const bool top = rp == 0, bot = rp == 3;
    float hz[4] = {0.0f, 0.0f, 0.0f, 0.0f}, hn[4][3] = {};
    unsigned hh = 0u;
    if (top || bot) {
        const unsigned e = (top ? ro[0] : ro[3]) + (unsigned)xc;
        const float4 zv = buf_f4(rz, e * 4u);
        hz[0] = zv.x;
        hz[1] = zv.y;
        hz[2] = zv.z;
        hz[3] = zv.w;
        float t0[4], t1[4], t2[4];
        NormalRow<NT>::load4(rn0, e, t0);
        NormalRow<NT>::load4(rn1, e, t1);
        NormalRow<NT>::load4(rn2, e, t2);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            hn[k][0] = t0[k];
            hn[k][1] = t1[k];
            hn[k][2] = t2[k];
        }
        if (HARD) hh = __builtin_amdgcn_raw_buffer_load_b32(rh, e, 0, 0);
    }
    const int lup = (lane + 48) & 63, ldn = (lane + 16) & 63;  // lanes 16 below / above
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float za = __shfl(z[2][k], lup, 64), zb = __shfl(z[1][k], ldn, 64);
        z[0][k] = top ? hz[k] : za;
        z[3][k] = bot ? hz[k] : zb;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float na = __shfl(n[2][k][c], lup, 64), nb_ = __shfl(n[1][k][c], ldn, 64);
            n[0][k][c] = top ? hn[k][c] : na;
            n[3][k][c] = bot ? hn[k][c] : nb_;
        }
    }
    if (HARD) {
        const unsigned ha = (unsigned)__shfl((int)hrow[2], lup, 64), hb = (unsigned)__shfl((int)hrow[1], ldn, 64);
        hrow[0] = top ? hh : ha;
        hrow[3] = bot ? hh : hb;
    }
    // Side columns x0 - 1 and x0 + 64 of the own rows.  With WIDE the four
    // waves of the block sit side by side: a wave's side column is a
    // neighbouring wave's first or last column, passed through LDS; only
    // the block's outer columns are loaded.  Otherwise every lane of a row
    // loads them from the same address (one cache line).
    auto load_side = [&](int r, int sd) {
        const unsigned e = ro[r + 1] + (sd ? xr : xl);
        zs[r][sd] = buf_f1(rz, e * 4u);
        ns[r][sd][0] = NormalRow<NT>::load1(rn0, e);
        ns[r][sd][1] = NormalRow<NT>::load1(rn1, e);
        ns[r][sd][2] = NormalRow<NT>::load1(rn2, e);
        if (HARD) hside[r][sd] = __builtin_amdgcn_raw_buffer_load_b8(rh, e, 0, 0);
    };
    if (WIDE) {
        __shared__ float sidex[4][2][8][5];  // [wave][first / last column][row][z, n, hard bits]
        const int rr = 2 * rp;
        if (cg == 0 || cg == 15) {
            const int sd = cg == 15 ? 1 : 0, k = sd ? 3 : 0;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                float* o = sidex[wave][sd][rr + r];
                o[0] = z[r + 1][k];
                o[1] = n[r + 1][k][0];
                o[2] = n[r + 1][k][1];
                o[3] = n[r + 1][k][2];
                o[4] = __uint_as_float(HARD ? (hrow[r + 1] >> (8 * k)) & 0xFFu : 0u);
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                const int nw = sd ? wave + 1 : wave - 1;  // the neighbouring wave (uniform)
                if (nw < 0 || nw > 3) {
                    load_side(r, sd);
                } else {
                    const float* i = sidex[nw][1 - sd][rr + r];
                    zs[r][sd] = i[0];
                    ns[r][sd][0] = i[1];
                    ns[r][sd][1] = i[2];
                    ns[r][sd][2] = i[3];
                    hside[r][sd] = __float_as_uint(i[4]);
                }
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            load_side(r, 0);
            load_side(r, 1);
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        // lane cg takes column xb - 1 from lane cg - 1 and xb + 4 from lane
        // cg + 1; lanes 0 and 15 of the row keep the side columns
        zs[r][0] = dpp_shr1(zs[r][0], z[r + 1][3]);
        zs[r][1] = dpp_shl1(zs[r][1], z[r + 1][0]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ns[r][0][c] = dpp_shr1(ns[r][0][c], n[r + 1][3][c]);
            ns[r][1][c] = dpp_shl1(ns[r][1][c], n[r + 1][0][c]);
        }
        if (HARD) {
            hside[r][0] = dpp_shr1u(hside[r][0], (hrow[r + 1] >> 24) & 0xFFu);
            hside[r][1] = dpp_shl1u(hside[r][1], hrow[r + 1] & 0xFFu);
        }
    }
    // normal pair tests, each pair once
    const float cn = a.normal_cos, td = a.depth_ratio;
    bool hp[2][5], vp[3][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        hp[r][0] = ndot_lt(ns[r][0], n[r + 1][0], cn);
#pragma unroll
        for (int c = 1; c < 4; ++c) hp[r][c] = ndot_lt(n[r + 1][c - 1], n[r + 1][c], cn);
        hp[r][4] = ndot_lt(n[r + 1][3], ns[r][1], cn);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) vp[k][c] = ndot_lt(n[k][c], n[k + 1][c], cn);
    // classify, branch-free (non-short-circuit logic)
    uint8_t e[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int y = yb + r;
        const bool hu = y > 0, hd = y < H - 1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int x = xb + c;
            const bool hl = x > 0, hr = x < W - 1;
            const float zc = z[r + 1][c];
            const float zl = c > 0 ? z[r + 1][c - 1] : zs[r][0];
            const float zr = c < 3 ? z[r + 1][c + 1] : zs[r][1];
            const float zu = z[r][c], zd = z[r + 2][c];
            bool ed = (hl & !valid_depth(zl)) | (hr & !valid_depth(zr)) | (hu & !valid_depth(zu)) |
                      (hd & !valid_depth(zd));
            const float thr = td * zc;
            const float two_z = 2.0f * zc;
            ed |= hl & hr & (fabsf((zl + zr) - two_z) > thr);
            ed |= hu & hd & (fabsf((zu + zd) - two_z) > thr);
            ed |= (hl & hp[r][c]) | (hr & hp[r][c + 1]) | (hu & vp[r][c]) | (hd & vp[r + 1][c]);
            if (HARD) {
                const unsigned sh = 8u * (unsigned)c;
                const unsigned hc = (hrow[r + 1] >> sh) & 0xFFu;
                const unsigned hl_ = c > 0 ? (hrow[r + 1] >> (sh - 8u)) & 0xFFu : hside[r][0];
                const unsigned hr_ = c < 3 ? (hrow[r + 1] >> (sh + 8u)) & 0xFFu : hside[r][1];
                const unsigned hu_ = (hrow[r] >> sh) & 0xFFu, hd_ = (hrow[r + 2] >> sh) & 0xFFu;
                ed |= (hl & (hl_ != hc)) | (hr & (hr_ != hc)) | (hu & (hu_ != hc)) | (hd & (hd_ != hc));
            }
            e[r][c] = (any & (y < H) & fovea(a, x, y, valid_depth(zc) & ed)) ? 1 : 0;
        }
    }
    if (BITS) {
        // bit-packed level 1: a tile row of 64 pixels is 2 words; the 8 lanes
        // of a word OR their shifted nibbles together (shuffles run on all lanes)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            unsigned v1 = (unsigned)(e[r][0] | (e[r][1] << 1) | (e[r][2] << 2) | (e[r][3] << 3)) << (4 * (cg & 7));
            v1 |= __shfl_xor(v1, 1, 64);
            v1 |= __shfl_xor(v1, 2, 64);
            v1 |= __shfl_xor(v1, 4, 64);
            if (any && (cg & 7) == 0 && yb + r < H)
                a.Eb[0][(unsigned)(yb + r) * (unsigned)a.wpr[0] + (unsigned)((xb >> 5))] = v1;
        }
        // level 2: 32 texels per tile row = one word
        unsigned v2 = ((unsigned)(e[0][0] | e[0][1] | e[1][0] | e[1][1]) |
                       ((unsigned)(e[0][2] | e[0][3] | e[1][2] | e[1][3]) << 1))
                      << (2 * cg);
        v2 |= __shfl_xor(v2, 1, 64);
        v2 |= __shfl_xor(v2, 2, 64);
        v2 |= __shfl_xor(v2, 4, 64);
        v2 |= __shfl_xor(v2, 8, 64);
        if (any && cg == 0 && a.Eb[1])
            a.Eb[1][(unsigned)(yb >> 1) * (unsigned)a.wpr[1] + (unsigned)(x0 >> 6)] = v2;
    }
    if (any && !BITS) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = yb + r;
            if (y < H)
                *reinterpret_cast<uchar4*>(a.E + (unsigned)y * (unsigned)W + (unsigned)xb) =
                    make_uchar4(e[r][0], e[r][1], e[r][2], e[r][3]);
        }
    }
    if (any) {
        // point-sampled level depth: z_i(X, Y) = z(s X + s/2, s Y + s/2).  For
        // s = 2 that is columns xb+1, xb+3 of row yb+1; for s >= 4 at most one
        // pixel of the block qualifies: column 2 (s = 4) or 0 (s >= 8) of row yb.
        if (a.zi[1]) {
            float* z2 = a.zi[1] + (unsigned)(yb >> 1) * (unsigned)a.Wi[1] + (unsigned)(xb >> 1);
            z2[0] = z[2][1];
            z2[1] = z[2][3];
        }
        for (int i = 3; i <= a.num_levels; ++i) {
            float* zi = a.zi[i - 1];
            if (!zi) continue;
            const int sh = i - 1, s = 1 << sh, hf = s >> 1;
            const int cs = s == 4 ? 2 : 0;
            if ((xb & (s - 1)) == hf - cs && (yb & (s - 1)) == hf)
                zi[(unsigned)(yb >> sh) * (unsigned)a.Wi[i - 1] + (unsigned)((xb + cs) >> sh)] =
                    s == 4 ? z[1][2] : z[1][0];
        }
        if (!BITS && a.Ei[1]) {
            uint8_t* e2 = a.Ei[1] + (unsigned)(yb >> 1) * (unsigned)a.Wi[1] + (unsigned)(xb >> 1);
            e2[0] = e[0][0] | e[0][1] | e[1][0] | e[1][1];
            e2[1] = e[0][2] | e[0][3] | e[1][2] | e[1][3];
        }
    }
    int v = e[0][0] | e[0][1] | e[0][2] | e[0][3] | e[1][0] | e[1][1] | e[1][2] | e[1][3];
    v |= __shfl_xor(v, 16, 64);
    if (BITS) {
        // level 3: 16 texels per tile row = half a word (ushort store)
        unsigned v3 = (unsigned)v << cg;
        v3 |= __shfl_xor(v3, 1, 64);
        v3 |= __shfl_xor(v3, 2, 64);
        v3 |= __shfl_xor(v3, 4, 64);
        v3 |= __shfl_xor(v3, 8, 64);
        if (any && cg == 0 && (rp & 1) == 0 && a.Eb[2])
            reinterpret_cast<uint16_t*>(a.Eb[2])[(unsigned)(yb >> 2) * (unsigned)(2 * a.wpr[2]) +
                                                 (unsigned)(x0 >> 6)] = (uint16_t)v3;
    } else if (any && a.Ei[2] && (rp & 1) == 0) {
        a.Ei[2][(unsigned)(yb >> 2) * (unsigned)a.Wi[2] + (unsigned)(xb >> 2)] = (uint8_t)v;
    }
    v |= __shfl_xor(v, 1, 64);
    v |= __shfl_xor(v, 32, 64);
    if (any && a.Ei[3] && (cg & 1) == 0 && rp == 0)
        a.Ei[3][(unsigned)(yb >> 3) * (unsigned)a.Wi[3] + (unsigned)(xb >> 3)] = (uint8_t)v;
    if (!WIDE && a.num_levels >= 5) {
        if (rp == 0 && (cg & 1) == 0) p4[wave][cg >> 1] = (uint8_t)v;
        __syncthreads();
        if (a.Ei[4] && t < 8) {
            const int w = (t >> 2) * 2, j = t & 3;
            const int X = (x0 >> 4) + j, Y = (y0 >> 4) + (w >> 1);
            if (X < a.Wi[4] && Y < a.Hi[4])
                a.Ei[4][(unsigned)Y * (unsigned)a.Wi[4] + (unsigned)X] =
                    p4[w][2 * j] | p4[w][2 * j + 1] | p4[w + 1][2 * j] | p4[w + 1][2 * j + 1];
        }
        if (a.num_levels >= 6 && a.Ei[5] && t < 2) {
            const int X = (x0 >> 5) + t, Y = y0 >> 5;
            uint8_t o = 0;
            for (int w = 0; w < 4; ++w)
                for (int j = 0; j < 4; ++j) o |= p4[w][4 * t + j];
            if (X < a.Wi[5] && Y < a.Hi[5]) a.Ei[5][(unsigned)Y * (unsigned)a.Wi[5] + (unsigned)X] = o;
        }
    }
}

}  // namespace mr
