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

// Raw loads of normal components (raw4: four consecutive pixels, raw1: one)
// and their conversion to FP32; the conversion is kept apart from the load so
// that a load can be issued long before its value is used.
template <>
struct NormalRow<float> {
    static constexpr unsigned kSize = 4;
    typedef float4 raw4;
    typedef float raw1;
    __device__ static raw4 ld4(__amdgpu_buffer_rsrc_t r, unsigned e) { return buf_f4(r, e * 4u); }
    __device__ static raw1 ld1(__amdgpu_buffer_rsrc_t r, unsigned e) { return buf_f1(r, e * 4u); }
    __device__ static void cvt4(const raw4& v, float* o) {
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
    __device__ static float cvt1(raw1 v) { return v; }
};

template <>
struct NormalRow<_Float16> {
    static constexpr unsigned kSize = 2;
    typedef _Float16 raw4 __attribute__((ext_vector_type(4)));
    typedef _Float16 raw1;
    __device__ static raw4 ld4(__amdgpu_buffer_rsrc_t r, unsigned e) {
        return __builtin_bit_cast(raw4, __builtin_amdgcn_raw_buffer_load_b64(r, e * 2u, 0, 0));
    }
    __device__ static raw1 ld1(__amdgpu_buffer_rsrc_t r, unsigned e) {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0));
    }
    __device__ static void cvt4(const raw4& v, float* o) {
        o[0] = (float)v.x;
        o[1] = (float)v.y;
        o[2] = (float)v.z;
        o[3] = (float)v.w;
    }
    __device__ static float cvt1(raw1 v) { return (float)v; }
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

// Where a lane's pixels of one tile lie: a 4 x 2 pixel block at (xb, yb),
// the clamped element offsets ro of rows yb - 1 .. yb + 2, the clamped
// column xc of the block's four-pixel loads and the wave's clamped outer
// columns xl = x0 - 1 and xr = x0 + 64.
struct EdgeGeom {
    int wave, lane, x0, y0, cg, rp, xb, yb, xc;
    bool any;
    unsigned ro[4], xl, xr;
};

template <bool WIDE>
__device__ __forceinline__ EdgeGeom edge_geom(const EdgeArgs& a, unsigned tile, unsigned tiles_x) {
    EdgeGeom g;
    const int t = threadIdx.x;
    g.wave = t >> 6;
    g.lane = t & 63;
    g.x0 = WIDE ? (int)(tile % tiles_x) * (4 * kEdgeTW) + g.wave * kEdgeTW : (int)(tile % tiles_x) * kEdgeTW;
    g.y0 = WIDE ? (int)(tile / tiles_x) * 8 : (int)(tile / tiles_x) * kEdgeTH;
    g.cg = g.lane & 15;
    g.rp = g.lane >> 4;
    g.xb = g.x0 + 4 * g.cg;
    g.yb = g.y0 + (WIDE ? 0 : 8 * g.wave) + 2 * g.rp;
    g.any = g.xb < a.W && g.yb < a.H;
    g.xc = min(g.xb, a.W - 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) g.ro[r] = (unsigned)min(max(g.yb - 1 + r, 0), a.H - 1) * (unsigned)a.W;
    g.xl = (unsigned)max(g.x0 - 1, 0);
    g.xr = (unsigned)min(g.x0 + 64, a.W - 1);
    return g;
}

// Everything one tile reads from memory, as loaded (normals not yet
// converted): a lane's own rows yb and yb + 1, the wave's halo row (row
// yb - 1 for the first row pair of the wave, yb + 2 for the last), and the
// side columns x0 - 1 and x0 + 64 of its own rows (with WIDE only the
// block's outer columns; the inner ones come from the neighbouring wave).
template <typename NT, bool HARD>
struct EdgeLoads {
    typedef typename NormalRow<NT>::raw4 N4;
    typedef typename NormalRow<NT>::raw1 N1;
    float4 z[2], hz;
    N4 n[2][3], hn[3];
    unsigned h[2], hh;
    float zs[2][2];
    N1 ns[2][2][3];
    unsigned hs[2][2];
};

// Issues every load of one tile, the block's outer side columns included,
// before any of them is waited for.  (Loading the outer columns after the
// exchange of the inner ones through LDS put a second memory latency on the
// outer waves, which the exchange's barrier passed on to the whole block.)
template <typename NT, bool HARD, bool WIDE>
__device__ __forceinline__ void edges_load(const EdgeArgs& a, const EdgeGeom& g, EdgeLoads<NT, HARD>& L) {
    typedef NormalRow<NT> NR;
    const unsigned plane = (unsigned)a.W * (unsigned)a.H;
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(a.depth, plane * 4u);
    const NT* nrm = static_cast<const NT*>(a.normal);
    const unsigned nb = plane * NR::kSize;
    const __amdgpu_buffer_rsrc_t rn[3] = {buf_rsrc(nrm, nb), buf_rsrc(nrm + plane, nb), buf_rsrc(nrm + 2 * plane, nb)};
    const __amdgpu_buffer_rsrc_t rh = buf_rsrc(a.hard, HARD ? plane : 0u);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const unsigned e = g.ro[r + 1] + (unsigned)g.xc;
        L.z[r] = buf_f4(rz, e * 4u);
#pragma unroll
        for (int c = 0; c < 3; ++c) L.n[r][c] = NR::ld4(rn[c], e);
        L.h[r] = HARD ? __builtin_amdgcn_raw_buffer_load_b32(rh, e, 0, 0) : 0u;
    }
    const bool top = g.rp == 0, bot = g.rp == 3;
    L.hz = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int c = 0; c < 3; ++c) L.hn[c] = typename NR::raw4{};
    L.hh = 0u;
    if (top || bot) {
        const unsigned e = (top ? g.ro[0] : g.ro[3]) + (unsigned)g.xc;
        L.hz = buf_f4(rz, e * 4u);
#pragma unroll
        for (int c = 0; c < 3; ++c) L.hn[c] = NR::ld4(rn[c], e);
        if (HARD) L.hh = __builtin_amdgcn_raw_buffer_load_b32(rh, e, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            L.zs[r][sd] = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) L.ns[r][sd][c] = typename NR::raw1{};
            L.hs[r][sd] = 0u;
            // with WIDE only the block's outer columns (a wave-uniform test)
            if (!WIDE || (sd ? g.wave == 3 : g.wave == 0)) {
                const unsigned e = g.ro[r + 1] + (sd ? g.xr : g.xl);
                L.zs[r][sd] = buf_f1(rz, e * 4u);
#pragma unroll
                for (int c = 0; c < 3; ++c) L.ns[r][sd][c] = NR::ld1(rn[c], e);
                if (HARD) L.hs[r][sd] = __builtin_amdgcn_raw_buffer_load_b8(rh, e, 0, 0);
            }
        }
}

// One tile of the edge image from its loads; tile k also zeroes counter
// words 256 k .. 256 k + 255 (those below zero_n).
template <typename NT, bool HARD, bool BITS, bool WIDE>
__device__ __forceinline__ void edges_process(const EdgeArgs& a, const EdgeGeom& g, unsigned tile,
                                              const EdgeLoads<NT, HARD>& L) {
    typedef NormalRow<NT> NR;
    __shared__ uint8_t p4[4][8];
    if (a.zero && tile * 256u + threadIdx.x < a.zero_n) a.zero[tile * 256u + threadIdx.x] = 0u;
    const int t = threadIdx.x, wave = g.wave, lane = g.lane, x0 = g.x0, y0 = g.y0, cg = g.cg, rp = g.rp;
    const int xb = g.xb, yb = g.yb;
    const bool any = g.any;
    const int W = a.W, H = a.H;
    float z[4][4], n[4][4][3];
    float zs[2][2], ns[2][2][3];
    unsigned hrow[4] = {0u, L.h[0], L.h[1], 0u}, hside[2][2];
    // Rows yb - 1 .. yb + 2: a lane has its own rows yb, yb + 1; the row
    // above is the second own row of the lane 16 below (the wave's row pairs
    // are consecutive) and the row below the first own row of the lane 16
    // above, except for the wave's first and last row pair, which have the
    // wave's halo rows.  Every row of the wave is read once.
#pragma unroll
    for (int r = 1; r <= 2; ++r) {
        z[r][0] = L.z[r - 1].x;
        z[r][1] = L.z[r - 1].y;
        z[r][2] = L.z[r - 1].z;
        z[r][3] = L.z[r - 1].w;
        float t3[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) NR::cvt4(L.n[r - 1][c], t3[c]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) n[r][k][c] = t3[c][k];
    }
    const bool top = rp == 0, bot = rp == 3;
    const float hz[4] = {L.hz.x, L.hz.y, L.hz.z, L.hz.w};
    float hn[4][3];
    {
        float t3[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c) NR::cvt4(L.hn[c], t3[c]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) hn[k][c] = t3[c][k];
    }
    const unsigned hh = L.hh;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            zs[r][sd] = L.zs[r][sd];
#pragma unroll
            for (int c = 0; c < 3; ++c) ns[r][sd][c] = NR::cvt1(L.ns[r][sd][c]);
            hside[r][sd] = L.hs[r][sd];
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
    // the block's outer columns were loaded.  Otherwise every lane of a row
    // loaded them from the same address (one cache line).
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
                if (nw >= 0 && nw <= 3) {
                    const float* i = sidex[nw][1 - sd][rr + r];
                    zs[r][sd] = i[0];
                    ns[r][sd][0] = i[1];
                    ns[r][sd][1] = i[2];
                    ns[r][sd][2] = i[3];
                    hside[r][sd] = __float_as_uint(i[4]);
                }
            }
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

// One tile of the edge image: its loads, then the classification.
template <typename NT, bool HARD, bool BITS, bool WIDE>
__device__ __forceinline__ void edges_tile(const EdgeArgs& a, unsigned tile, unsigned tiles_x) {
    const EdgeGeom g = edge_geom<WIDE>(a, tile, tiles_x);
    EdgeLoads<NT, HARD> L;
    edges_load<NT, HARD, WIDE>(a, g, L);
    edges_process<NT, HARD, BITS, WIDE>(a, g, tile, L);
}

}  // namespace mr
