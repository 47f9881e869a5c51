// Mask creation kernels: edge image with fused OR-downsampling (Sec. 3.1),
// separable Gaussian blur with the Table 1 variances and stencil = mask > 0
// (Sec. 3.1, Sec. 4.1), nesting of the inclusive levels and the owner-level
// map.
#include "edges_tile.hpp"
#include "mr_internal.hpp"

namespace mr {

// ---------------------------------------------------------------------------
// edge image + pooling.  One workgroup = 64 x 32 pixel tile (aligned to every
// pooling block up to s = 32), 256 threads.  The tile and a one-pixel halo of
// depth and normals (and shadow bits) are staged in LDS with 16-byte loads,
// then every thread classifies a 4 x 2 pixel block, ORs it to the level-2
// texels in registers and the coarser levels through LDS.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void row4(const T* p, unsigned off, bool vec, int n, float* o);

template <>
__device__ __forceinline__ void row4<float>(const float* p, unsigned off, bool vec, int n, float* o) {
    if (vec) {
        const float4 v = *reinterpret_cast<const float4*>(p + off);
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    } else {
        for (int k = 0; k < 4; ++k) o[k] = k < n ? p[off + k] : 0.0f;
    }
}

template <>
__device__ __forceinline__ void row4<_Float16>(const _Float16* p, unsigned off, bool vec, int n, float* o) {
    if (vec) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        const h4 v = *reinterpret_cast<const h4*>(p + off);
        o[0] = (float)v.x;
        o[1] = (float)v.y;
        o[2] = (float)v.z;
        o[3] = (float)v.w;
    } else {
        for (int k = 0; k < 4; ++k) o[k] = k < n ? (float)p[off + k] : 0.0f;
    }
}

// One workgroup = 64 x 32 pixel tile (aligned to every pooling block up to
// s = 32), 256 threads; a thread owns a 4 x 2 pixel block and loads it with a
// one-pixel ring straight from memory (rows above and below and the side
// columns are shared with neighbouring threads through L1/L2), so no LDS
// staging limits occupancy.  Each normal pair is tested once.  Level 2 is
// ORed in registers, levels 3 and 4 with lane shuffles, 5 and 6 through LDS.
template <typename NT>
__global__ __launch_bounds__(256) void k_edges_generic(EdgeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ uint8_t p4[4][8];
    const unsigned tile = xcd_remap(blockIdx.x, ntiles);
    if (a.zero && tile * 256u + threadIdx.x < a.zero_n) a.zero[tile * 256u + threadIdx.x] = 0u;
    const int x0 = (int)(tile % tiles_x) * kEdgeTW;
    const int y0 = (int)(tile / tiles_x) * kEdgeTH;
    const int W = a.W, H = a.H;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int cg = lane & 15, rp = lane >> 4;
    const int xb = x0 + 4 * cg, yb = y0 + 8 * wave + 2 * rp;
    const unsigned plane = (unsigned)W * (unsigned)H;
    const NT* nrm = static_cast<const NT*>(a.normal);
    const bool has_hard = a.hard != nullptr;
    const bool any = xb < W && yb < H;
    const int ncol = min(4, W - xb);
    const bool vec = ((W & 3) == 0) && ncol == 4;

    // ---- loads: rows yb-1 .. yb+2 (index 0..3), columns xb .. xb+3, and the
    // side columns xb-1 / xb+4 of rows yb, yb+1 ----
    float z[4][4], n[4][4][3];
    float zs[2][2], ns[2][2][3];  // [row][left/right]
    uint8_t h[4][4], hs[2][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int y = yb - 1 + r;
        const bool rok = any && y >= 0 && y < H;
        float tz[4] = {0, 0, 0, 0}, t0[4] = {0, 0, 0, 0}, t1[4] = {0, 0, 0, 0}, t2[4] = {0, 0, 0, 0};
        uint8_t th[4] = {0, 0, 0, 0};
        if (rok) {
            const unsigned off = (unsigned)y * (unsigned)W + (unsigned)xb;
            row4<float>(a.depth, off, vec, ncol, tz);
            row4<NT>(nrm, off, vec, ncol, t0);
            row4<NT>(nrm + plane, off, vec, ncol, t1);
            row4<NT>(nrm + 2 * plane, off, vec, ncol, t2);
            if (has_hard) {
                if (vec) {
                    const uchar4 v = *reinterpret_cast<const uchar4*>(a.hard + off);
                    th[0] = v.x;
                    th[1] = v.y;
                    th[2] = v.z;
                    th[3] = v.w;
                } else {
                    for (int k = 0; k < ncol; ++k) th[k] = a.hard[off + k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            z[r][k] = tz[k];
            n[r][k][0] = t0[k];
            n[r][k][1] = t1[k];
            n[r][k][2] = t2[k];
            h[r][k] = th[k];
        }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int y = yb + r;
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const int x = sd ? xb + 4 : xb - 1;
            zs[r][sd] = 0.0f;
            ns[r][sd][0] = ns[r][sd][1] = ns[r][sd][2] = 0.0f;
            hs[r][sd] = 0;
            if (any && y < H && x >= 0 && x < W) {
                const unsigned off = (unsigned)y * (unsigned)W + (unsigned)x;
                zs[r][sd] = a.depth[off];
                ns[r][sd][0] = ld(nrm, off);
                ns[r][sd][1] = ld(nrm, plane + off);
                ns[r][sd][2] = ld(nrm, 2 * plane + off);
                if (has_hard) hs[r][sd] = a.hard[off];
            }
        }
    }

    // ---- normal pair tests, each pair once ----
    const float cn = a.normal_cos, td = a.depth_ratio;
    bool hp[2][5];  // row r: pair (c-1, c), c = 0..4
    bool vp[3][4];  // column c: pair (row k, row k+1)
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

    // ---- classify the 8 pixels ----
    uint8_t e[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int y = yb + r;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int x = xb + c;
            const float zc = z[r + 1][c];
            const float zl = c > 0 ? z[r + 1][c - 1] : zs[r][0];
            const float zr = c < 3 ? z[r + 1][c + 1] : zs[r][1];
            const float zu = z[r][c], zd = z[r + 2][c];
            const bool hl = x > 0, hr = x < W - 1, hu = y > 0, hd = y < H - 1;
            bool ed = (hl && !valid_depth(zl)) || (hr && !valid_depth(zr)) || (hu && !valid_depth(zu)) ||
                      (hd && !valid_depth(zd));
            const float thr = td * zc;
            const float two_z = 2.0f * zc;
            ed = ed || (hl && hr && fabsf((zl + zr) - two_z) > thr);
            ed = ed || (hu && hd && fabsf((zu + zd) - two_z) > thr);
            ed = ed || (hl && hp[r][c]) || (hr && hp[r][c + 1]) || (hu && vp[r][c]) || (hd && vp[r + 1][c]);
            if (has_hard) {
                const uint8_t hc = h[r + 1][c];
                const uint8_t hl_ = c > 0 ? h[r + 1][c - 1] : hs[r][0];
                const uint8_t hr_ = c < 3 ? h[r + 1][c + 1] : hs[r][1];
                ed = ed || (hl && hl_ != hc) || (hr && hr_ != hc) || (hu && h[r][c] != hc) ||
                     (hd && h[r + 2][c] != hc);
            }
            e[r][c] = (any && x < W && y < H && fovea(a, x, y, valid_depth(zc) && ed)) ? 1 : 0;
        }
    }
    if (any) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = yb + r;
            if (y >= H) continue;
            const unsigned off = (unsigned)y * (unsigned)W + (unsigned)xb;
            if (vec)
                *reinterpret_cast<uchar4*>(a.E + off) = make_uchar4(e[r][0], e[r][1], e[r][2], e[r][3]);
            else
                for (int k = 0; k < ncol; ++k) a.E[off + k] = e[r][k];
        }
        // point-sampled level depth: z_i(X, Y) = z(s X + s/2, s Y + s/2)
        for (int i = 2; i <= a.num_levels; ++i) {
            float* zi = a.zi[i - 1];
            if (!zi) continue;
            const int sh = i - 1, s = 1 << sh, hf = s >> 1;
            const unsigned wi = (unsigned)a.Wi[i - 1];
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int x = xb + c, y = yb + r;
                    if (x < W && y < H && (x & (s - 1)) == hf && (y & (s - 1)) == hf)
                        zi[(unsigned)(y >> sh) * wi + (unsigned)(x >> sh)] = z[r + 1][c];
                }
        }
    }
    // ---- pooled edges ----
    // level 2: texels (xb/2 + j, yb/2), in registers
    if (any && a.Ei[1]) {
        const unsigned off = (unsigned)(yb >> 1) * (unsigned)a.Wi[1] + (unsigned)(xb >> 1);
        a.Ei[1][off] = e[0][0] | e[0][1] | e[1][0] | e[1][1];
        if (ncol > 2) a.Ei[1][off + 1] = e[0][2] | e[0][3] | e[1][2] | e[1][3];
    }
    // level 3: 4 x 4 = this thread and the one below (lane + 16)
    int v = e[0][0] | e[0][1] | e[0][2] | e[0][3] | e[1][0] | e[1][1] | e[1][2] | e[1][3];
    v |= __shfl_xor(v, 16, 64);
    if (any && a.Ei[2] && (rp & 1) == 0)
        a.Ei[2][(unsigned)(yb >> 2) * (unsigned)a.Wi[2] + (unsigned)(xb >> 2)] = (uint8_t)v;
    // level 4: 8 x 8 = pairs of column groups and the other row pair
    v |= __shfl_xor(v, 1, 64);
    v |= __shfl_xor(v, 32, 64);
    if (any && a.Ei[3] && (cg & 1) == 0 && rp == 0)
        a.Ei[3][(unsigned)(yb >> 3) * (unsigned)a.Wi[3] + (unsigned)(xb >> 3)] = (uint8_t)v;
    if (a.num_levels >= 5) {
        // levels 5 and 6 combine the waves' 8 x 8 blocks through LDS
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



template <typename NT, bool HARD, bool BITS, bool WIDE>
__global__ __launch_bounds__(256) void k_edges_vec(EdgeArgs a, unsigned tiles_x, unsigned ntiles) {
    edges_tile<NT, HARD, BITS, WIDE>(a, xcd_remap(blockIdx.x, ntiles), tiles_x);
}

// Frames of a batch: one grid over all frames' tiles (tile_base[f] = first
// tile of frame f, tile_base[n] = total); tiles_x[f] per frame.  The frame
// tables of a batch launch are never written while it runs: __restrict__ on
// them (here and in the other batch kernels) lets the compiler keep a frame's
// fields in registers across the kernel's own stores instead of loading them
// again after each (the batch edge kernel ran 18 % faster with it).
template <typename NT, bool HARD, bool BITS, bool WIDE>
__global__ __launch_bounds__(256) void k_edges_batch(const EdgeArgs* __restrict__ T,
                                                     const unsigned* __restrict__ tile_base,
                                                     const unsigned* __restrict__ tiles_x, int n, unsigned* queue) {
    if (blockIdx.x == 0 && threadIdx.x < kBatchCounters) queue[threadIdx.x] = 0u;
    const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
    int f = 0;
    for (int k = 1; k < n; ++k) f += g >= tile_base[k] ? 1 : 0;
    const unsigned local = g - tile_base[f];
    edges_tile<NT, HARD, BITS, WIDE>(T[f], local, tiles_x[f]);
}

hipError_t launch_edges_batch(const EdgeArgs* T, const unsigned* tile_base, const unsigned* tiles_x, int n,
                              unsigned total, int normal_dtype, bool hard, bool wide, unsigned* queue,
                              hipStream_t s) {
    // compact frame path only: bit-packed edges (BITS) and widths divisible by 4
#define MR_EB(NT, HD, WD)                                                                                  \
    hipLaunchKernelGGL((k_edges_batch<NT, HD, true, WD>), dim3(total), dim3(256), 0, s, T, tile_base, tiles_x, n, \
                       queue)
    const bool f16 = normal_dtype == MR_F16;
    if (wide) {
        if (f16 && hard) MR_EB(_Float16, true, true);
        else if (f16) MR_EB(_Float16, false, true);
        else if (hard) MR_EB(float, true, true);
        else MR_EB(float, false, true);
    } else {
        if (f16 && hard) MR_EB(_Float16, true, false);
        else if (f16) MR_EB(_Float16, false, false);
        else if (hard) MR_EB(float, true, false);
        else MR_EB(float, false, false);
    }
#undef MR_EB
    return hipGetLastError();
}

void edges_grid(int W, int H, int num_levels, bool& wide, unsigned& tiles_x, unsigned& ntiles) {
    wide = num_levels <= 4;
    edges_tiles(W, H, wide, tiles_x, ntiles);
}

void edges_tiles(int W, int H, bool wide, unsigned& tiles_x, unsigned& ntiles) {
    if (wide) {
        tiles_x = (unsigned)((W + 4 * kEdgeTW - 1) / (4 * kEdgeTW));
        ntiles = tiles_x * (unsigned)((H + 7) / 8);
    } else {
        tiles_x = (unsigned)((W + kEdgeTW - 1) / kEdgeTW);
        ntiles = tiles_x * (unsigned)((H + kEdgeTH - 1) / kEdgeTH);
    }
}

hipError_t launch_edges(const EdgeArgs& a, int normal_dtype, hipStream_t s) {
    const unsigned tx = (a.W + kEdgeTW - 1) / kEdgeTW, ty = (a.H + kEdgeTH - 1) / kEdgeTH;
    const unsigned n = tx * ty;
    const bool f16 = normal_dtype == MR_F16, hard = a.hard != nullptr, bits = a.Eb[0] != nullptr;
    if ((a.W & 3) == 0 && a.W >= 4) {
        const bool wide = a.num_levels <= 4;
        const unsigned wx = (a.W + 4 * kEdgeTW - 1) / (4 * kEdgeTW), wy = (a.H + 7) / 8;
#define MR_EDGES(NT, HD, BT)                                                                                 \
    do {                                                                                                     \
        if (wide)                                                                                            \
            hipLaunchKernelGGL((k_edges_vec<NT, HD, BT, true>), dim3(wx * wy), dim3(256), 0, s, a, wx, wx * wy); \
        else                                                                                                 \
            hipLaunchKernelGGL((k_edges_vec<NT, HD, BT, false>), dim3(n), dim3(256), 0, s, a, tx, n);        \
    } while (0)
        if (bits) {
            if (f16 && hard) MR_EDGES(_Float16, true, true);
            else if (f16) MR_EDGES(_Float16, false, true);
            else if (hard) MR_EDGES(float, true, true);
            else MR_EDGES(float, false, true);
        } else {
            if (f16 && hard) MR_EDGES(_Float16, true, false);
            else if (f16) MR_EDGES(_Float16, false, false);
            else if (hard) MR_EDGES(float, true, false);
            else MR_EDGES(float, false, false);
        }
#undef MR_EDGES
    } else if (f16) {
        hipLaunchKernelGGL(k_edges_generic<_Float16>, dim3(n), dim3(256), 0, s, a, tx, n);
    } else {
        hipLaunchKernelGGL(k_edges_generic<float>, dim3(n), dim3(256), 0, s, a, tx, n);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// separable blur of every level below the coarsest in one launch.  A
// workgroup owns 256 columns x 32 rows of one level: the edge bytes of the
// tile plus its halo are staged in LDS in one batch, then each thread walks
// down its column keeping the last 2r+1 horizontal sums in a register shift
// ring, so every output needs one new horizontal sum.
// h(x, y) = sum_k g[k] E(x + k, y) then a(x, y) = sum_k g[k] h(x, y + k), taps
// in ascending k, accumulators from +0, zero outside the image; S = a > 0.
// Terms with E = 0 contribute g * 0 = +0, so h adds g[k] exactly for the set
// taps.
// ---------------------------------------------------------------------------
constexpr int kBlurTW = 256, kBlurTH = 32;
constexpr int kBlurLW = kBlurTW + 2 * kMaxRadius;  // staged row stride (bytes)

template <int R>
__device__ __forceinline__ float hsum(const uint8_t* row, const float* g) {
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) acc = acc + g[k] * (row[k] ? 1.0f : 0.0f);
    return acc;
}

template <int R>
__device__ __forceinline__ void blur_columns(const BlurLevel& a, const uint8_t* es, int x0, int y0) {
    const int t = threadIdx.x;
    const int X = x0 + t;
    const int W = a.W, H = a.H;
    float g[2 * R + 1];
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) g[k] = a.g[k];
    // staged row yy holds image row y0 - R + yy, column t + k holds x0 - R + t + k
    float ring[2 * R + 1];
    ring[0] = 0.0f;
#pragma unroll
    for (int yy = 0; yy < 2 * R; ++yy) ring[yy + 1] = hsum<R>(es + yy * kBlurLW + t, g);
    const bool colok = X < W;
    const int rows = min(kBlurTH, H - y0);
    for (int oy = 0; oy < rows; ++oy) {
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) ring[k] = ring[k + 1];
        ring[2 * R] = hsum<R>(es + (oy + 2 * R) * kBlurLW + t, g);
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k <= 2 * R; ++k) acc = acc + g[k] * ring[k];
        if (colok) {
            const long long p = (long long)(y0 + oy) * W + X;
            a.a[p] = acc;
            a.S[p] = acc > 0.0f ? 1 : 0;
        }
    }
}

// Stage the tile's edge bytes (rows y0 - r .. y0 + 31 + r, columns
// x0 - r .. x0 + 255 + r) into LDS with all global loads issued first.
__device__ __forceinline__ void blur_stage(const BlurLevel& a, uint8_t* es, int x0, int y0) {
    const int r = a.r, W = a.W, H = a.H, t = threadIdx.x;
    const int eh = kBlurTH + 2 * r;
    const bool vec = (W & 3) == 0;
    constexpr int kWords = kBlurTW / 4;
    constexpr int kMaxSlots = ((kBlurTH + 2 * kMaxRadius) * kWords + 255) / 256;
    uchar4 v[kMaxSlots];
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) {
        const int idx = t + 256 * j;
        const int yy = idx / kWords, q = idx % kWords;
        const int Y = y0 - r + yy, X = x0 + 4 * q;
        v[j] = make_uchar4(0, 0, 0, 0);
        if (yy < eh && Y >= 0 && Y < H && X < W) {
            const long long p = (long long)Y * W + X;
            if (vec) {
                v[j] = *reinterpret_cast<const uchar4*>(a.Ei + p);
            } else {
                uint8_t e4[4] = {0, 0, 0, 0};
                for (int k = 0; k < 4 && X + k < W; ++k) e4[k] = a.Ei[p + k];
                v[j] = make_uchar4(e4[0], e4[1], e4[2], e4[3]);
            }
        }
    }
    // side halos: r columns on each side, at most (32 + 2*16) * 2*16 = 2048 bytes
    constexpr int kHaloSlots = (kBlurTH + 2 * kMaxRadius) * 2 * kMaxRadius / 256;
    uint8_t hb[kHaloSlots];
#pragma unroll
    for (int j = 0; j < kHaloSlots; ++j) {
        hb[j] = 0;
        const int idx = t + 256 * j;
        if (idx >= eh * 2 * r) continue;
        const int yy = idx / (2 * r), jj = idx % (2 * r);
        const int xx = jj < r ? jj : kBlurTW + jj;
        const int X = x0 - r + xx, Y = y0 - r + yy;
        if (X >= 0 && X < W && Y >= 0 && Y < H) hb[j] = a.Ei[(long long)Y * W + X];
    }
#pragma unroll
    for (int j = 0; j < kMaxSlots; ++j) {
        const int idx = t + 256 * j;
        const int yy = idx / kWords, q = idx % kWords;
        if (yy >= eh) continue;
        uint8_t* d = es + yy * kBlurLW + r + 4 * q;
        d[0] = v[j].x;
        d[1] = v[j].y;
        d[2] = v[j].z;
        d[3] = v[j].w;
    }
#pragma unroll
    for (int j = 0; j < kHaloSlots; ++j) {
        const int idx = t + 256 * j;
        if (idx >= eh * 2 * r) continue;
        const int yy = idx / (2 * r), jj = idx % (2 * r);
        const int xx = jj < r ? jj : kBlurTW + jj;
        es[yy * kBlurLW + xx] = hb[j];
    }
    __syncthreads();
}

// radius <= 8: every such level of the frame in one launch.  Tiles of all
// levels share one index range; the plain block order spreads the costlier
// coarse-level tiles over all XCDs.
__global__ __launch_bounds__(256) void k_blur(BlurArgs A) {
    __shared__ uint8_t es[(kBlurTH + 2 * kMaxRadius) * kBlurLW];
    const unsigned b = blockIdx.x;
    int l = 0;
    while (l + 1 < A.nlev && b >= A.lv[l + 1].tile_base) ++l;
    const BlurLevel& a = A.lv[l];
    const unsigned tile = b - a.tile_base;
    const int x0 = (int)(tile % a.tiles_x) * kBlurTW;
    const int y0 = (int)(tile / a.tiles_x) * kBlurTH;
    blur_stage(a, es, x0, y0);
    const int r = a.r;
    switch (r) {
#define MR_BLUR_CASE(R) \
    case R: blur_columns<R>(a, es, x0, y0); break;
        MR_BLUR_CASE(0) MR_BLUR_CASE(1) MR_BLUR_CASE(2) MR_BLUR_CASE(3) MR_BLUR_CASE(4) MR_BLUR_CASE(5)
        MR_BLUR_CASE(6) MR_BLUR_CASE(7) MR_BLUR_CASE(8)
#undef MR_BLUR_CASE
        default: break;
    }
}

// radius 9..16: one launch per level, radius fixed at compile time
template <int R>
__global__ __launch_bounds__(256) void k_blur_wide(BlurLevel a) {
    __shared__ uint8_t es[(kBlurTH + 2 * kMaxRadius) * kBlurLW];
    const unsigned tile = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (int)(tile % a.tiles_x) * kBlurTW;
    const int y0 = (int)(tile / a.tiles_x) * kBlurTH;
    blur_stage(a, es, x0, y0);
    blur_columns<R>(a, es, x0, y0);
}

hipError_t launch_blur_wide(const BlurLevel& a, hipStream_t s) {
    const unsigned n = a.tiles_x * (unsigned)((a.H + kBlurTH - 1) / kBlurTH);
    switch (a.r) {
#define MR_BLUR_WIDE(R) \
    case R: hipLaunchKernelGGL(k_blur_wide<R>, dim3(n), dim3(256), 0, s, a); break;
        MR_BLUR_WIDE(9) MR_BLUR_WIDE(10) MR_BLUR_WIDE(11) MR_BLUR_WIDE(12) MR_BLUR_WIDE(13) MR_BLUR_WIDE(14)
        MR_BLUR_WIDE(15) MR_BLUR_WIDE(16)
#undef MR_BLUR_WIDE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_blur(const BlurArgs& a, hipStream_t s) {
    if (a.nlev == 0 || a.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blur, dim3(a.ntiles), dim3(256), 0, s, a);
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
