// Shared pieces of the per-level evaluation kernels (Sec. 3.2 / 4.1): the
// mapping of a flat item index onto (level, texel) over the work lists and
// the dense coarsest level, and the view-space position of a texel.
#pragma once

#include "mr_internal.hpp"

namespace mr {

// Item ranges: level j owns items [cum[j], cum[j+1]); list levels take their
// length from the device counts, dense levels from dense_n.
struct ItemMap {
    unsigned cum[kMaxLevels + 1];
    int nlev;
};

__device__ __forceinline__ ItemMap make_item_map(const EvalCommon& c) {
    ItemMap m;
    m.nlev = c.nlev;
    m.cum[0] = 0;
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) {
        unsigned n = 0;
        if (j < c.nlev) {
            // a list never holds more entries than its level has texels
            n = c.lv[j].list ? min(c.counts[c.lv[j].count_idx], c.lv[j].dense_n) : c.lv[j].dense_n;
        }
        m.cum[j + 1] = m.cum[j] + n;
    }
    return m;
}

// total item count (cum[nlev]; the entries past nlev repeat it)
__device__ __forceinline__ unsigned item_total(const ItemMap& m) { return m.cum[kMaxLevels]; }

// level of an item: unrolled comparisons (a dynamically indexed prefix
// array would be demoted to per-thread LDS)
__device__ __forceinline__ int item_level(const ItemMap& m, unsigned item) {
    int j = 0;
#pragma unroll
    for (int k = 1; k < kMaxLevels; ++k) j += (k < m.nlev && item >= m.cum[k]) ? 1 : 0;
    return j;
}

// item index relative to its level's first item
__device__ __forceinline__ unsigned item_local(const ItemMap& m, unsigned item, int j) {
    unsigned base = 0;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k)
        if (k == j) base = m.cum[k];
    return item - base;
}

// Item chunks of 256 are handed out in rounds of gridDim.x blocks; inside a
// round, block b takes chunk xcd_remap(b, n), so each XCD works through one
// contiguous run of chunks (consecutive items are neighbouring texels, and
// their sample gathers then share that XCD's L2).  Returns the first item of
// the block's chunk in round `base`, or ~0u when the block has none.
__device__ __forceinline__ unsigned chunk_of(unsigned base, unsigned nchunks) {
    const unsigned n = min(gridDim.x, nchunks - base);
    if (blockIdx.x >= n) return ~0u;
    return (base + xcd_remap(blockIdx.x, n)) * 256u;
}

// Sample sets of at most this many entries are staged in LDS once per
// workgroup; the sample loops then read them with uniform LDS addresses
// instead of a vector load (and its full wait) per sample.
constexpr int kLdsSamples = 1024;

// a_i at every listed texel: the separable blur of the dense path with the
// zero terms left out (g * 0 = +0 and acc + 0 = acc, so the sums are equal).
// The radius is a template parameter so that all 2R+1 rows' words are loaded
// in one batch.
template <int R>
__device__ __forceinline__ float alpha_at(const uint32_t* Eb, int wpr, int H, const float* g, int x, int y) {
    constexpr int N = 2 * R + 1;
    const int x0 = x - R;
    const int w0 = x0 >> 5, sh = x0 & 31;
    const bool lo_ok = w0 >= 0 && w0 < wpr, hi_ok = w0 + 1 >= 0 && w0 + 1 < wpr;
    unsigned lo[N], hi[N];
#pragma unroll
    for (int ky = 0; ky < N; ++ky) {
        const int yy = y - R + ky;
        const bool rok = yy >= 0 && yy < H;
        const uint32_t* row = Eb + (unsigned)(rok ? yy : 0) * (unsigned)wpr;
        lo[ky] = (rok && lo_ok) ? row[w0] : 0u;
        hi[ky] = (rok && hi_ok) ? row[w0 + 1] : 0u;
    }
    float a = 0.0f;
#pragma unroll
    for (int ky = 0; ky < N; ++ky) {
        unsigned m = sh ? (lo[ky] >> sh) | (hi[ky] << (32 - sh)) : lo[ky];
        m &= (1u << N) - 1u;
        if (!m) continue;
        float h = 0.0f;
        while (m) {
            const int k = __builtin_ctz(m);
            m &= m - 1;
            h = h + g[k];
        }
        a = a + g[ky] * h;
    }
    return a;
}

// blur taps of every level in LDS (the caller synchronises before use)
constexpr int kEgStride = 2 * kBlurFusedMaxRadiusC + 1;
__device__ __forceinline__ void stage_taps(const EvalCommon& c, float* eg) {
    for (int i = threadIdx.x; i < kMaxLevels * kEgStride; i += blockDim.x) {
        const int j = i / kEgStride, k = i - j * kEgStride;
        eg[i] = c.lv[j].Eg[k];
    }
}

// a_i of a listed texel for the evaluators (radius <= 8, else 0)
__device__ __forceinline__ float alpha_dispatch(const EvalLevel& L, const float* g, int x, int y) {
    switch (L.Er) {
#define MR_ALPHA(R) \
    case R: return alpha_at<R>(L.Eb, L.Ewpr, L.H, g, x, y);
        MR_ALPHA(0) MR_ALPHA(1) MR_ALPHA(2) MR_ALPHA(3) MR_ALPHA(4) MR_ALPHA(5) MR_ALPHA(6) MR_ALPHA(7) MR_ALPHA(8)
#undef MR_ALPHA
        default: return 0.0f;
    }
}

// P = (X z, Y z, -z), X = ((x + 0.5) - cx) / f, Y = (cy - (y + 0.5)) / f
__device__ __forceinline__ void view_pos(int x, int y, float z, float f, float cx, float cy,
                                         float& px, float& py, float& pz) {
    const float X = (((float)x + 0.5f) - cx) / f;
    const float Y = (cy - ((float)y + 0.5f)) / f;
    px = X * z;
    py = Y * z;
    pz = -z;
}

// Duff et al. 2017 branch-free orthonormal basis around n
__device__ __forceinline__ void onb(float nx, float ny, float nz, float& tx, float& ty, float& tz,
                                    float& bx, float& by, float& bz) {
    const float sg = copysignf(1.0f, nz);
    const float a = -1.0f / (sg + nz);
    const float b = (nx * ny) * a;
    tx = 1.0f + ((sg * (nx * nx)) * a);
    ty = sg * b;
    tz = -(sg * nx);
    bx = b;
    by = sg + ((ny * ny) * a);
    bz = -ny;
}

// whether any level has the evaluator write a_i (selects the kernel instance
// that carries the blur code, so that the others keep their register budget)
__host__ inline bool fused_alpha(const EvalCommon& c) {
    for (int j = 0; j < c.nlev; ++j)
        if (c.lv[j].ac) return true;
    return false;
}

// grid for a grid-stride evaluation pass over `total_hint` items at most
__host__ inline unsigned eval_blocks(unsigned total_hint) {
    unsigned b = (total_hint + 255) / 256;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return b;
}

}  // namespace mr
