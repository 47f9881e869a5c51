// Shared pieces of the per-level evaluation kernels (Sec. 3.2 / 4.1): the
// mapping of a flat item index onto (level, texel) over the work lists and
// the dense coarsest level, and the view-space position of a texel.
#pragma once
#include <atomic>

#include "mr_internal.hpp"
#include "recip.hpp"

namespace mr {

// Item ranges: level j owns items [cum[j], cum[j+1]), its cnt[j] texels
// padded to a multiple of 64, so that every wave's 64 items belong to one
// level: the level index is then wave-uniform and the level's parameters
// are read with scalar loads (the padding items are skipped).  List levels
// take their length from the device counts, dense levels from dense_n.
struct ItemMap {
    unsigned cum[kMaxLevels + 1];
    unsigned cnt[kMaxLevels];
    int nlev;
};

// tiles of the dense coarsest level when EvalCommon.dense_tiles is set
constexpr int kDenseTile = 16;
__host__ __device__ __forceinline__ unsigned dense_tiles_x(int W) { return (unsigned)(W + kDenseTile - 1) / kDenseTile; }

// TILES: the dense coarsest level in 16 x 16 texel tiles even where
// c.dense_tiles is not set (the batch launch with LDS depth tiles)
template <bool TILES = false>
__device__ __forceinline__ ItemMap make_item_map(const EvalCommon& c) {
    ItemMap m;
    m.nlev = c.nlev;
    m.cum[0] = 0;
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) {
        unsigned n = 0;
        if (j < c.nlev) {
            const EvalLevel& L = c.lv[j];
            // a list never holds more entries than its level has texels
            n = L.list ? min(c.counts[L.count_idx], L.dense_n) : L.dense_n;
            if ((TILES || c.dense_tiles) && j == c.nlev - 1 && !L.list) {
                n = dense_tiles_x(L.W) * ((unsigned)(L.H + kDenseTile - 1) / kDenseTile) * 256u;
                m.cum[j] = (m.cum[j] + 255u) & ~255u;  // a chunk per tile
            }
        }
        m.cnt[j] = n;
        m.cum[j + 1] = m.cum[j] + ((n + 63u) & ~63u);
    }
    return m;
}

// total item count (cum[nlev]; the entries past nlev repeat it)
__device__ __forceinline__ unsigned item_total(const ItemMap& m) { return m.cum[kMaxLevels]; }

// level of an item: unrolled comparisons (a dynamically indexed prefix
// array would be demoted to per-thread LDS); the same for all lanes of a
// wave, which readfirstlane tells the compiler
__device__ __forceinline__ int item_level(const ItemMap& m, unsigned item) {
    int j = 0;
#pragma unroll
    for (int k = 1; k < kMaxLevels; ++k) j += (k < m.nlev && item >= m.cum[k]) ? 1 : 0;
    return __builtin_amdgcn_readfirstlane(j);
}

// item index relative to its level's first item, or ~0u for a padding item
__device__ __forceinline__ unsigned item_local(const ItemMap& m, unsigned item, int j) {
    unsigned base = 0, n = 0;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k)
        if (k == j) {
            base = m.cum[k];
            n = m.cnt[k];
        }
    const unsigned local = item - base;
    return local < n ? local : ~0u;
}

// Item chunks of 256 (neighbouring texels) are split into 8 contiguous
// regions, one per XCD (block b runs on XCD b % 8); the blocks of an XCD
// sweep its region in rounds, so that the depth rows its sample gathers touch
// stay in that XCD's L2 from one round to the next.  Grids of fewer than 8
// blocks stride over all chunks.
struct ChunkRange {
    unsigned first, end, step;
};

__device__ __forceinline__ ChunkRange chunk_range(unsigned nchunks) {
    const unsigned G = gridDim.x, b = blockIdx.x;
    if (G < 8) return {b, nchunks, G};
    const unsigned x = b & 7u, k = b >> 3;
    const unsigned per = (G - x + 7u) >> 3;  // blocks of this XCD
    const unsigned lo = (unsigned)((unsigned long long)nchunks * x / 8u);
    const unsigned hi = (unsigned)((unsigned long long)nchunks * (x + 1u) / 8u);
    return {lo + k, hi, per};
}

// Chunks of a launch's item space handed to its blocks.  Q false: each block
// takes a fixed stride of its XCD's region (chunk_range).  Q true: the blocks
// of an XCD take that region's chunks one at a time from the XCD's counter
// (queue[x], zero when the launch starts), so blocks that finish early take
// more.  Both visit every chunk exactly once.  The body must not synchronise
// the block.
template <bool Q, typename F>
__device__ __forceinline__ void for_each_chunk(unsigned nchunks, unsigned* queue, F&& body) {
    if constexpr (!Q) {
        const ChunkRange cr = chunk_range(nchunks);
        for (unsigned c = cr.first; c < cr.end; c += cr.step) body(c);
    } else {
        __shared__ unsigned next;
        const unsigned G = gridDim.x;
        unsigned x = 0, lo = 0, hi = nchunks;
        if (G >= 8) {
            x = blockIdx.x & 7u;
            lo = (unsigned)((unsigned long long)nchunks * x / 8u);
            hi = (unsigned)((unsigned long long)nchunks * (x + 1u) / 8u);
        }
        for (;;) {
            if (threadIdx.x == 0) next = lo + atomicAdd(queue + x, 1u);
            __syncthreads();
            const unsigned c = next;
            __syncthreads();
            if (c >= hi) break;
            body(c);
        }
    }
}

// Frames of one batched launch at most.
constexpr int kMaxBatch = kMaxBatchFrames;

// cbase[f] = first chunk (of `per` items, a multiple of 256) of frame f in a
// batch's item space, cbase[n] = total: each frame's item range (from its
// device counts; TILES: with the dense coarsest level in tiles) rounded up
// to whole chunks.  Computed by the first wave; ends with a barrier.
template <bool TILES = false, typename Args>
__device__ __forceinline__ void batch_chunk_bases(const Args* T, int n, unsigned per, unsigned* cbase) {
    if (threadIdx.x < 64) {
        const int f = threadIdx.x;
        unsigned cnt = 0;
        if (f < n) cnt = (item_total(make_item_map<TILES>(T[f].c)) + per - 1u) / per;
        unsigned inc = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned o = __shfl_up(inc, d, 64);
            if (f >= d) inc += o;
        }
        if (f == 0) cbase[0] = 0;
        if (f < n) cbase[f + 1] = inc;
    }
    __syncthreads();
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

// store one sub-image value (f16 storage rounds to nearest even)
__device__ __forceinline__ void store_out(const EvalLevel& L, unsigned idx, float v) {
    if (L.out16)
        reinterpret_cast<_Float16*>(L.out)[idx] = (_Float16)v;
    else if (L.stream)  // a final image: nothing in the frame reads it again
        __builtin_nontemporal_store(v, L.out + idx);
    else
        L.out[idx] = v;
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

// per-device caches of device properties: filled on first use on each
// device (with that device current), read-only afterwards; 0 = not yet
// queried.  Concurrent first uses store the same value.
constexpr int kMaxPropDevices = 64;

__host__ inline int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxPropDevices) return -1;
    return dev;
}

__host__ inline unsigned query_cus(int dev) {
    int cus = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256u;
    return (unsigned)cus;
}

// Blocks of 256 threads of `Kernel` that are resident on the current device
// at once (CUs x blocks per CU at the kernel's occupancy), queried once per
// kernel and device.
template <auto Kernel>
__host__ unsigned resident_blocks() {
    static std::atomic<unsigned> cache[kMaxPropDevices];
    const int dev = current_device();
    if (dev >= 0) {
        const unsigned v = cache[dev].load(std::memory_order_relaxed);
        if (v) return v;
    }
    int per = 0;
    unsigned n = 8192u;
    if (dev >= 0 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(Kernel), 256, 0) ==
            hipSuccess &&
        per > 0)
        n = query_cus(dev) * (unsigned)per;
    if (dev >= 0) cache[dev].store(n, std::memory_order_relaxed);
    return n;
}

// grid for a grid-stride evaluation pass over `total_hint` items at most:
// one chunk of 256 items per block, at most one resident wave of blocks
// (more blocks would only wait for a slot and repeat the per-block set-up)
template <auto Kernel>
__host__ inline unsigned eval_blocks(unsigned total_hint) {
    unsigned b = (total_hint + 255) / 256;
    const unsigned cap = resident_blocks<Kernel>();
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return b;
}

// compute units of the current device, queried once per device
__host__ inline unsigned cu_count() {
    static std::atomic<unsigned> cache[kMaxPropDevices];
    const int dev = current_device();
    if (dev < 0) return query_cus(dev);
    unsigned v = cache[dev].load(std::memory_order_relaxed);
    if (!v) {
        v = query_cus(dev);
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return v;
}

// eval_blocks capped at blocks_per_cu blocks on every CU (0: no cap)
template <auto Kernel>
__host__ inline unsigned eval_blocks_capped(unsigned total_hint, int blocks_per_cu) {
    unsigned b = eval_blocks<Kernel>(total_hint);
    if (blocks_per_cu > 0) {
        const unsigned cap = cu_count() * (unsigned)blocks_per_cu;
        if (b > cap) b = cap;
    }
    return b;
}

}  // namespace mr
