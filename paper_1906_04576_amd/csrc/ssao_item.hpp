// SSAO evaluated per sub-image (Sec. 3.2 / 4.1) and as the naive full-res
// pass (Sec. 5).  The paper cites Mittring 2007 and Bavoil et al. 2008 for
// SSAO without printing an estimator; this one is a normal-oriented
// hemisphere with a fixed caller-supplied kernel, a hard range check and a
// relative depth bias; output = occluded fraction.
#pragma once
#include "eval_common.hpp"

namespace mr {


// Occluding samples of one texel.  Branch-free: every sample computes its
// projection and gathers (a texel of the depth plane also when it is
// off-screen or behind the eye), and counts only if all tests pass; the
// count is the same as skipping the sample.  Samples go in groups of G
// whose gathers are issued back to back, so that several are in flight per
// wave.  FAST: 1/d by recip_fast, which the caller has shown to equal
// 1.0f / d for every sample of the texel.
struct SsaoTexel {
    float px, py, pz, z;
    float rtx, rty, rtz, rbx, rby, rbz, rnx, rny, rnz;
};

// group sizes (measured): the naive pass over every pixel, and the
// multi-resolution launches, whose lists are shorter and whose blocks also
// compute a_i
constexpr int kGroupPlain = 8, kGroupMulti = 2;

// off: offset of the sample's texel in the depth plane, in bytes when CLAMP,
// else in elements (element pitches zpy, zpx; last = byte offset of the
// plane's last texel).  Two exact forms:
// CLAMP tests 0 <= u < W and 0 <= v < H as unsigned compares of the bit
// patterns and gathers at whatever offset an off-screen sample gives (the
// depth plane is a buffer resource: past its end a load returns 0 without
// an access), five instructions fewer per sample than selecting texel 0 off
// screen; with groups of 8 samples in flight the second form keeps register
// use at full occupancy (measured).
template <bool FAST, bool CLAMP, typename KP>
__device__ __forceinline__ void ssao_project(const EvalLevel& L, KP K, int s, const SsaoTexel& T, unsigned zpy,
                                             unsigned zpx, unsigned last, bool& on, float& d, unsigned& off,
                                             unsigned& sx, unsigned& sy) {
    const float Wf = (float)L.W, Hf = (float)L.H;
    const float kx = K[3 * s], ky = K[3 * s + 1], kz = K[3 * s + 2];
    const float qz = ((T.pz + kx * T.rtz) + ky * T.rbz) + kz * T.rnz;
    d = -qz;
    const float qx = ((T.px + kx * T.rtx) + ky * T.rbx) + kz * T.rnx;
    const float qy = ((T.py + kx * T.rty) + ky * T.rby) + kz * T.rny;
    const float inv = FAST ? recip_fast(d) : 1.0f / d;
    const float u = L.cx + (qx * inv) * L.f;
    const float v = L.cy - (qy * inv) * L.f;
    if (CLAMP) {
        // exact for every u other than -0: u = cx + t and v = cy - t' are
        // never -0 because cx, cy > 0 (a sum is -0 only when both terms are).
        // FAST: every d of the texel is at least 2^-126, so d > 0 holds.
        on = (FAST || d > 0.0f) & (__float_as_uint(u) < __float_as_uint(Wf)) &
             (__float_as_uint(v) < __float_as_uint(Hf));
        // u, v >= 0 when on, so truncation is floor.  Coordinates < 2^14 and
        // byte pitches < 2^22 fit the 24-bit products, so on screen the
        // offset is the texel's.  Off screen it is any value: the buffer
        // resource returns 0 past the plane and no access faults, and the
        // value is not used.
        sx = (unsigned)cvt_i32_sat(u);
        sy = (unsigned)cvt_i32_sat(v);
        off = (unsigned)__umul24(sy, 4u * zpy) + (unsigned)__umul24(sx, 4u * zpx);
        (void)last;
    } else {
        on = (FAST || d > 0.0f) & (u >= 0.0f) & (u < Wf) & (v >= 0.0f) & (v < Hf);
        // u, v >= 0 when on, so truncation is floor; rows < 2^14 and pitches
        // < 2^20 keep the offset products within 24 bits
        sx = (unsigned)(int)(on ? u : 0.0f);
        sy = (unsigned)(int)(on ? v : 0.0f);
        off = __umul24(sy, zpy) + __umul24(sx, zpx);
    }
}

// A staged copy of the level depth around a tile: tw x tw texels from
// (x0, y0), in LDS.  TILE: a sample whose texel lies in it reads it there,
// the others read the depth plane.
struct DepthTile {
    const float* t;
    unsigned x0, y0, tw;
};

// Gathers of a group of G samples are issued together, one projection at a
// time (sched_barrier: interleaving the projections buys little ILP and costs
// registers, i.e. occupancy); the group size sets how many gathers of a wave
// are in flight.
template <bool FAST, int G, bool TILE = false, typename SA, typename KP>
__device__ __forceinline__ int ssao_count(const SA& a, const EvalLevel& L, KP K, const SsaoTexel& T,
                                          const DepthTile& dt = DepthTile{}) {
    constexpr bool CLAMP = G <= 2;
    const float r = a.r, b = a.b;
    const int S = a.S;
    // L is wave-uniform here: the depth plane is a buffer resource
    const unsigned zpy = (unsigned)L.zpy, zpx = (unsigned)L.zpx;
    const unsigned last = ((unsigned)(L.H - 1) * zpy + (unsigned)(L.W - 1) * zpx) * 4u;
    const __amdgpu_buffer_rsrc_t rz = buf_rsrc(L.z, last + 4u);
    // z_s <= 0 must not count; +inf and NaN fail the depth test
    auto occluded = [&](bool on, float d, float zs) {
        return (on & (zs > 0.0f) & (zs < d - (b * d)) & (fabsf(T.z - zs) < r)) ? 1 : 0;
    };
    auto gather = [&](unsigned sx, unsigned sy, unsigned off) -> float {
        if constexpr (TILE) {
            const unsigned dx = sx - dt.x0, dy = sy - dt.y0;
            if ((dx < dt.tw) & (dy < dt.tw)) return dt.t[dy * dt.tw + dx];
        }
        return buf_f1(rz, CLAMP ? off : off * 4u);
    };
    int occ = 0;
    int s = 0;
    for (; s + G <= S; s += G) {
        bool on[G];
        float d[G], zs[G];
        unsigned off[G], sx[G], sy[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            ssao_project<FAST, CLAMP>(L, K, s + k, T, zpy, zpx, last, on[k], d[k], off[k], sx[k], sy[k]);
            // one projection at a time: interleaving them buys little ILP
            // and costs registers (occupancy)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < G; ++k) zs[k] = gather(sx[k], sy[k], off[k]);
#pragma unroll
        for (int k = 0; k < G; ++k) occ += occluded(on[k], d[k], zs[k]);
    }
    for (; s < S; ++s) {
        bool on;
        float d;
        unsigned off, sx, sy;
        ssao_project<FAST, CLAMP>(L, K, s, T, zpy, zpx, last, on, d, off, sx, sy);
        occ += occluded(on, d, gather(sx, sy, off));
    }
    return occ;
}

// occlusion of one texel; K points to LDS (staged samples) or global memory;
// kmax = the largest |component| over the samples (+inf when unknown); a
// holds the sampling parameters r, b and S (SsaoArgs or SsaoSampling)
template <typename NT, int G, bool TILE = false, typename SA, typename KP>
__device__ __forceinline__ float ssao_texel(const SA& a, const EvalLevel& L, const NT* nrm, unsigned plane,
                                            KP K, float kmax, int x, int y, float z,
                                            const DepthTile& dt = DepthTile{}) {
    const float r = a.r;
    const unsigned g = (unsigned)L.goff + (unsigned)y * (unsigned)L.gpy + (unsigned)x * (unsigned)L.gpx;
    const float nx = ld(nrm, g), ny = ld(nrm, plane + g), nz = ld(nrm, 2 * plane + g);
    SsaoTexel T;
    T.z = z;
    view_pos(x, y, z, L.f, L.cx, L.cy, T.px, T.py, T.pz);
    float tx, ty, tz, bx, by, bz;
    onb(nx, ny, nz, tx, ty, tz, bx, by, bz);
    T.rtx = r * tx, T.rty = r * ty, T.rtz = r * tz;
    T.rbx = r * bx, T.rby = r * by, T.rbz = r * bz;
    T.rnx = r * nx, T.rny = r * ny, T.rnz = r * nz;
    // Every sample's d = z - (kx rtz + ky rbz + kz rnz) (rounded) lies within
    // B0 = kmax (|rtz| + |rbz| + |rnz|) of z, up to a relative 2^-21; with
    // these margins all d are in [2^-126, 2^126), where recip_fast is exact.
    const float B0 = kmax * ((fabsf(T.rtz) + fabsf(T.rbz)) + fabsf(T.rnz));
    const bool safe = (z * 0.999f > B0 * 1.001f + 1e-37f) && ((z + B0) * 1.001f < 0x1p125f);
    const int occ =
        __ballot(!safe) == 0 ? ssao_count<true, G, TILE>(a, L, K, T, dt) : ssao_count<false, G, TILE>(a, L, K, T, dt);
    return (float)occ / (float)a.S;
}

// one item (a listed texel, or a texel of a dense level)
template <typename NT, bool KLDS, bool AL>
__device__ __forceinline__ void ssao_item(const SsaoArgs& a, const ItemMap& m, unsigned item, const float* ks,
                                          const float* eg, float kmax) {
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const unsigned plane = (unsigned)a.c.plane;
    const int j = item_level(m, item);
    const EvalLevel& L = a.c.lv[j];
    const unsigned local = item_local(m, item, j);
    if (local == ~0u) return;  // padding of the level's item range
    const unsigned t = L.list ? L.list[local] : local;
    if (t >= L.dense_n) return;  // malformed list entry
    const int y = (int)(t / (unsigned)L.W), x = (int)(t - (unsigned)y * (unsigned)L.W);
    if (AL && L.ac) L.ac[local] = alpha_dispatch(L, eg + j * kEgStride, x, y);
    const float z = L.z[(unsigned)y * L.zpy + (unsigned)x * L.zpx];
    float res = 0.0f;
    if (valid_depth(z)) {
        if (KLDS)
            res = ssao_texel<NT, AL ? kGroupMulti : kGroupPlain>(a, L, nrm, plane, ks, kmax, x, y, z);
        else
            res = ssao_texel<NT, AL ? kGroupMulti : kGroupPlain>(a, L, nrm, plane, a.kernel, kmax, x, y, z);
    }
    store_out(L, L.compact ? local : (unsigned)y * (unsigned)L.W + (unsigned)x, res);
}

template <typename NT, bool KLDS, bool AL>
__device__ __forceinline__ void ssao_items(const SsaoArgs& a, const float* ks, const float* eg, float kmax) {
    const ItemMap m = make_item_map(a.c);
    const unsigned total = item_total(m);
    const ChunkRange cr = chunk_range((total + 255) / 256);
    for (unsigned c = cr.first; c < cr.end; c += cr.step) {
        const unsigned item = c * 256u + threadIdx.x;
        if (item < total) ssao_item<NT, KLDS, AL>(a, m, item, ks, eg, kmax);
    }
}

// The multi-resolution evaluation with the dense coarsest level in 16 x 16
// texel tiles, each with a halo of H texels of its depth staged in LDS (zt,
// (16 + 2H)^2 floats) before its texels' samples gather: the samples that
// land in the staged square read it there.  Values outside the level are
// staged clamped; only off-screen samples, which never count, can reach
// them.  The list levels' chunks run as in ssao_items.
template <typename NT, int H>
__device__ __forceinline__ void ssao_items_tiled(const SsaoArgs& a, const float* ks, const float* eg, float kmax,
                                                 float* zt) {
    constexpr int TW = kDenseTile + 2 * H;
    const ItemMap m = make_item_map(a.c);
    const unsigned total = item_total(m);
    const int jd = m.nlev - 1;  // the dense coarsest level
    unsigned dense0 = 0;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) dense0 = k == jd ? m.cum[k] : dense0;
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const unsigned plane = (unsigned)a.c.plane;
    const ChunkRange cr = chunk_range((total + 255) / 256);
    for (unsigned c = cr.first; c < cr.end; c += cr.step) {
        if (c * 256u < dense0) {
            const unsigned item = c * 256u + threadIdx.x;
            if (item < total) ssao_item<NT, true, true>(a, m, item, ks, eg, kmax);
            continue;
        }
        const EvalLevel& L = a.c.lv[jd];
        const unsigned tile = c - dense0 / 256u, tx = dense_tiles_x(L.W);
        const int x0 = (int)(tile % tx) * kDenseTile, y0 = (int)(tile / tx) * kDenseTile;
        for (int i = threadIdx.x; i < TW * TW; i += 256) {
            const int ry = i / TW, rx = i - ry * TW;
            const int gx = min(max(x0 - H + rx, 0), L.W - 1), gy = min(max(y0 - H + ry, 0), L.H - 1);
            zt[i] = L.z[(unsigned)gy * (unsigned)L.zpy + (unsigned)gx * (unsigned)L.zpx];
        }
        __syncthreads();
        const int x = x0 + (int)(threadIdx.x % kDenseTile), y = y0 + (int)(threadIdx.x / kDenseTile);
        if (x < L.W && y < L.H) {
            const float z = zt[(y - y0 + H) * TW + (x - x0 + H)];
            float res = 0.0f;
            if (valid_depth(z)) {
                const DepthTile dt{zt, (unsigned)(x0 - H), (unsigned)(y0 - H), (unsigned)TW};
                res = ssao_texel<NT, kGroupMulti, true>(a, L, nrm, plane, ks, kmax, x, y, z, dt);
            }
            store_out(L, (unsigned)y * (unsigned)L.W + (unsigned)x, res);
        }
        __syncthreads();  // the next tile's staging overwrites zt
    }
}

// One chunk c of a frame's item space with the dense coarsest level in
// tiles (m built with TILES): a chunk of list items, or one 16 x 16 tile of
// the dense level evaluated from its LDS depth tile as in ssao_items_tiled.
// Every thread of the block takes part (the tile staging ends with
// barriers).  Used by the batch launch, whose frames share the LDS.
template <typename NT, int H>
__device__ __forceinline__ void ssao_chunk_tiled(const SsaoArgs& a, const ItemMap& m, unsigned c, const float* ks,
                                                 const float* eg, float kmax, float* zt) {
    constexpr int TW = kDenseTile + 2 * H;
    const unsigned total = item_total(m);
    const int jd = m.nlev - 1;  // the dense coarsest level
    unsigned dense0 = 0;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) dense0 = k == jd ? m.cum[k] : dense0;
    if (c * 256u < dense0) {
        const unsigned item = c * 256u + threadIdx.x;
        if (item < total) ssao_item<NT, true, true>(a, m, item, ks, eg, kmax);
        return;
    }
    const NT* nrm = static_cast<const NT*>(a.c.normal);
    const unsigned plane = (unsigned)a.c.plane;
    const EvalLevel& L = a.c.lv[jd];
    const unsigned tile = c - dense0 / 256u, tx = dense_tiles_x(L.W);
    const int x0 = (int)(tile % tx) * kDenseTile, y0 = (int)(tile / tx) * kDenseTile;
    for (int i = threadIdx.x; i < TW * TW; i += 256) {
        const int ry = i / TW, rx = i - ry * TW;
        const int gx = min(max(x0 - H + rx, 0), L.W - 1), gy = min(max(y0 - H + ry, 0), L.H - 1);
        zt[i] = L.z[(unsigned)gy * (unsigned)L.zpy + (unsigned)gx * (unsigned)L.zpx];
    }
    __syncthreads();
    const int x = x0 + (int)(threadIdx.x % kDenseTile), y = y0 + (int)(threadIdx.x / kDenseTile);
    if (x < L.W && y < L.H) {
        const float z = zt[(y - y0 + H) * TW + (x - x0 + H)];
        float res = 0.0f;
        if (valid_depth(z)) {
            const DepthTile dt{zt, (unsigned)(x0 - H), (unsigned)(y0 - H), (unsigned)TW};
            res = ssao_texel<NT, kGroupMulti, true>(a, L, nrm, plane, ks, kmax, x, y, z, dt);
        }
        store_out(L, (unsigned)y * (unsigned)L.W + (unsigned)x, res);
    }
    __syncthreads();  // the next tile's staging overwrites zt
}

// samples of the tiled evaluation (staged in LDS with the depth tile)
constexpr int kTiledSamples = 256;

// Per block: the blur taps (AL) and, KLDS, the S <= kLdsSamples samples in
// LDS; returns the largest |component| of the samples (+inf when not staged).
template <bool AL, bool KLDS>
__device__ __forceinline__ float ssao_stage(const SsaoArgs& a, float* ks, float* eg) {
    __shared__ unsigned kmax_bits;  // as bits: all values >= 0
    if (AL) stage_taps(a.c, eg);
    if (!KLDS) {
        __syncthreads();
        return __builtin_inff();
    }
    if (threadIdx.x == 0) kmax_bits = 0u;
    __syncthreads();
    unsigned m = 0u;
    for (int i = threadIdx.x; i < 3 * a.S; i += 256) {
        const float v = a.kernel[i];
        ks[i] = v;
        m = max(m, __float_as_uint(fabsf(v)));
    }
    for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
    if (__lane_id() == 0) atomicMax(&kmax_bits, m);
    __syncthreads();
    return __uint_as_float(kmax_bits);
}

}  // namespace mr
