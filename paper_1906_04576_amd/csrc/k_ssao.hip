// SSAO evaluated per sub-image (Sec. 3.2 / 4.1) and as the naive full-res
// pass (Sec. 5).  The paper cites Mittring 2007 and Bavoil et al. 2008 for
// SSAO without printing an estimator; this one is a normal-oriented
// hemisphere with a fixed caller-supplied kernel, a hard range check and a
// relative depth bias; output = occluded fraction.
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
// patterns and clamps the offset to last, four instructions fewer per sample
// than selecting texel 0 off screen; with groups of 8 samples in flight the
// second form keeps register use at full occupancy (measured).
template <bool FAST, bool CLAMP, typename KP>
__device__ __forceinline__ void ssao_project(const EvalLevel& L, KP K, int s, const SsaoTexel& T, unsigned zpy,
                                             unsigned zpx, unsigned last, bool& on, float& d, unsigned& off) {
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
        // never -0 because cx, cy > 0 (a sum is -0 only when both terms are)
        on = (d > 0.0f) & (__float_as_uint(u) < __float_as_uint(Wf)) & (__float_as_uint(v) < __float_as_uint(Hf));
        // u, v >= 0 when on, so truncation is floor.  Coordinates < 2^14 and
        // byte pitches < 2^22 fit the 24-bit products; on screen the offset
        // is at most last, so the clamp leaves it unchanged, and off screen
        // it keeps the gather inside the plane (its value is not used).
        const unsigned sx = (unsigned)cvt_i32_sat(u), sy = (unsigned)cvt_i32_sat(v);
        off = __builtin_elementwise_min((unsigned)__umul24(sy, 4u * zpy) + (unsigned)__umul24(sx, 4u * zpx), last);
    } else {
        on = (d > 0.0f) & (u >= 0.0f) & (u < Wf) & (v >= 0.0f) & (v < Hf);
        // u, v >= 0 when on, so truncation is floor; rows < 2^14 and pitches
        // < 2^20 keep the offset products within 24 bits
        const unsigned sx = (unsigned)(int)(on ? u : 0.0f), sy = (unsigned)(int)(on ? v : 0.0f);
        off = __umul24(sy, zpy) + __umul24(sx, zpx);
    }
}

// Gathers of a group of G samples are issued together, one projection at a
// time (sched_barrier: interleaving the projections buys little ILP and costs
// registers, i.e. occupancy); the group size sets how many gathers of a wave
// are in flight.
template <bool FAST, int G, typename SA, typename KP>
__device__ __forceinline__ int ssao_count(const SA& a, const EvalLevel& L, KP K, const SsaoTexel& T) {
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
    int occ = 0;
    int s = 0;
    for (; s + G <= S; s += G) {
        bool on[G];
        float d[G], zs[G];
        unsigned off[G];
#pragma unroll
        for (int k = 0; k < G; ++k) {
            ssao_project<FAST, CLAMP>(L, K, s + k, T, zpy, zpx, last, on[k], d[k], off[k]);
            // one projection at a time: interleaving them buys little ILP
            // and costs registers (occupancy)
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int k = 0; k < G; ++k) zs[k] = buf_f1(rz, CLAMP ? off[k] : off[k] * 4u);
#pragma unroll
        for (int k = 0; k < G; ++k) occ += occluded(on[k], d[k], zs[k]);
    }
    for (; s < S; ++s) {
        bool on;
        float d;
        unsigned off;
        ssao_project<FAST, CLAMP>(L, K, s, T, zpy, zpx, last, on, d, off);
        occ += occluded(on, d, buf_f1(rz, CLAMP ? off : off * 4u));
    }
    return occ;
}

// occlusion of one texel; K points to LDS (staged samples) or global memory;
// kmax = the largest |component| over the samples (+inf when unknown); a
// holds the sampling parameters r, b and S (SsaoArgs or SsaoSampling)
template <typename NT, int G, typename SA, typename KP>
__device__ __forceinline__ float ssao_texel(const SA& a, const EvalLevel& L, const NT* nrm, unsigned plane,
                                            KP K, float kmax, int x, int y, float z) {
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
    const int occ = __ballot(!safe) == 0 ? ssao_count<true, G>(a, L, K, T) : ssao_count<false, G>(a, L, K, T);
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

// KLDS: the S <= kLdsSamples samples are staged in LDS (else read from
// global memory); separate instances keep the common one's register budget.
template <typename NT, bool AL, bool KLDS>
__global__ __launch_bounds__(256) void k_ssao(SsaoArgs a) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    const float kmax = ssao_stage<AL, KLDS>(a, ks, eg);
    ssao_items<NT, KLDS, AL>(a, ks, eg, kmax);
}

// Frames of a batch (same samples, mask and effect parameters): one item
// space over all frames, each frame's range padded to whole chunks of 256,
// swept by a resident grid like the single-frame launch.
template <typename NT, bool AL, bool KLDS, bool Q>
__global__ __launch_bounds__(256) void k_ssao_batch(const SsaoArgs* T, int n, unsigned* queue) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ unsigned cbase[kMaxBatch + 1];
    const float kmax = ssao_stage<AL, KLDS>(T[0], ks, eg);
    batch_chunk_bases(T, n, cbase);
    for_each_chunk<Q>(cbase[n], queue, [&](unsigned c) {
        int f = 0;
        for (int k = 1; k < n; ++k) f += c >= cbase[k] ? 1 : 0;
        const SsaoArgs& a = T[f];
        const ItemMap m = make_item_map(a.c);
        const unsigned item = (c - cbase[f]) * 256u + threadIdx.x;
        if (item < item_total(m)) ssao_item<NT, KLDS, AL>(a, m, item, ks, eg, kmax);
    });
}

hipError_t launch_ssao_batch(const SsaoArgs* T, int n, int S, int normal_dtype, unsigned total_hint,
                             const BatchSchedule& bs, hipStream_t s) {
    // the compact frame path fuses a_i into the evaluation
    const bool lds = S <= kLdsSamples;
#define MR_SB(NT, KL, Q)                                                                                    \
    hipLaunchKernelGGL((k_ssao_batch<NT, true, KL, Q>),                                                     \
                       dim3(eval_blocks_capped<k_ssao_batch<NT, true, KL, Q>>(total_hint, bs.blocks_per_cu)), \
                       dim3(256), 0, s, T, n, bs.queue)
#define MR_SBQ(NT, KL)            \
    do {                          \
        if (bs.queue_mode)        \
            MR_SB(NT, KL, true);  \
        else                      \
            MR_SB(NT, KL, false); \
    } while (0)
    if (normal_dtype == MR_F16) {
        if (lds) MR_SBQ(_Float16, true);
        else MR_SBQ(_Float16, false);
    } else {
        if (lds) MR_SBQ(float, true);
        else MR_SBQ(float, false);
    }
#undef MR_SBQ
#undef MR_SB
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sub-images at full resolution with fewer samples: per pixel, the Eq. 1
// blend of the levels' values, each the SSAO of this full-resolution pixel
// with the level's own samples, with the merge's alpha_i.  A level whose
// alpha_i is 0 adds c_i * 0 = +0 and keeps the composite (c' * 1), and below
// the finest level with alpha_i = 1 the composite is c_i * 1 + c' * 0 = c_i:
// those evaluations are skipped without changing a bit (all values are
// finite).  The loop over levels is uniform; lanes take part where their
// pixel needs the level.

// alpha_i at full-res pixel (x, y): min(A w, 1), A the bilinear of a_i
// (texel centres, clamp to edge), 0 where none of the four taps is in the
// stencil; sums from +0 in tap order
__device__ __forceinline__ float fullres_alpha(const FullresLevel& V, int x, int y) {
    const float s = (float)(1 << V.sh);
    const float u = ((float)x + 0.5f) / s - 0.5f, v = ((float)y + 0.5f) / s - 0.5f;
    const float ux = floorf(u), vy = floorf(v);
    const float fx = u - ux, fy = v - vy;
    const int x0 = (int)ux, y0 = (int)vy;
    const int xa = min(max(x0, 0), V.W - 1), xb = min(max(x0 + 1, 0), V.W - 1);
    const int ya = min(max(y0, 0), V.H - 1), yb = min(max(y0 + 1, 0), V.H - 1);
    const float b0 = (1.0f - fx) * (1.0f - fy), b1 = fx * (1.0f - fy), b2 = (1.0f - fx) * fy, b3 = fx * fy;
    const unsigned r0 = (unsigned)ya * (unsigned)V.W, r1 = (unsigned)yb * (unsigned)V.W;
    float den = 0.0f;
    den = den + (V.S[r0 + xa] ? b0 : 0.0f);
    den = den + (V.S[r0 + xb] ? b1 : 0.0f);
    den = den + (V.S[r1 + xa] ? b2 : 0.0f);
    den = den + (V.S[r1 + xb] ? b3 : 0.0f);
    float A = 0.0f;
    A = A + b0 * V.a[r0 + xa];
    A = A + b1 * V.a[r0 + xb];
    A = A + b2 * V.a[r1 + xa];
    A = A + b3 * V.a[r1 + xb];
    return den > 0.0f ? fminf(A * V.w, 1.0f) : 0.0f;
}

template <typename NT>
__global__ __launch_bounds__(256) void k_ssao_fullres(FullresArgs a) {
    __shared__ float ks[3 * kFullresMaxSamples];
    __shared__ unsigned kmax_bits[kMaxLevels];  // per level, as bits: all values >= 0
    // per-level sampling parameters in LDS: indexing the kernel argument by the
    // level loop would copy it to scratch
    __shared__ SsaoSampling sp[kMaxLevels];
    __shared__ int skoff[kMaxLevels];
    if (threadIdx.x < kMaxLevels) kmax_bits[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < kMaxLevels; ++j) {
            sp[j] = a.lv[j].p;
            skoff[j] = a.lv[j].koff;
        }
    }
    __syncthreads();
    for (int j = 0; j < a.nlev; ++j) {
        const FullresLevel& V = a.lv[j];
        unsigned m = 0u;
        for (int i = threadIdx.x; i < 3 * V.p.S; i += 256) {
            const float v = V.p.kernel[i];
            ks[3 * V.koff + i] = v;
            m = max(m, __float_as_uint(fabsf(v)));
        }
        for (int o = 32; o >= 1; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
        if (__lane_id() == 0) atomicMax(&kmax_bits[j], m);
    }
    __syncthreads();
    const EvalLevel& L = a.L;
    const NT* nrm = static_cast<const NT*>(a.normal);
    const unsigned plane = (unsigned)a.plane, npx = (unsigned)a.W * (unsigned)a.H;
    const int top = a.nlev - 1;  // the coarsest level
    const ChunkRange cr = chunk_range((npx + 255u) / 256u);
    for (unsigned ch = cr.first; ch < cr.end; ch += cr.step) {
        const unsigned p = ch * 256u + threadIdx.x;
        const bool in = p < npx;
        const int y = in ? (int)(p / (unsigned)a.W) : 0, x = in ? (int)(p - (unsigned)y * (unsigned)a.W) : 0;
        const float z = in ? L.z[(unsigned)y * L.zpy + (unsigned)x * L.zpx] : 0.0f;
        const bool geo = in && valid_depth(z);
        // alpha of the levels below the coarsest (registers: constant indices)
        float al[kMaxLevels - 1];
        int k = top;  // finest level with alpha 1, else the coarsest
#pragma unroll
        for (int j = kMaxLevels - 2; j >= 0; --j) {
            al[j] = 0.0f;
            if (j < top && geo) {
                al[j] = fullres_alpha(a.lv[j], x, y);
                if (al[j] == 1.0f) k = j;
            }
        }
        float c = 0.0f;
        for (int j = top; j >= 0; --j) {
            float alj = 0.0f;
#pragma unroll
            for (int q = 0; q < kMaxLevels - 1; ++q) alj = q == j ? al[q] : alj;
            const bool need = geo && (j == k || (j < k && alj > 0.0f));
            if (__ballot(need) == 0) continue;
            if (need) {
                const float v = ssao_texel<NT, kGroupPlain>(sp[j], L, nrm, plane, (const float*)ks + 3 * skoff[j],
                                                     __uint_as_float(kmax_bits[j]), x, y, z);
                c = j == k ? v : v * alj + c * (1.0f - alj);
            }
        }
        if (in) a.out[p] = c;
    }
}

hipError_t launch_ssao_fullres(const FullresArgs& a, int normal_dtype, hipStream_t s) {
    const unsigned chunks = ((unsigned)a.W * (unsigned)a.H + 255u) / 256u;
    if (normal_dtype == MR_F16)
        hipLaunchKernelGGL((k_ssao_fullres<_Float16>), dim3(eval_blocks<k_ssao_fullres<_Float16>>(chunks * 256u)),
                           dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_ssao_fullres<float>), dim3(eval_blocks<k_ssao_fullres<float>>(chunks * 256u)),
                           dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ssao(const SsaoArgs& a, int normal_dtype, unsigned total_hint, hipStream_t s) {
    const bool al = fused_alpha(a.c), lds = a.S <= kLdsSamples;
#define MR_SSAO(NT, AL, KL) \
    hipLaunchKernelGGL((k_ssao<NT, AL, KL>), dim3(eval_blocks<k_ssao<NT, AL, KL>>(total_hint)), dim3(256), 0, s, a)
    if (normal_dtype == MR_F16) {
        if (al) {
            if (lds) MR_SSAO(_Float16, true, true);
            else MR_SSAO(_Float16, true, false);
        } else {
            if (lds) MR_SSAO(_Float16, false, true);
            else MR_SSAO(_Float16, false, false);
        }
    } else {
        if (al) {
            if (lds) MR_SSAO(float, true, true);
            else MR_SSAO(float, true, false);
        } else {
            if (lds) MR_SSAO(float, false, true);
            else MR_SSAO(float, false, false);
        }
    }
#undef MR_SSAO
    return hipGetLastError();
}

}  // namespace mr
