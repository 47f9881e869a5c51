// SSAO per sub-image (Sec. 3.2 / 4.1) and as the naive full-res pass (Sec. 5):
// the launches over the per-texel code of ssao_item.hpp, and sub-images at
// full resolution with fewer samples.
#include "ssao_item.hpp"

namespace mr {

// KLDS: the S <= kLdsSamples samples are staged in LDS (else read from
// global memory); separate instances keep the common one's register budget.
template <typename NT, bool AL, bool KLDS>
__global__ __launch_bounds__(256) void k_ssao(SsaoArgs a) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    const float kmax = ssao_stage<AL, KLDS>(a, ks, eg);
    ssao_items<NT, KLDS, AL>(a, ks, eg, kmax);
}

// The compact frame path with the coarsest level in 16 x 16 tiles whose depth
// (with a halo of H texels) is staged in LDS; at most kTiledSamples samples,
// staged in LDS as well.
template <typename NT, int H>
__global__ __launch_bounds__(256) void k_ssao_tiled(SsaoArgs a) {
    __shared__ float ks[3 * kTiledSamples];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ float zt[(kDenseTile + 2 * H) * (kDenseTile + 2 * H)];
    const float kmax = ssao_stage<true, true>(a, ks, eg);
    ssao_items_tiled<NT, H>(a, ks, eg, kmax, zt);
}

// Frames of a batch (same samples, mask and effect parameters): one item
// space over all frames, each frame's range padded to whole chunks of 256,
// swept by a resident grid like the single-frame launch.
template <typename NT, bool AL, bool KLDS, bool Q>
__global__ __launch_bounds__(256) void k_ssao_batch(const SsaoArgs* __restrict__ T, int n, unsigned* queue) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ unsigned cbase[kMaxBatch + 1];
    const float kmax = ssao_stage<AL, KLDS>(T[0], ks, eg);
    batch_chunk_bases(T, n, 256u, cbase);
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
    if (a.halo) {
        if (!al || !a.c.dense_tiles || a.S > kTiledSamples) return hipErrorInvalidValue;
#define MR_ST(NT, H) \
    hipLaunchKernelGGL((k_ssao_tiled<NT, H>), dim3(eval_blocks<k_ssao_tiled<NT, H>>(total_hint)), dim3(256), 0, s, a)
#define MR_STH(NT)                                \
    do {                                          \
        if (a.halo == 8)                          \
            MR_ST(NT, 8);                         \
        else if (a.halo == 16)                    \
            MR_ST(NT, 16);                        \
        else if (a.halo == 24)                    \
            MR_ST(NT, 24);                        \
        else                                      \
            return hipErrorInvalidValue;          \
    } while (0)
        if (normal_dtype == MR_F16)
            MR_STH(_Float16);
        else
            MR_STH(float);
#undef MR_STH
#undef MR_ST
        return hipGetLastError();
    }
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
