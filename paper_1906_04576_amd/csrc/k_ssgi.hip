// One-bounce screen-space indirect light (Sec. 2.4): the per-level, batched
// and naive launches over the per-texel code of ssgi_item.hpp.
#include "ssgi_item.hpp"

namespace mr {

// KLDS: the samples are staged in LDS (S <= kLdsSamples), else read from
// global memory; one instance each keeps the sample loop inlined once
template <typename NT, typename CT, bool AL, bool KLDS>
__global__ __launch_bounds__(256) void k_ssgi(SsgiArgs a) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    ssgi_stage<AL, KLDS>(a, ks, eg);
    if (KLDS)
        ssgi_items<NT, CT, AL>(a, (const float*)ks, (const float*)eg);
    else
        ssgi_items<NT, CT, AL>(a, a.kernel, (const float*)eg);
}

// frames of a batch (see k_ssao_batch)
template <typename NT, typename CT, bool Q, bool KLDS>
__global__ __launch_bounds__(256) void k_ssgi_batch(const SsgiArgs* __restrict__ T, int n, unsigned* queue) {
    __shared__ float ks[KLDS ? 3 * kLdsSamples : 1];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ unsigned cbase[kMaxBatch + 1];
    ssgi_stage<true, KLDS>(T[0], ks, eg);
    batch_chunk_bases(T, n, 256u, cbase);
    for_each_chunk<Q>(cbase[n], queue, [&](unsigned c) {
        int f = 0;
        for (int k = 1; k < n; ++k) f += c >= cbase[k] ? 1 : 0;
        const SsgiArgs& a = T[f];
        const ItemMap m = make_item_map(a.c);
        const unsigned item = (c - cbase[f]) * 256u + threadIdx.x;
        if (item >= item_total(m)) return;
        if (KLDS)
            ssgi_item<NT, CT, true>(a, m, item, (const float*)ks, (const float*)eg);
        else
            ssgi_item<NT, CT, true>(a, m, item, T[0].kernel, (const float*)eg);
    });
}

hipError_t launch_ssgi_batch(const SsgiArgs* T, int n, int S, int normal_dtype, int color_dtype,
                             unsigned total_hint, const BatchSchedule& bs, hipStream_t s) {
    const bool lds = S <= kLdsSamples;
#define MR_GB(NT, CT, Q, KL)                                                                                   \
    hipLaunchKernelGGL((k_ssgi_batch<NT, CT, Q, KL>),                                                          \
                       dim3(eval_blocks_capped<k_ssgi_batch<NT, CT, Q, KL>>(total_hint, bs.blocks_per_cu)), \
                       dim3(256), 0, s, T, n, bs.queue)
#define MR_GBQ(NT, CT)                   \
    do {                                 \
        if (bs.queue_mode) {             \
            if (lds)                     \
                MR_GB(NT, CT, true, true);  \
            else                         \
                MR_GB(NT, CT, true, false); \
        } else {                         \
            if (lds)                     \
                MR_GB(NT, CT, false, true); \
            else                         \
                MR_GB(NT, CT, false, false); \
        }                                \
    } while (0)
    if (normal_dtype == MR_F16 && color_dtype == MR_F16)
        MR_GBQ(_Float16, _Float16);
    else if (normal_dtype == MR_F16)
        MR_GBQ(_Float16, float);
    else if (color_dtype == MR_F16)
        MR_GBQ(float, _Float16);
    else
        MR_GBQ(float, float);
#undef MR_GBQ
#undef MR_GB
    return hipGetLastError();
}

hipError_t launch_ssgi(const SsgiArgs& a, int normal_dtype, int color_dtype, unsigned total_hint,
                       hipStream_t s) {
    const bool al = fused_alpha(a.c), lds = a.S <= kLdsSamples;
#define MR_SK(NT, CT, AL, KL) \
    hipLaunchKernelGGL((k_ssgi<NT, CT, AL, KL>), dim3(eval_blocks<k_ssgi<NT, CT, AL, KL>>(total_hint)), dim3(256), 0, s, a)
#define MR_SSGI(NT, CT)                \
    do {                               \
        if (al) {                      \
            if (lds)                   \
                MR_SK(NT, CT, true, true);  \
            else                       \
                MR_SK(NT, CT, true, false); \
        } else {                       \
            if (lds)                   \
                MR_SK(NT, CT, false, true); \
            else                       \
                MR_SK(NT, CT, false, false); \
        }                              \
    } while (0)
    if (normal_dtype == MR_F16 && color_dtype == MR_F16)
        MR_SSGI(_Float16, _Float16);
    else if (normal_dtype == MR_F16)
        MR_SSGI(_Float16, float);
    else if (color_dtype == MR_F16)
        MR_SSGI(float, _Float16);
    else
        MR_SSGI(float, float);
#undef MR_SSGI
#undef MR_SK
    return hipGetLastError();
}

}  // namespace mr
