// SSAO over a batch of frames (Sec. 3.2 / 4.1 for each frame) with every
// frame's dense coarsest level evaluated in LDS-staged depth tiles: the
// batch form of the single-frame tiled launch in k_ssao.hip.
#include "ssao_item.hpp"

namespace mr {

// Frames of a batch with each frame's dense coarsest level in 16 x 16 tiles
// whose depth, with a halo of H texels, is staged in LDS (as k_ssao_tiled):
// one item space over all frames, each frame's range padded to whole chunks
// of 256, swept by a resident grid in fixed strides.  At most kTiledSamples
// samples.
template <typename NT, int H>
__global__ __launch_bounds__(256) void k_ssao_batch_tiled(const SsaoArgs* __restrict__ T, int n) {
    __shared__ float ks[3 * kTiledSamples];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ float zt[(kDenseTile + 2 * H) * (kDenseTile + 2 * H)];
    __shared__ unsigned cbase[kMaxBatch + 1];
    const float kmax = ssao_stage<true, true>(T[0], ks, eg);
    batch_chunk_bases<true>(T, n, 256u, cbase);
    const ChunkRange cr = chunk_range(cbase[n]);
    for (unsigned c = cr.first; c < cr.end; c += cr.step) {
        int f = 0;
        for (int k = 1; k < n; ++k) f += c >= cbase[k] ? 1 : 0;
        const SsaoArgs& a = T[f];
        ssao_chunk_tiled<NT, H>(a, make_item_map<true>(a.c), c - cbase[f], ks, eg, kmax, zt);
    }
}

hipError_t launch_ssao_batch_tiled(const SsaoArgs* T, int n, int S, int normal_dtype, int halo, unsigned total_hint,
                                   hipStream_t s) {
    if (S > kTiledSamples) return hipErrorInvalidValue;
#define MR_SBT(NT, H)                                                                                      \
    hipLaunchKernelGGL((k_ssao_batch_tiled<NT, H>), dim3(eval_blocks<k_ssao_batch_tiled<NT, H>>(total_hint)), \
                       dim3(256), 0, s, T, n)
#define MR_SBTH(NT)                     \
    do {                                \
        if (halo == 8)                  \
            MR_SBT(NT, 8);              \
        else if (halo == 16)            \
            MR_SBT(NT, 16);             \
        else if (halo == 24)            \
            MR_SBT(NT, 24);             \
        else                            \
            return hipErrorInvalidValue; \
    } while (0)
    if (normal_dtype == MR_F16)
        MR_SBTH(_Float16);
    else
        MR_SBTH(float);
#undef MR_SBTH
#undef MR_SBT
    return hipGetLastError();
}

}  // namespace mr
