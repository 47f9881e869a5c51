// Lean frame path kernels: ranking, owner-level map and merge launches over
// the tile functions of lean_tiles.hpp.
#include "lean_tiles.hpp"

namespace mr {

__global__ __launch_bounds__(kRankThreads) void k_lean_stencil(LeanArgs A) {
    __shared__ StencilLds<kRankThreads> sm;
    stencil_block(A, blockIdx.x, sm);
}
__global__ __launch_bounds__(kRankThreads) void k_lean_list(LeanArgs A) {
    __shared__ ListLds<kRankThreads, kRankStage> sm;
    list_block(A, blockIdx.x, sm);
}

// frames of a batch: blk_base[f] = first tile of frame f, blk_base[n] = total
__device__ __forceinline__ int batch_frame(const unsigned* blk_base, int n, unsigned g) {
    int f = 0;
    for (int k = 1; k < n; ++k) f += g >= blk_base[k] ? 1 : 0;
    return f;
}

__global__ __launch_bounds__(kRankThreads) void k_lean_stencil_batch(const LeanArgs* __restrict__ T,
                                                                     const unsigned* __restrict__ blk_base, int n) {
    __shared__ StencilLds<kRankThreads> sm;
    const int f = batch_frame(blk_base, n, blockIdx.x);
    stencil_block(T[f], blockIdx.x - blk_base[f], sm);
}

__global__ __launch_bounds__(kRankThreads) void k_lean_list_batch(const LeanArgs* __restrict__ T,
                                                                  const unsigned* __restrict__ blk_base, int n) {
    __shared__ ListLds<kRankThreads, kRankStage> sm;
    const int f = batch_frame(blk_base, n, blockIdx.x);
    list_block(T[f], blockIdx.x - blk_base[f], sm);
}

hipError_t launch_lean_masks(const LeanArgs& a, hipStream_t s) {
    if (a.nblk) {
        hipLaunchKernelGGL(k_lean_stencil, dim3(a.nblk), dim3(kRankThreads), 0, s, a);
        hipLaunchKernelGGL(k_lean_list, dim3(a.nblk), dim3(kRankThreads), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_lean_masks_batch(const LeanArgs* T, const unsigned* blk_base, int n, unsigned total,
                                   hipStream_t s) {
    if (total) {
        hipLaunchKernelGGL(k_lean_stencil_batch, dim3(total), dim3(kRankThreads), 0, s, T, blk_base, n);
        hipLaunchKernelGGL(k_lean_list_batch, dim3(total), dim3(kRankThreads), 0, s, T, blk_base, n);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// owner-level map from the stencil bits
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lean_level_map(LeanMapArgs a) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= a.W || y >= a.H) return;
    uint8_t lvl = (uint8_t)a.coarsest;
    for (int j = a.nlev - 1; j >= 0; --j) {
        const int sh = a.level[j] - 1;
        const int X = x >> sh, Y = y >> sh;
        if ((a.Sb[j][(unsigned)Y * (unsigned)a.wpr[j] + (unsigned)(X >> 5)] >> (X & 31)) & 1u)
            lvl = (uint8_t)a.level[j];
    }
    a.out[(unsigned)y * (unsigned)a.W + (unsigned)x] = lvl;
}

hipError_t launch_lean_level_map(const LeanMapArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_lean_level_map, dim3((a.W + 63) / 64, (a.H + 3) / 4), dim3(256), 0, s, a);
    return hipGetLastError();
}


// The three-channel general merge needs about 96 registers, at the step
// between 5 and 4 waves per SIMD, and small changes elsewhere in the file
// move the allocator above it: its occupancy is fixed at 5 (measured faster
// than 4 waves without the few spilled registers).
constexpr int merge_waves(int C) { return C == 1 ? 1 : 5; }

template <int C, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(merge_waves(C))))
void k_lean_merge(LeanMergeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ float la[kMergeLDS];
    __shared__ uint8_t ls[kMergeLDS];
    __shared__ float lc[C][kMergeLDS];
    __shared__ int lvl_any[kMaxLevels];
    merge_tile<C, VT>(a, xcd_remap(blockIdx.x, ntiles), tiles_x, la, ls, lc, lvl_any);
}

// L2 false: the levels 1, 3 and 4
template <int C, typename VT, bool L2>
__global__ __launch_bounds__(256) void k_lean_merge4(LeanMergeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ Merge4Lds<C> sm;
    merge4_tile<C, VT, L2>(a, xcd_remap(blockIdx.x, ntiles), tiles_x, sm);
}

// frames of a batch: tile_base[f] = first merge tile of frame f; GEO one of
// kMergeGeneral, kMerge1234, kMerge134
template <int C, typename VT, int GEO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GEO != kMergeGeneral ? 1 : merge_waves(C))))
void k_lean_merge_batch(const LeanMergeArgs* __restrict__ T, const unsigned* __restrict__ tile_base,
                        const unsigned* __restrict__ tiles_x, int n) {
    const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
    int f = 0;
    for (int k = 1; k < n; ++k) f += g >= tile_base[k] ? 1 : 0;
    if constexpr (GEO != kMergeGeneral) {
        __shared__ Merge4Lds<C> sm;
        merge4_tile<C, VT, GEO == kMerge1234>(T[f], g - tile_base[f], tiles_x[f], sm);
    } else {
        __shared__ float la[kMergeLDS];
        __shared__ uint8_t ls[kMergeLDS];
        __shared__ float lc[C][kMergeLDS];
        __shared__ int lvl_any[kMaxLevels];
        merge_tile<C, VT>(T[f], g - tile_base[f], tiles_x[f], la, ls, lc, lvl_any);
    }
}

// levels 1, 2, 3, 4 with level 1 by rank (the common 4-level frame)
bool merge4_applies(const LeanMergeArgs& a) {
    if (a.nlev != 4 || !a.fine1 || (a.W & 3) != 0) return false;
    for (int j = 0; j < 4; ++j)
        if (a.lv[j].sh != j) return false;
    return true;
}

// levels 1, 3, 4 with level 1 by rank (SSGI's Table 1 column)
bool merge134_applies(const LeanMergeArgs& a) {
    return a.nlev == 3 && a.fine1 && (a.W & 3) == 0 && a.lv[0].sh == 0 && a.lv[1].sh == 2 && a.lv[2].sh == 3;
}

int merge_geometry(const LeanMergeArgs& a) {
    return merge4_applies(a) ? kMerge1234 : (merge134_applies(a) ? kMerge134 : kMergeGeneral);
}

template <typename VT>
hipError_t launch_lean_merge_t(const LeanMergeArgs& a, hipStream_t s) {
    const unsigned tx = (a.W + kMergeTW - 1) / kMergeTW, ty = (a.H + kMergeTH - 1) / kMergeTH;
    const int geo = merge_geometry(a);
#define MR_LM(CC)                                                                                              \
    do {                                                                                                       \
        if (geo == kMerge1234)                                                                                 \
            hipLaunchKernelGGL((k_lean_merge4<CC, VT, true>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);  \
        else if (geo == kMerge134)                                                                             \
            hipLaunchKernelGGL((k_lean_merge4<CC, VT, false>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty); \
        else                                                                                                   \
            hipLaunchKernelGGL((k_lean_merge<CC, VT>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);         \
    } while (0)
    if (a.C == 3)
        MR_LM(3);
    else
        MR_LM(1);
#undef MR_LM
    return hipGetLastError();
}

hipError_t launch_lean_merge(const LeanMergeArgs& a, hipStream_t s) {
    return a.c16 ? launch_lean_merge_t<_Float16>(a, s) : launch_lean_merge_t<float>(a, s);
}

hipError_t launch_lean_merge_batch(const LeanMergeArgs* T, const unsigned* tile_base, const unsigned* tiles_x, int n,
                                   unsigned total, int C, bool c16, int geo, hipStream_t s) {
#define MR_MB(CC, VT, G) \
    hipLaunchKernelGGL((k_lean_merge_batch<CC, VT, G>), dim3(total), dim3(256), 0, s, T, tile_base, tiles_x, n)
#define MR_MBG(CC, VT)                  \
    do {                                \
        if (geo == kMerge1234)          \
            MR_MB(CC, VT, kMerge1234);  \
        else if (geo == kMerge134)      \
            MR_MB(CC, VT, kMerge134);   \
        else                            \
            MR_MB(CC, VT, kMergeGeneral); \
    } while (0)
    if (C == 3) {
        if (c16) MR_MBG(3, _Float16);
        else MR_MBG(3, float);
    } else {
        if (c16) MR_MBG(1, _Float16);
        else MR_MBG(1, float);
    }
#undef MR_MBG
#undef MR_MB
    return hipGetLastError();
}

}  // namespace mr
