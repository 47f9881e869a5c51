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

__global__ __launch_bounds__(kRankThreads) void k_lean_stencil_batch(const LeanArgs* T, const unsigned* blk_base,
                                                                     int n) {
    __shared__ StencilLds<kRankThreads> sm;
    const int f = batch_frame(blk_base, n, blockIdx.x);
    stencil_block(T[f], blockIdx.x - blk_base[f], sm);
}

__global__ __launch_bounds__(kRankThreads) void k_lean_list_batch(const LeanArgs* T, const unsigned* blk_base, int n) {
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

template <int C, typename VT>
__global__ __launch_bounds__(256) void k_lean_merge4(LeanMergeArgs a, unsigned tiles_x, unsigned ntiles) {
    __shared__ Merge4Lds<C> sm;
    merge4_tile<C, VT>(a, xcd_remap(blockIdx.x, ntiles), tiles_x, sm);
}

// frames of a batch: tile_base[f] = first merge tile of frame f
template <int C, typename VT, bool M4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M4 ? 1 : merge_waves(C))))
void k_lean_merge_batch(const LeanMergeArgs* T, const unsigned* tile_base,
                                                          const unsigned* tiles_x, int n) {
    const unsigned g = xcd_remap(blockIdx.x, gridDim.x);
    int f = 0;
    for (int k = 1; k < n; ++k) f += g >= tile_base[k] ? 1 : 0;
    if constexpr (M4) {
        __shared__ Merge4Lds<C> sm;
        merge4_tile<C, VT>(T[f], g - tile_base[f], tiles_x[f], sm);
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

template <typename VT>
hipError_t launch_lean_merge_t(const LeanMergeArgs& a, hipStream_t s) {
    const unsigned tx = (a.W + kMergeTW - 1) / kMergeTW, ty = (a.H + kMergeTH - 1) / kMergeTH;
    const bool m4 = merge4_applies(a);
    if (a.C == 3) {
        if (m4)
            hipLaunchKernelGGL((k_lean_merge4<3, VT>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
        else
            hipLaunchKernelGGL((k_lean_merge<3, VT>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    } else {
        if (m4)
            hipLaunchKernelGGL((k_lean_merge4<1, VT>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
        else
            hipLaunchKernelGGL((k_lean_merge<1, VT>), dim3(tx * ty), dim3(256), 0, s, a, tx, tx * ty);
    }
    return hipGetLastError();
}

hipError_t launch_lean_merge(const LeanMergeArgs& a, hipStream_t s) {
    return a.c16 ? launch_lean_merge_t<_Float16>(a, s) : launch_lean_merge_t<float>(a, s);
}

hipError_t launch_lean_merge_batch(const LeanMergeArgs* T, const unsigned* tile_base, const unsigned* tiles_x, int n,
                                   unsigned total, int C, bool c16, bool m4, hipStream_t s) {
#define MR_MB(CC, VT, M) \
    hipLaunchKernelGGL((k_lean_merge_batch<CC, VT, M>), dim3(total), dim3(256), 0, s, T, tile_base, tiles_x, n)
    if (C == 3) {
        if (c16) {
            if (m4) MR_MB(3, _Float16, true);
            else MR_MB(3, _Float16, false);
        } else {
            if (m4) MR_MB(3, float, true);
            else MR_MB(3, float, false);
        }
    } else {
        if (c16) {
            if (m4) MR_MB(1, _Float16, true);
            else MR_MB(1, _Float16, false);
        } else {
            if (m4) MR_MB(1, float, true);
            else MR_MB(1, float, false);
        }
    }
#undef MR_MB
    return hipGetLastError();
}

}  // namespace mr
