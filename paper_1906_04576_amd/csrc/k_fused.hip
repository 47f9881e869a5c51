// A batch of frames in one persistent launch: the edge image and level depth
// (Sec. 3.1), the stencils and work lists (Sec. 4.1), the masked per-level
// evaluation (Sec. 3.2) and the merge (Sec. 4.2, Eq. 1) of every frame, taken
// as tickets from one counter by a grid of resident blocks.  Each stage runs
// the same tile code as the per-stage launches, so the images are bit for bit
// those of the staged batch; only the order in which tiles run changes, and
// every tile still sees the finished results of the stage before it.
#include "edges_tile.hpp"
#include "lean_tiles.hpp"
#include "ssao_item.hpp"
#include "ssgi_item.hpp"

namespace mr {

// list runs staged in LDS up to this many entries (longer runs are stored
// straight from the threads), so that the stage union stays within the LDS
// of four resident blocks per CU
constexpr unsigned kFusedListStage = 4096;

// ranking tiles per ticket of the stencil and list passes: every finished
// ticket writes its XCD's L2 back, so fewer, larger tickets cost fewer
// write-backs (24-frame SSGI batch: 3.61 ms with one tile per ticket, 3.48
// with 4, 3.42 with 8, 3.40 with 16)
constexpr unsigned kFusedRankGroup = 8;

// counter words (see FusedArgs)
__device__ __forceinline__ unsigned* fused_ready(const FusedArgs& A, int stage, int f) {
    return A.ctr + 3 + stage * kMaxBatchFrames + f;
}
__device__ __forceinline__ unsigned* fused_eval_ctr(const FusedArgs& A, int f) {
    return A.ctr + 3 + kFusedReady * kMaxBatchFrames + 8 * f;
}

// Visibility between stages.  The L2 caches are per XCD and not coherent
// with each other, so a finished ticket writes its XCD's dirty L2 lines back
// (an agent-scope release by thread 0, after every wave's stores have
// reached that L2) before it is counted.  The waiting side does not
// invalidate its caches: no block reads a stage's results before that stage
// of the frame has finished, every array of the layout starts on its own
// 256-byte boundary, and the caches hold nothing of the workspace from
// before the launch, so no cache holds a stale copy of a finished result.
// (An acquire on every poll, or after every wait, invalidated the L2 of
// every XCD thousands of times per run: the persistent launch ran 4x
// slower than the staged launches.)

// s_waitcnt vmcnt(0): this wave's loads and stores have completed
constexpr int kWaitVmcnt0 = 0x0F70;

// Wait until `need` tickets of a stage of a frame have finished: thread 0
// polls the counter; the barrier holds the block until then.
__device__ __forceinline__ void fused_wait(const FusedArgs& A, const unsigned* ready, unsigned need) {
    if (threadIdx.x == 0) {
        unsigned it = 0;
        while (__hip_atomic_load(ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            __builtin_amdgcn_s_sleep(8);
            if (++it >= A.spin_limit) {
                __hip_atomic_fetch_or(A.ctr + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __syncthreads();
}

// A finished ticket: every wave waits for its stores, then thread 0 writes
// the XCD's L2 back and counts the ticket.
__device__ __forceinline__ void fused_done(unsigned* ready) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the L2 write-back ...
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);            // ... has completed before the count
        __hip_atomic_fetch_add(ready, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// one value of block-wide scalar traffic: thread 0 writes, all read
__device__ __forceinline__ unsigned fused_bcast(unsigned* slot, unsigned v) {
    if (threadIdx.x == 0) *slot = v;
    __syncthreads();
    const unsigned r = *slot;
    __syncthreads();
    return r;
}

// Stage calls through restrict-qualified table parameters: inlined, they
// keep the tables' no-alias guarantee, so a frame's fields need not be read
// again after the stage's own stores.
template <typename NT>
__device__ __forceinline__ void fused_edges(const EdgeArgs* __restrict__ te, int f, unsigned i, unsigned tx) {
    edges_tile<NT, false, true, true>(te[f], i, tx);
}
template <bool LIST, typename LDS>
__device__ __forceinline__ void fused_rank(const LeanArgs* __restrict__ tl, int f, unsigned i, LDS& sm) {
    if constexpr (LIST)
        list_block<256, kFusedListStage>(tl[f], i, sm);
    else
        stencil_block<256>(tl[f], i, sm);
}
template <int C, typename VT, typename LDS>
__device__ __forceinline__ void fused_merge4(const LeanMergeArgs* __restrict__ tm, int f, unsigned i, unsigned tx,
                                             LDS& sm) {
    merge4_tile<C, VT>(tm[f], i, tx, sm);
}

template <int C>
union FusedLds {
    StencilLds<256> st;
    ListLds<256, kFusedListStage> li;
    Merge4Lds<C> m4;
    MergeLds<C> mg;
};

// EFFECT: MR_EFFECT_SSAO or MR_EFFECT_SSGI; NT / CT: normal and colour
// storage; M4: the merge of levels 1-4 (else the general merge).  Edge tiles
// are 256 x 8 pixels (at most 4 levels).  The samples are staged in LDS once
// per block (S <= kFusedSamples).  Four waves per SIMD: the edge tiles need
// about 120 registers, the other stages fewer.
template <int EFFECT, typename NT, typename CT, bool M4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_batch_fused(FusedArgs A) {
    constexpr int C = EFFECT == MR_EFFECT_SSGI ? 3 : 1;
    __shared__ float ks[3 * kFusedSamples];
    __shared__ float eg[kMaxLevels * kEgStride];
    __shared__ FusedLds<C> u;
    __shared__ unsigned slot;
    // tb[s][f]: frame f's first ticket of stage s, relative to the stage
    // (tb[s][n] = the stage's tickets): edge and merge tiles in groups of
    // A.group, ranking tiles in groups of kFusedRankGroup (stencil, then
    // list), and
    // ceil(px / worker_px) evaluation workers per frame
    __shared__ unsigned tb[kFusedStages][kMaxBatchFrames + 1];
    float kmax = 0.0f;
    if constexpr (EFFECT == MR_EFFECT_SSAO) {
        kmax = ssao_stage<true, true>(static_cast<const SsaoArgs*>(A.tv)[0], ks, eg);
    } else {
        ssgi_stage<true, true>(static_cast<const SsgiArgs*>(A.tv)[0], ks, eg);
    }
    const unsigned G = (unsigned)A.group;
    if (threadIdx.x < 64) {
        const int f = threadIdx.x;
        const bool in = f < A.n;
        unsigned w[kFusedStages];
        w[0] = in ? (A.base[0][f + 1] - A.base[0][f] + G - 1u) / G : 0u;
        w[1] = in ? (A.base[1][f + 1] - A.base[1][f] + kFusedRankGroup - 1u) / kFusedRankGroup : 0u;
        w[2] = w[1];
        w[3] = in ? (A.px[f] + A.worker_px - 1u) / A.worker_px : 0u;
        w[4] = in ? (A.base[4][f + 1] - A.base[4][f] + G - 1u) / G : 0u;
#pragma unroll
        for (int k = 0; k < kFusedStages; ++k) {
            const unsigned inc = wave_scan_incl(w[k]);
            if (f == 0) tb[k][0] = 0u;
            if (in) tb[k][f + 1] = inc;
        }
    }
    __syncthreads();
    unsigned start[kFusedStages + 1];
    start[0] = 0u;
#pragma unroll
    for (int k = 0; k < kFusedStages; ++k) start[k + 1] = start[k] + tb[k][A.n];
    const unsigned total = start[kFusedStages];
    int waited = -1;  // the last dependency this block waited for
    // thread 0 claims the next ticket while the block works on this one
    unsigned next = threadIdx.x == 0 ? atomicAdd(A.ctr, 1u) : 0u;
    for (;;) {
        const unsigned t = fused_bcast(&slot, next);
        if (t >= total) break;
        if (threadIdx.x == 0) next = atomicAdd(A.ctr, 1u);
        int s = 0;
#pragma unroll
        for (int k = 1; k < kFusedStages; ++k) s += t >= start[k] ? 1 : 0;
        s = __builtin_amdgcn_readfirstlane(s);
        unsigned lo = start[0];
#pragma unroll
        for (int k = 1; k < kFusedStages; ++k) lo = s == k ? start[k] : lo;
        const unsigned local = t - lo;
        const unsigned* fb = tb[s];
        int f = 0;
        for (int k = 1; k < A.n; ++k) f += local >= fb[k] ? 1 : 0;
        f = __builtin_amdgcn_readfirstlane(f);
        const unsigned j = local - fb[f];  // the ticket within its stage and frame
        // A stage's results do not change once it has finished, so a block
        // that has waited for (stage s - 1, frame f) does not wait again.
        const int key = s * kMaxBatchFrames + f;
        if (s > 0 && key != waited) {
            fused_wait(A, fused_ready(A, s - 1, f), tb[s - 1][f + 1] - tb[s - 1][f]);
            waited = key;
        }
        // tiles [j G, min((j + 1) G, n)) of the frame's edge or merge tiles
        const unsigned tile0 = j * G;
        if (s == 0) {
            const unsigned nt = A.base[0][f + 1] - A.base[0][f];
            for (unsigned i = tile0; i < nt && i < tile0 + G; ++i) {
                if (i > tile0) __syncthreads();  // the previous tile's LDS reads are done
                fused_edges<NT>(A.te, f, i, A.edge_tx[f]);
            }
        } else if (s == 1 || s == 2) {
            // ranking tiles [j R, min((j + 1) R, n)): the stencil pass, or the
            // list pass (which waited for the frame's whole stencil pass)
            const unsigned nt = A.base[1][f + 1] - A.base[1][f];
            for (unsigned i = j * kFusedRankGroup; i < nt && i < (j + 1u) * kFusedRankGroup; ++i) {
                if (i > j * kFusedRankGroup) __syncthreads();  // the previous tile's LDS reads are done
                if (s == 1)
                    fused_rank<false>(A.tl, f, i, u.st);
                else
                    fused_rank<true>(A.tl, f, i, u.li);
            }
        } else if (s == 3) {
            // an evaluation worker: chunks of the frame's items until none is left
            using Args = std::conditional_t<EFFECT == MR_EFFECT_SSAO, SsaoArgs, SsgiArgs>;
            const Args& a = static_cast<const Args*>(A.tv)[f];
            const ItemMap m = make_item_map(a.c);
            const unsigned items = item_total(m), per = 256u * (unsigned)A.items;
            const unsigned nch = (items + per - 1u) / per;
            unsigned* q = fused_eval_ctr(A, f);
            const unsigned home = blockIdx.x & 7u;
            for (unsigned r = 0; r < 8u; ++r) {
                const unsigned x = (home + r) & 7u;  // this XCD's region first
                const unsigned lo = (unsigned)((unsigned long long)nch * x / 8u);
                const unsigned hi = (unsigned)((unsigned long long)nch * (x + 1u) / 8u);
                for (;;) {
                    const unsigned c = lo + fused_bcast(&slot, threadIdx.x == 0 ? atomicAdd(q + x, 1u) : 0u);
                    if (c >= hi) break;
                    for (int i = 0; i < A.items; ++i) {
                        const unsigned item = c * per + (unsigned)i * 256u + threadIdx.x;
                        if (item >= items) continue;
                        if constexpr (EFFECT == MR_EFFECT_SSAO)
                            ssao_item<NT, true, true>(a, m, item, ks, eg, kmax);
                        else
                            ssgi_item<NT, CT, true>(a, m, item, (const float*)ks, (const float*)eg);
                    }
                }
            }
        } else {
            const LeanMergeArgs& ma = A.tm[f];
            const unsigned nt = A.base[4][f + 1] - A.base[4][f];
            for (unsigned i = tile0; i < nt && i < tile0 + G; ++i) {
                if (i > tile0) __syncthreads();  // the previous tile's LDS reads are done
                if constexpr (M4) {
                    if (ma.c16)
                        fused_merge4<C, _Float16>(A.tm, f, i, A.merge_tx[f], u.m4);
                    else
                        fused_merge4<C, float>(A.tm, f, i, A.merge_tx[f], u.m4);
                } else {
                    if (ma.c16)
                        merge_tile<C, _Float16>(ma, i, A.merge_tx[f], u.mg.la, u.mg.ls, u.mg.lc, u.mg.lvl_any);
                    else
                        merge_tile<C, float>(ma, i, A.merge_tx[f], u.mg.la, u.mg.ls, u.mg.lc, u.mg.lvl_any);
                }
            }
        }
        if (s < kFusedReady)
            fused_done(fused_ready(A, s, f));
        else
            __syncthreads();  // the LDS union is reused by the next ticket
    }
    // the last block to leave has seen every ticket finish: clear the
    // counters (not the error word) for the next run
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned left = __hip_atomic_fetch_add(A.ctr + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        slot = left == gridDim.x - 1u ? 1u : 0u;
    }
    __syncthreads();
    if (slot) {
        for (int i = threadIdx.x; i < kFusedCounters; i += 256)
            if (i != 2) __hip_atomic_store(A.ctr + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_batch_fused(const FusedArgs& a, int effect, int S, int normal_dtype, int color_dtype,
                              unsigned* grid_out, hipStream_t s) {
    if (S > kFusedSamples || !a.wide) return hipErrorInvalidValue;
    const bool n16 = normal_dtype == MR_F16, col16 = color_dtype == MR_F16, m4 = a.m4 != 0;
#define MR_FU(E, NT, CT, M)                                                               \
    do {                                                                                  \
        const unsigned g = resident_blocks<k_batch_fused<E, NT, CT, M>>();                \
        if (grid_out) *grid_out = g;                                                      \
        hipLaunchKernelGGL((k_batch_fused<E, NT, CT, M>), dim3(g), dim3(256), 0, s, a);   \
    } while (0)
#define MR_FU_M(E, NT, CT)             \
    do {                               \
        if (m4)                        \
            MR_FU(E, NT, CT, true);    \
        else                           \
            MR_FU(E, NT, CT, false);   \
    } while (0)
    if (effect == MR_EFFECT_SSAO) {
        if (n16) MR_FU_M(MR_EFFECT_SSAO, _Float16, float);
        else MR_FU_M(MR_EFFECT_SSAO, float, float);
    } else {
        if (n16 && col16) MR_FU_M(MR_EFFECT_SSGI, _Float16, _Float16);
        else if (n16) MR_FU_M(MR_EFFECT_SSGI, _Float16, float);
        else if (col16) MR_FU_M(MR_EFFECT_SSGI, float, _Float16);
        else MR_FU_M(MR_EFFECT_SSGI, float, float);
    }
#undef MR_FU_M
#undef MR_FU
    return hipGetLastError();
}

}  // namespace mr
