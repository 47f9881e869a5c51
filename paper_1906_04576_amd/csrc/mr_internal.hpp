// Internal declarations shared by the host API and the HIP kernels of libmr.
// Nothing here is part of the public C ABI (include/mr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mr.h"

namespace mr {

constexpr int kMaxLevels = MR_MAX_LEVELS;
constexpr int kBlurFusedMaxRadiusC = 8;  // largest radius of the single-launch blur and the lean path
constexpr int kMaxRadius = MR_MAX_RADIUS;
constexpr int kChunk = 4096;  // texels per compaction chunk (256 threads x 16)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool valid_depth(float z) {
    // geometry iff finite and > 0 (inf and NaN fail both tests below)
    return z > 0.0f && z < __builtin_inff();
}

// Four consecutive floats of a frame's final image, stored non-temporally:
// nothing in the frame reads them again, and streaming them out keeps the
// caches for the next frame's inputs (merge 22.1 -> 20.8 us, the following
// edge kernel 36.9 -> 35.1 us at 4K).  p is 16-byte aligned.
__device__ __forceinline__ void store_stream4(float* p, float a, float b, float c, float d) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(p));
}

// float -> int32 with the conversion instruction's own result for every
// input (truncation; NaN gives 0, values out of range saturate), where a
// C++ conversion of such a value is undefined
__device__ __forceinline__ int cvt_i32_sat(float x) {
    int r;
    asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

template <typename T>
__device__ __forceinline__ float ld(const T* p, long long i) {
    return static_cast<float>(p[i]);
}

// Raw buffer resource over `bytes` bytes at `p` (gfx9 family: dword 3 =
// 0x00020000).  With stride 0 the hardware checks each load's byte offset
// against `bytes`: a load at or past the end returns 0 and makes no memory
// access.  Most loads through these keep their offset in range by clamping;
// the SSAO sample gathers rely on the check for off-screen samples, whose
// values are never used.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float4 buf_f4(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0));
}

__device__ __forceinline__ float buf_f1(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// Blocks of a 1-D grid are handed to the 8 XCDs round robin (block b runs on
// XCD b % 8).  Remap so that every XCD works on one contiguous range of tiles:
// neighbouring tiles then share that XCD's L2 (halo rows and columns hit).
__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned n) {
    const unsigned q = n >> 3, rem = n & 7u, x = b & 7u, k = b >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------------------
// argument blocks (passed by value to the kernels)
// ---------------------------------------------------------------------------
struct EdgeArgs {
    const float* depth;
    const void* normal;
    const uint8_t* hard;  // optional one-sample shadow bits
    int W, H;
    float depth_ratio, normal_cos;
    uint8_t* E;                          // full-res edges
    uint8_t* Ei[kMaxLevels];             // pooled edges per level (null = not needed)
    float* zi[kMaxLevels];               // point-sampled level depth (null = not needed)
    int Wi[kMaxLevels], Hi[kMaxLevels];
    int num_levels;
    // bit-packed edges (lean frame path): levels 1..3, 32 texels per word,
    // bit x % 32 of word x / 32, rows of wpr words; null = not written
    uint32_t* Eb[3];
    int wpr[3];
    // optional: words zero[0 .. zero_n) set to 0, 256 per tile (the frame's
    // level counts)
    uint32_t* zero;
    unsigned zero_n;
    // importance mask of a gaze point (fov != 0): squared radii, FP32
    int fov;
    float fgx, fgy, fri2, fro2;
};

struct BlurLevel {
    const uint8_t* Ei;
    float* a;
    uint8_t* S;
    int W, H, r;
    unsigned tiles_x, tile_base;
    float g[2 * kMaxRadius + 1];
};

struct BlurArgs {
    BlurLevel lv[kMaxLevels - 1];  // every enabled level below the coarsest
    int nlev;
    unsigned ntiles;
};

struct NestArgs {
    const uint8_t* Sf;  // finer stencil
    uint8_t* Sc;        // coarser stencil (updated in place)
    int Wf, Hf, Wc, Hc, k;
};

struct LevelMapArgs {
    const uint8_t* S[kMaxLevels];
    int Wi[kMaxLevels];
    int levels[kMaxLevels];  // enabled levels ascending (1-based); last = coarsest
    int nlev;
    int W, H;
    uint8_t* out;
};

struct CompactArgs {
    const uint8_t* S[kMaxLevels];
    uint32_t* list[kMaxLevels];
    uint32_t n[kMaxLevels];          // texels per compacted level
    uint32_t chunk_base[kMaxLevels + 1];
    int count_idx[kMaxLevels];       // index into count[] per compacted level
    int nlev;                        // compacted levels
    uint32_t* chunk_count;           // [total chunks]
    uint32_t* chunk_off;             // [total chunks]
    uint32_t* count;                 // [MR_MAX_LEVELS]
};

// One level of an evaluation pass.  Depth of texel (x, y) is
// z[y * zpy + x * zpx]; normals and colour of texel (x, y) sit at full-res
// element index goff + y * gpy + x * gpx of their planes.
struct EvalLevel {
    const float* z;
    int zpy, zpx;  // element strides of the depth view (32-bit: images are at most 16384^2)
    long long goff, gpy;
    int gpx;
    int W, H;
    float f, cx, cy;
    float* out;            // f32, or f16 when out16
    int out16;
    int stream;            // out is a final image (evaluation without masks): non-temporal stores
    long long out_plane;
    const uint32_t* list;  // null = dense
    int count_idx;         // list length = counts[count_idx]
    unsigned dense_n;
    int compact;           // list levels: output at the list position instead of the texel
    // lean frame path: also write a_i at the list position (ac != null),
    // computed from the edge bits Eb (Ewpr words per row) with radius Er
    float* ac;
    const uint32_t* Eb;
    int Ewpr, Er;
    float Eg[2 * kBlurFusedMaxRadiusC + 1];
};

struct EvalCommon {
    EvalLevel lv[kMaxLevels];
    int nlev;
    const uint32_t* counts;
    const void* normal;
    const void* color;
    long long plane;  // H * W, full-res plane stride of normal/colour
    // the dense coarsest level's items in 16 x 16 texel tiles (one chunk of
    // 256 items per tile, its range starting on a chunk boundary)
    int dense_tiles;
};

struct SsaoArgs {
    EvalCommon c;
    const float* kernel;
    int S;
    float r, b;
    // LDS halo in texels around a tile of the dense coarsest level (0: its
    // samples read the depth plane); needs c.dense_tiles
    int halo;
};

struct ShadowArgs {
    EvalCommon c;
    const float* sm;
    int size;
    float M[12];
    float fL, lsize, nL, bias;
    const float* bd;
    const float* pd;
    int nb, np;
};

struct SsgiArgs {
    EvalCommon c;
    const float* kernel;
    int S;
    float r, b;
};

struct HardArgs {
    const float* depth;
    int W, H;
    float f;
    const float* sm;
    int size;
    float M[12];
    float fL, bias;
    uint8_t* hard;
};

struct MergeLevel {
    const float* c;
    long long c_plane;
    const float* a;     // null for the coarsest
    const uint8_t* S;   // null for the coarsest
    int s, sh, W, H;    // scale s = 2^sh and level size
    float w;
    // levels with s >= 2: texels a 64 x 16 pixel tile's bilinear taps can
    // touch, rw x rh starting at ((x0 >> sh) - 1, (y0 >> sh) - 1), staged at
    // LDS offset roff; rmagic = ceil(65536 / rw) divides the staging index
    int rw, rh, roff;
    unsigned rmagic;
};

struct MergeArgs {
    MergeLevel lv[kMaxLevels];  // enabled levels ascending; last = coarsest
    int nlev;
    int W, H, C;
    int staged;  // total staged texels
    float* out;
};

constexpr int kMergeTW = 64, kMergeTH = 16;
// >= sum of rw * rh over levels 2..6 (518), and of those sums rounded up to
// whole waves as the compact path lays them out (384 + 128 + 3 x 64 = 704)
constexpr int kMergeLDS = 768;

// ---------------------------------------------------------------------------
// lean frame path (bit-packed stencils, values stored by rank)
// ---------------------------------------------------------------------------
constexpr int kLeanTileWords = 16, kLeanTileRows = 32;  // 512 words per ranking tile (measured)

struct LeanLevel {
    const uint32_t* Eb;  // edge bits
    uint32_t* Sb;        // stencil bits
    uint32_t* woff;      // per word: number of stencil texels ranked before it
    uint32_t* list;      // stencil texels in rank (tile) order
    float* ac;           // a_i by rank
    int W, H, wpr, r;
    int tiles_x;         // ranking tiles per row of words
    unsigned nwords, blk_base, ntiles;
    int count_idx;
    float g[2 * kMaxRadius + 1];
};

struct LeanArgs {
    LeanLevel lv[3];    // enabled levels below the coarsest (levels 1..3)
    int nlev;
    unsigned nblk;      // ranking tiles (one block each) over all levels
    uint32_t* count;    // per level, written by the level's last tile
    uint32_t* tot;      // per ranking tile: its number of stencil texels
};

struct LeanMapArgs {
    const uint32_t* Sb[3];
    int wpr[3];
    int level[3];
    int nlev;
    int coarsest;
    int W, H;
    uint8_t* out;
};

struct LeanMergeLevel {
    const void* c;       // f32 or f16 values by rank (levels below the coarsest) or dense (coarsest)
    long long c_plane;
    const uint32_t* Sb;  // null for the coarsest
    const uint32_t* woff;
    const float* ac;
    int s, sh, W, H, wpr;
    float w;
    int rw, rh, roff;
    unsigned rmagic;
};

struct LeanMergeArgs {
    LeanMergeLevel lv[kMaxLevels];
    int nlev;
    int W, H, C;
    int staged;
    bool fine1;
    bool c16;  // sub-image values stored as f16
    float* out;
};

// bilateral blur of SSAO sub-images (compact frame path): levels below the
// coarsest hold their values by rank, the coarsest densely
struct BilateralLevel {
    const float* z;        // level depth, dense W x H
    const void* c;         // values (f32, or f16 when c16)
    void* out;             // blurred values, same layout and type
    const uint32_t* list;  // rendered texels by rank; null: dense level
    const uint32_t* Sb;    // stencil bits (list levels)
    const uint32_t* woff;  // rank of each stencil word's first texel
    int W, H, wpr, count_idx;
    unsigned dense_n;
};

struct BilateralArgs {
    BilateralLevel lv[kMaxLevels];  // the blurred levels, ascending
    int nlev;
    const uint32_t* counts;
    int R;
    float wb[5];  // binomial weights of order 2R
    float drel;
    int c16;
};

// sub-images at full resolution with fewer samples
constexpr int kFullresMaxSamples = 1024;  // samples over all levels (staged in LDS)

struct SsaoSampling {
    const float* kernel;
    int S;
    float r, b;
};

struct FullresLevel {
    const float* a;    // a_i, dense level image (null for the coarsest)
    const uint8_t* S;  // stencil, dense level image (null for the coarsest)
    int W, H, sh;
    float w;           // blend weight w_i
    SsaoSampling p;    // the level's samples
    int koff;          // first sample in the block's LDS copy
};

struct FullresArgs {
    FullresLevel lv[kMaxLevels];  // enabled levels ascending; last = coarsest
    int nlev;
    EvalLevel L;  // full-resolution geometry
    const void* normal;
    long long plane;
    float* out;
    int W, H;
};

// ---------------------------------------------------------------------------
// launchers (return hipSuccess or the launch error)
// ---------------------------------------------------------------------------
hipError_t launch_edges(const EdgeArgs& a, int normal_dtype, hipStream_t s);
hipError_t launch_blur(const BlurArgs& a, hipStream_t s);       // levels with radius <= 8
hipError_t launch_blur_wide(const BlurLevel& a, hipStream_t s);  // one level, radius 9..16
constexpr int kBlurFusedMaxRadius = kBlurFusedMaxRadiusC;
hipError_t launch_nest(const NestArgs& a, hipStream_t s);
hipError_t launch_level_map(const LevelMapArgs& a, hipStream_t s);
hipError_t launch_compact(const CompactArgs& a, hipStream_t s);
hipError_t launch_ssao(const SsaoArgs& a, int normal_dtype, unsigned total_hint, hipStream_t s);
hipError_t launch_hard(const HardArgs& a, hipStream_t s);
hipError_t launch_shadow(const ShadowArgs& a, unsigned total_hint, hipStream_t s);
hipError_t launch_ssgi(const SsgiArgs& a, int normal_dtype, int color_dtype, unsigned total_hint,
                       hipStream_t s);
hipError_t launch_merge(const MergeArgs& a, hipStream_t s);
hipError_t launch_lean_masks(const LeanArgs& a, hipStream_t s);
hipError_t launch_lean_level_map(const LeanMapArgs& a, hipStream_t s);
hipError_t launch_lean_merge(const LeanMergeArgs& a, hipStream_t s);
hipError_t launch_bilateral(const BilateralArgs& a, unsigned total_hint, hipStream_t s);
hipError_t launch_ssao_fullres(const FullresArgs& a, int normal_dtype, hipStream_t s);
bool merge4_applies(const LeanMergeArgs& a);
// merge kernels: the general one, or fixed tap geometry for the levels 1-4
// or 1, 3, 4 (level 1 by rank, width divisible by 4)
constexpr int kMergeGeneral = 0, kMerge1234 = 1, kMerge134 = 2;
int merge_geometry(const LeanMergeArgs& a);

// edge kernel tiling for an image (the choice launch_edges makes)
void edges_grid(int W, int H, int num_levels, bool& wide, unsigned& tiles_x, unsigned& ntiles);
// tiling for one tile shape: 256x8 pixels (wide, at most 4 levels) or 64x32
void edges_tiles(int W, int H, bool wide, unsigned& tiles_x, unsigned& ntiles);

// batched frames: argument tables in device memory, one launch per stage.
// The edge launch also zeroes `queue` (the evaluation's per-XCD counters).
hipError_t launch_edges_batch(const EdgeArgs* T, const unsigned* tile_base, const unsigned* tiles_x, int n,
                              unsigned total, int normal_dtype, bool hard, bool wide, unsigned* queue,
                              hipStream_t s);
hipError_t launch_lean_masks_batch(const LeanArgs* T, const unsigned* blk_base, int n, unsigned total,
                                   hipStream_t s);
// how a batched evaluation hands out its chunks
constexpr int kQueueCounters = 8;  // work-queue counters: one per XCD
// words zeroed by the batch's edge launch: the queue counters
constexpr int kBatchCounters = kQueueCounters;
struct BatchSchedule {
    bool queue_mode;    // per-XCD work queues instead of fixed strides
    int blocks_per_cu;  // grid cap per CU, 0: as many blocks as are resident
    unsigned* queue;    // kQueueCounters counters, zeroed by the edge launch
};
hipError_t launch_ssao_batch(const SsaoArgs* T, int n, int S, int normal_dtype, unsigned total_hint,
                             const BatchSchedule& bs, hipStream_t s);
// the SSAO batch with LDS depth tiles of the dense coarsest level (halo 8, 16
// or 24 texels; at most 256 samples)
hipError_t launch_ssao_batch_tiled(const SsaoArgs* T, int n, int S, int normal_dtype, int halo, unsigned total_hint,
                                   hipStream_t s);
hipError_t launch_ssgi_batch(const SsgiArgs* T, int n, int S, int normal_dtype, int color_dtype,
                             unsigned total_hint, const BatchSchedule& bs, hipStream_t s);
hipError_t launch_lean_merge_batch(const LeanMergeArgs* T, const unsigned* tile_base, const unsigned* tiles_x, int n,
                                   unsigned total, int C, bool c16, int geo, hipStream_t s);

// The whole batch in one persistent launch.  Blocks take tickets from one
// counter; tickets run in stage order (edge tiles, stencil tiles, list tiles,
// evaluation workers, merge tiles; frames in order within a stage), and a
// ticket first waits until every ticket of the previous stage of its frame
// has finished.  Every ticket it waits for was taken earlier by a running
// block, so the waits always end; each is bounded all the same (spin_limit
// polls), and one that runs out sets the error word and goes on.  An
// evaluation worker takes its frame's chunks of 256 x items texels from
// per-XCD counters (its own XCD's region first, then the others').  The last
// block to leave zeroes the counters for the next run.
constexpr int kFusedStages = 5;
constexpr int kFusedSamples = 256;  // sample sets staged in LDS at most
constexpr int kFusedReady = 4;      // stages whose completion is counted
// counter words: ticket, blocks left, error word, then ready[kFusedReady][kMaxBatchFrames] and
// eval[kMaxBatchFrames][8]
constexpr int kMaxBatchFrames = 64;
constexpr int kFusedCounters = 3 + kFusedReady * kMaxBatchFrames + 8 * kMaxBatchFrames;
struct FusedArgs {
    const EdgeArgs* te;
    const LeanArgs* tl;
    const void* tv;  // SsaoArgs or SsgiArgs
    const LeanMergeArgs* tm;
    // per stage: frame f's first tile (edge, ranking, -, ranking, merge)
    // within the stage, n + 1 entries (base[3] unused); the blocks derive
    // their ticket tables from these, the pixel counts px and the group and
    // worker sizes
    const unsigned* base[kFusedStages];
    const unsigned* px;
    const unsigned* edge_tx;   // edge tiles per row, per frame
    const unsigned* merge_tx;  // merge tiles per row, per frame
    unsigned worker_px;        // pixels of a frame per evaluation worker ticket
    int group;                 // edge and merge tiles per ticket
    unsigned* ctr;             // kFusedCounters words, zero between runs
    int n, wide, m4, items;
    unsigned spin_limit;
};
hipError_t launch_batch_fused(const FusedArgs& a, int effect, int S, int normal_dtype, int color_dtype,
                              unsigned* grid_out, hipStream_t s);

}  // namespace mr
