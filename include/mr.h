/*
 * mr.h - multi-resolution screen-space lighting on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libmr.so.  The operations follow Besenthal, Maisch and Ropinski,
 * "Multi-Resolution Rendering for Computationally Expensive Lighting
 * Effects" (arXiv 1906.04576):
 *
 *   mr_build_masks     Sec. 3.1 (edge image, downsampling, blur with the
 *                      Table 1 variances, inclusive levels) and Sec. 4.1
 *                      (stencil = mask > 0), plus per-level work lists that
 *                      replace the stencil test.
 *   mr_eval_ssao       Sec. 3.2 / 4.1: the effect rendered per sub-image only
 *   mr_eval_shadow     where the level's stencil permits (Sec. 2.4 names the
 *   mr_eval_ssgi       three effects); with no masks, the naive full-resolution
 *                      pass of Sec. 5.
 *   mr_upsample_merge  Sec. 3.3 / 4.2, Eq. 1: bilinear upsampling and the
 *                      sequential blend from the coarsest level.
 *   mr_frame           the whole pipeline for one effect (optionally with
 *                      FP16 sub-image storage, the bilateral blur of SSAO
 *                      sub-images of Sec. 4.1 and the foveated mask of
 *                      Sec. 6).
 *   mr_eval_ssao_fullres  Sec. 6: sub-images at full resolution with fewer
 *                      samples instead of a lower resolution.
 *   mr_batch_*         frames of uneven sizes with one launch per stage.
 *
 * Conventions (all functions):
 *  - Every array argument is DEVICE memory owned by the caller, unless the
 *    comment says "host".  The library never allocates or frees memory;
 *    intermediate storage comes from a caller-provided workspace sized by
 *    mr_workspace_bytes.  Device pointers must be 16-byte aligned.
 *  - Images are row-major [y][x], row 0 at the top; multi-channel images are
 *    planar [c][y][x].  Level i (1-based) has scale s_i = 2^(i-1) and size
 *    W_i = W / s_i, H_i = H / s_i; W and H must be divisible by 2^(N-1).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *    enqueues work on it and returns; there is no host synchronisation and
 *    work-list counts stay on the device (except mr_batch_setup and
 *    mr_batch_tune, which wait for the stream).  Device faults surface at
 *    the caller's next synchronisation.
 *  - Every call validates all arguments before it enqueues anything; on
 *    error it returns a negative MR_E_* code, enqueues nothing, leaves the
 *    outputs untouched and sets a thread-local message (mr_last_error).
 *  - Calls are re-entrant.  Besides the thread-local error message the
 *    library keeps only per-device facts, each set on its first use on that
 *    device and read-only afterwards: the compute-unit count, kernels'
 *    resident-block counts and the address of the static scratch
 *    (mr_frame_static).  Calls that share output or workspace memory must be
 *    ordered by the caller (same stream or events).
 *  - Floating point: IEEE binary32, round to nearest even, no fused
 *    multiply-add, correctly rounded division and square root, denormals
 *    kept; results are deterministic run to run.
 */
#ifndef MR_H
#define MR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MR_API __attribute__((visibility("default")))

#define MR_MAX_LEVELS 6
#define MR_MAX_RADIUS 16   /* largest blur radius in level texels */
#define MR_MAX_SAMPLES 8192
#define MR_MAX_DIM 16384
#define MR_VERSION 101
#define MR_FRAME_EVENTS 5  /* stage events of mr_frame_desc */

/* status codes */
#define MR_OK 0
#define MR_E_NULL (-1)      /* a required pointer is NULL */
#define MR_E_SHAPE (-2)     /* width/height <= 0, > MR_MAX_DIM or not divisible by 2^(N-1) */
#define MR_E_PARAM (-3)     /* a parameter is out of range, or a pointer is misaligned */
#define MR_E_WORKSPACE (-4) /* workspace smaller than mr_workspace_bytes */
#define MR_E_DTYPE (-5)     /* unsupported element type */
#define MR_E_DEVICE (-6)    /* a HIP launch or query failed */

/* element types */
#define MR_F32 0
#define MR_F16 1

/* effects */
#define MR_EFFECT_SSAO 0
#define MR_EFFECT_SHADOW 1
#define MR_EFFECT_SSGI 2
#define MR_WS_MASKS (-1) /* mr_workspace_bytes purpose: scratch of mr_build_masks */

/* G-buffer (Sec. 3.1 uses depth and normals; SSGI also reads a lit colour
 * buffer).  depth: f32 [H][W] linear view depth, a pixel is geometry iff its
 * depth is finite and > 0.  normal: [3][H][W] view-space unit normals,
 * element type normal_dtype (MR_F32 or MR_F16).  color: [3][H][W] directly lit
 * colour, color_dtype (MR_F32 or MR_F16); only mr_eval_ssgi reads it. */
typedef struct {
    const float* depth;
    const void* normal;
    int normal_dtype;
    const void* color;
    int color_dtype;
} mr_gbuffer;

/* Pinhole camera: pixel (x, y) has its centre ray along
 * ((x + 0.5 - W/2) / f, (H/2 - (y + 0.5)) / f, -1) in view space. */
typedef struct {
    int width, height;
    float focal_px;
} mr_camera;

/* Mask parameters (Sec. 3.1, Table 1, Sec. 4).
 * num_levels   N in [1, MR_MAX_LEVELS].
 * level_enable bit (i-1) set = level i used; bits 0 and N-1 must be set
 *              (the paper's SSGI uses levels {1, 3, 4}).
 * depth_ratio  edge if the depth second difference along x or y exceeds
 *              depth_ratio * z (finite, >= 0).
 * normal_cos   edge if the dot product with a 4-neighbour's normal is
 *              below normal_cos (in [-1, 1]).
 * sigma2[i-1]  blur variance of level i in level-i texels (>= 0).
 * weight[i-1]  blend weight w_i (> 0, finite).
 * radius[i-1]  blur radius in level-i texels, -1 = ceil(3 sigma), at most
 *              MR_MAX_RADIUS.  Entries of disabled levels and of level N are
 *              ignored.
 * fovea        optional importance mask of a gaze point (Sec. 6: foveated
 *              rendering by modulating the mask; masks combined by minimum
 *              and maximum, Sec. 3.1), applied to the edge image before the
 *              pyramid: with d2 = dx*dx + dy*dy, dx = (x + 0.5f) - gaze_x,
 *              dy = (y + 0.5f) - gaze_y (FP32, in that order),
 *              E'(x, y) = (E(x, y) && d2 <= r_outer*r_outer) || d2 <= r_inner*r_inner:
 *              full detail near the gaze, the coarsest level beyond r_outer.
 *              enable = 0 turns it off; radii finite and >= 0. */
typedef struct {
    int enable;
    float gaze_x, gaze_y;
    float r_inner, r_outer;
} mr_fovea;

typedef struct {
    int num_levels;
    uint32_t level_enable;
    float depth_ratio;
    float normal_cos;
    float sigma2[MR_MAX_LEVELS];
    float weight[MR_MAX_LEVELS];
    int radius[MR_MAX_LEVELS];
    mr_fovea fovea;
} mr_mask_params;

/* Mask pyramid (outputs of mr_build_masks, inputs of eval/merge).  Index
 * [i-1] is level i.  For every enabled level i < N:
 *   alpha[i-1]     f32 [H_i][W_i] blurred mask a_i (required)
 *   stencil[i-1]   u8  [H_i][W_i] S_i = a_i > 0 after nesting (required)
 *   worklist[i-1]  u32 [H_i * W_i capacity] row-major ascending y*W_i + x of
 *                  the texels with S_i = 1 (required)
 * For every enabled level i >= 2:
 *   level_depth[i-1] f32 [H_i][W_i] point-sampled depth z(s x + s/2, s y + s/2)
 *                  (optional; NULL = the evaluators read the full-resolution
 *                  depth with stride s).
 * edge       u8 [H][W] full-resolution edge image (required).
 * level_map  u8 [H][W] owner level of every pixel = finest enabled level
 *            whose stencil covers it (optional, NULL = not written).
 * count      u32 [MR_MAX_LEVELS] device counts; count[i-1] = list length of
 *            level i (required; entries of other levels are set to 0).
 * Stencil and work-list entries of level N are never read: level N is
 * treated as covering the whole image. */
typedef struct {
    uint8_t* edge;
    uint8_t* level_map;
    float* alpha[MR_MAX_LEVELS];
    uint8_t* stencil[MR_MAX_LEVELS];
    uint32_t* worklist[MR_MAX_LEVELS];
    float* level_depth[MR_MAX_LEVELS];
    uint32_t* count;
} mr_masks;

/* SSAO (Sec. 2.4; estimator fixed by this library): normal-oriented
 * hemisphere with a caller-supplied kernel.
 * kernel   f32 [samples][3] sample offsets in the tangent frame (device)
 * samples  in [1, MR_MAX_SAMPLES]
 * radius   world-space radius r (> 0, finite)
 * bias_rel relative depth bias (>= 0, finite) */
typedef struct {
    const float* kernel;
    int samples;
    float radius;
    float bias_rel;
} mr_ssao_params;

/* Soft shadows (Sec. 2.4: shadow map, PCF, PCSS penumbra).
 * shadow_map   f32 [sm_size][sm_size] linear light depth (device)
 * view_to_light host 3x4 row-major affine map from camera view space to
 *              light view space (the light looks down its -z axis)
 * light_focal_px focal length of the light camera in texels
 * light_size   side of the square area light, light_near its near plane
 * bias         absolute depth bias of every shadow-map comparison
 * blocker_disk f32 [n_blocker][2], pcf_disk f32 [n_pcf][2] unit-disk
 *              points (device); n_* in [1, MR_MAX_SAMPLES] */
typedef struct {
    const float* shadow_map;
    int sm_size;
    float view_to_light[12];
    float light_focal_px;
    float light_size;
    float light_near;
    float bias;
    const float* blocker_disk;
    const float* pcf_disk;
    int n_blocker, n_pcf;
} mr_shadow_params;

/* One-bounce screen-space indirect light (Sec. 2.4): same sampling as SSAO,
 * occluding samples add the colour of the texel they hit. */
typedef struct {
    const float* kernel;
    int samples;
    float radius;
    float bias_rel;
} mr_ssgi_params;

/* Bilateral blur of SSAO sub-images before the merge (Sec. 4.1: smooths the
 * variance of few samples without carrying values from texels a level did
 * not render).  For every rendered texel p of a chosen level with valid
 * depth: the (2r+1)^2 window of taps q inside the level that the level
 * rendered (stencil 1) and whose depth is valid, weight
 *   w = b[dy] * b[dx] * max(0, 1 - |z_q - z_p| / (depth_rel * z_p)),
 * b the binomial weights of order 2r (1 2 1 / 4, 1 4 6 4 1 / 16), z the
 * level's point-sampled depth; result sum(w c) / sum(w), both summed in
 * window order (rows top to bottom, left to right), FP32.
 * levels     bit i-1 blurs level i (enabled levels only); 0 = off.
 * radius     1 or 2.
 * depth_rel  > 0, finite (0.05 is the edge detector's depth ratio). */
typedef struct {
    uint32_t levels;
    int radius;
    float depth_rel;
} mr_bilateral_params;

/* Whole-frame descriptor for mr_frame.
 * effect     MR_EFFECT_*; the matching params pointer must be non-NULL (host).
 * multires   0 = naive full-resolution pass (masks unused), 1 = multi-res.
 * out        f32 [C][H][W], C = 3 for SSGI, else 1.
 * level_map  optional u8 [H][W] owner-level output (multires only).
 * level_dtype  MR_F32 (0) or MR_F16: storage of the sub-image values between
 *            the evaluation and the merge (FP16 halves that traffic; every
 *            value is rounded to nearest even once, all arithmetic stays
 *            FP32).  MR_F16 needs the compact frame path (coarsest level
 *            <= 4, width divisible by 128, blur radii <= 8), else MR_E_DTYPE.
 * stage_events  optional hipEvent_t handles (each may be NULL), recorded on
 *            the frame's stream: [0] before the first kernel, [1] after the
 *            masks and work lists (after the hard-shadow pass on the naive
 *            path), [2] after the per-level evaluation, [3] after the merge,
 *            and [4] after the edge image (Sec. 3.1) on the compact frame
 *            path when it builds its masks, else at the same point as [1].
 *            They are owned by the caller and must have been created on the
 *            stream's device; event [k+1] minus event [k] (k < 3) is the GPU
 *            time of that stage, [4] minus [0] that of the edge image and [1]
 *            minus [4] that of the stencils, ranks and lists.
 * bilateral  optional blur of the SSAO sub-images (levels = 0: off); needs
 *            MR_EFFECT_SSAO, multires = 1 and the compact frame path, else
 *            MR_E_PARAM.  Counted in the evaluation stage.
 * eval_halo  0, 8, 16 or 24: how the SSAO evaluation gathers the depth of
 *            the dense coarsest level.  0: from the level's depth plane.  >0:
 *            the level is evaluated in 16 x 16 texel tiles whose depth, with
 *            a border of eval_halo texels, is staged in LDS, and the samples
 *            that land in that square read it there.  The image is
 *            bit-identical either way.  Nonzero needs MR_EFFECT_SSAO,
 *            multires = 1, the compact frame path and at most 256 samples,
 *            else MR_E_PARAM. */
typedef struct {
    int effect;
    int multires;
    mr_gbuffer g;
    mr_camera cam;
    mr_mask_params mp;
    const mr_ssao_params* ssao;
    const mr_shadow_params* shadow;
    const mr_ssgi_params* ssgi;
    float* out;
    uint8_t* level_map;
    int level_dtype;
    void* stage_events[MR_FRAME_EVENTS];
    mr_bilateral_params bilateral;
    int eval_halo;
} mr_frame_desc;

/* Workspace bytes needed by mr_frame for `effect` (MR_EFFECT_*) or by
 * mr_build_masks (purpose MR_WS_MASKS); cam and mp are host pointers.
 * Returns 0 and sets mr_last_error if the arguments are invalid. */
MR_API size_t mr_workspace_bytes(const mr_camera* cam, const mr_mask_params* mp, int purpose);

/* Sec. 3.1 + Sec. 4.1: edge image, OR-downsampled edges, blurred masks,
 * stencils, nesting, owner-level map, work lists and counts.
 * hard_shadow: optional u8 [H][W] one-sample shadow bits (mr_shadow_hard);
 * when given, pixels whose shadow bit differs from a 4-neighbour's are
 * edges too (the mask for soft shadows keeps geometry and shadow edges).
 * ws / ws_bytes: device scratch, at least mr_workspace_bytes(..., MR_WS_MASKS). */
MR_API int mr_build_masks(const mr_gbuffer* g, const mr_camera* cam, const mr_mask_params* mp,
                          const uint8_t* hard_shadow, const mr_masks* out, void* ws,
                          size_t ws_bytes, void* stream);

/* Sec. 3.2 / 4.1: SSAO occlusion per sub-image.  masks != NULL: for every
 * enabled level i < N the texels of worklist[i-1] (count on the device) are
 * evaluated, level N densely; out[i-1] is f32 [H_i][W_i] and is written only
 * at evaluated texels.  masks == NULL: the naive full-resolution pass into
 * out[0] (f32 [H][W]); other entries ignored.  Output 0 = unoccluded. */
MR_API int mr_eval_ssao(const mr_gbuffer* g, const mr_camera* cam, const mr_mask_params* mp,
                        const mr_masks* masks, const mr_ssao_params* p, float* const out[MR_MAX_LEVELS],
                        void* stream);

/* Sec. 3.1: one-sample hard shadow test per full-resolution pixel,
 * hard u8 [H][W] (1 = shadowed). */
MR_API int mr_shadow_hard(const mr_gbuffer* g, const mr_camera* cam, const mr_shadow_params* p,
                          uint8_t* hard, void* stream);

/* Soft-shadow visibility (1 = lit) per sub-image; same texel selection and
 * output layout as mr_eval_ssao. */
MR_API int mr_eval_shadow(const mr_gbuffer* g, const mr_camera* cam, const mr_mask_params* mp,
                          const mr_masks* masks, const mr_shadow_params* p,
                          float* const out[MR_MAX_LEVELS], void* stream);

/* Indirect RGB per sub-image; out[i-1] is f32 [3][H_i][W_i]; needs g->color. */
MR_API int mr_eval_ssgi(const mr_gbuffer* g, const mr_camera* cam, const mr_mask_params* mp,
                        const mr_masks* masks, const mr_ssgi_params* p,
                        float* const out[MR_MAX_LEVELS], void* stream);

/* Sec. 3.3 / 4.2, Eq. 1: every enabled level is upsampled bilinearly (taps
 * restricted to its stencil and renormalised), then blended from the
 * coarsest: c' = c_N, c' = C_i alpha_i + c' (1 - alpha_i) for enabled i < N
 * descending, alpha_i = min(bilinear(a_i) w_i, 1).  level_out[i-1] is
 * f32 [C][H_i][W_i]; out is f32 [C][H][W]; channels C in {1, 3}. */
MR_API int mr_upsample_merge(const mr_camera* cam, const mr_mask_params* mp, const mr_masks* masks,
                             const float* const level_out[MR_MAX_LEVELS], int channels, float* out,
                             void* stream);

/* SSAO with the sub-images realised at full resolution with fewer samples
 * instead of at a lower resolution (Sec. 6).  Every enabled level keeps its
 * mask from mr_build_masks (alpha and stencil of every enabled level below
 * the coarsest are read), but its value at a pixel is the SSAO of that
 * full-resolution pixel with the level's own sample set level_params[i-1]
 * (each as in mr_eval_ssao, typically fewer samples for coarser levels; at
 * most 1024 samples over the enabled levels; entries of disabled levels are
 * ignored).  The levels are blended per pixel with Eq. 1 from the coarsest:
 * out = c_L, then out = c_i alpha_i + out (1 - alpha_i) for the finer levels,
 * alpha_i = min(A w_i, 1) with A the bilinear of a_i as in mr_upsample_merge
 * (0 where no tap is in the stencil).  A level's evaluation is skipped where
 * alpha_i = 0 and the coarser ones below a level with alpha_i = 1; neither
 * changes a bit of the result.  out: f32 [H][W]; background pixels 0. */
MR_API int mr_eval_ssao_fullres(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp,
                                const mr_masks* masks, const mr_ssao_params* const level_params[MR_MAX_LEVELS],
                                float* out, void* stream);

/* Whole frame for one effect: masks (with shadow edges for MR_EFFECT_SHADOW),
 * per-level evaluation and merge, or the naive pass when multires == 0.
 * ws / ws_bytes: at least mr_workspace_bytes(&d->cam, &d->mp, d->effect). */
MR_API int mr_frame(const mr_frame_desc* d, void* ws, size_t ws_bytes, void* stream);

/* Autotuner for one frame configuration: how the evaluation of the coarsest
 * level gathers its depth (Sec. 4.1 renders each sub-image; eval_halo above).
 * Times mr_frame on `stream` with eval_halo = 0, 8, 16 and 24 (one warm-up
 * run, then `reps` runs, 1..1000), skipping the values the frame does not
 * admit (only 0 for the naive pass, effects other than SSAO and more than
 * 256 samples), and stores the fastest in d->eval_halo.  ms, when not NULL,
 * receives 4 floats: the milliseconds per frame of each value, -1 for one
 * that was skipped.  d as given must be valid for mr_frame (ws of at least
 * mr_workspace_bytes); its stage events are not recorded.  Runs the frame on
 * its current inputs, writes d->out and waits for the stream: not for use
 * under graph capture.  On an error d is unchanged. */
MR_API int mr_frame_tune(mr_frame_desc* d, void* ws, size_t ws_bytes, int reps, float* ms, void* stream);

/* A frame whose mask pyramid stays resident in caller memory across frames
 * (serving a static scene: the masks of Sec. 3.1 depend only on the
 * G-buffer, so requests after the first skip the mask kernels).  Compact
 * frame path only (coarsest level <= 4, width divisible by 128, blur radii
 * <= 8), else MR_E_PARAM.
 * mr_pyramid_bytes: sizes of the pyramid (edge and stencil bits, ranks, work
 * lists, counts, point-sampled level depth) and of the per-frame scratch.
 * mr_frame_cached: build = 1 computes the masks of d's inputs into `pyramid`,
 * then evaluates and merges as mr_frame does; build = 0 evaluates and merges
 * on the masks already in `pyramid`, which must come from an earlier call
 * with build = 1 on the same G-buffer contents, camera, mask parameters and
 * effect (and, for soft shadows, the same shadow inputs) -- the library
 * cannot check this.  The image is bit-identical to mr_frame's.  ws holds
 * the frame's scratch (at least the scratch size).  Frames that read one
 * pyramid may run concurrently; a build must be ordered before them.  The
 * stage events of d are recorded as in mr_frame (the mask stage is empty
 * when build = 0). */
MR_API int mr_pyramid_bytes(const mr_camera* cam, const mr_mask_params* mp, int effect, size_t* pyramid,
                            size_t* scratch);
MR_API int mr_frame_cached(const mr_frame_desc* d, void* pyramid, size_t pyramid_bytes, int build, void* ws,
                           size_t ws_bytes, void* stream);

/* mr_frame for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same frame with the workspace taken from a static device array of
 * MR_STATIC_SCRATCH_BYTES, one per device, that the library holds until the
 * process ends.  It enqueues the same kernels as mr_frame and calls no
 * allocating routine.  The stream's device must be the current device.
 * Frames whose intermediates need more than MR_STATIC_SCRATCH_BYTES (on the
 * compact path a 3840x2160 frame needs 27-39 MB; the other path needs about
 * 4.5 B/px more) are rejected with MR_E_WORKSPACE.  Every call on a device
 * shares that device's array: calls that may overlap on one device (other
 * streams, other threads) race and must be ordered by the caller; the array
 * keeps the last frame's intermediates, and each frame initialises what it
 * reads. */
#define MR_STATIC_SCRATCH_BYTES (64u << 20)
MR_API int mr_frame_static(const mr_frame_desc* d, void* stream);

/* Where the compact frame path keeps its masks in the workspace, as byte
 * offsets from ws (host; for callers and tests that read them after a
 * frame has completed).  compact = 1 when mr_frame takes the compact path
 * for these parameters (coarsest level <= 4, width divisible by 128, blur
 * radii <= 8); the other fields are then set, else they are 0.  Index [i-1]
 * is level i, for every enabled level i below the coarsest:
 *   worklist      u32 [count[i-1]] the texels y*W_i + x with S_i = 1 (Sec.
 *                 4.1), in ranking-tile order: tiles of tile_words x
 *                 tile_rows stencil words (32 texels each) row-major over
 *                 the level, words row-major inside a tile, texels left to
 *                 right inside a word.  The order is fixed (the same on
 *                 every run); sorting it gives the row-major list of
 *                 mr_build_masks.
 *   stencil_bits  u32 [H_i][W_i / 32] S_i, bit x % 32 of word x / 32
 *   rank          u32 [H_i][W_i / 32] list position of each word's first
 *                 stencil texel
 *   count         u32 [MR_MAX_LEVELS] list lengths
 * Returns MR_OK, or a negative code for invalid arguments. */
typedef struct {
    int compact;
    int tile_words, tile_rows;
    size_t count;
    size_t worklist[MR_MAX_LEVELS];
    size_t stencil_bits[MR_MAX_LEVELS];
    size_t rank[MR_MAX_LEVELS];
} mr_frame_layout;

MR_API int mr_frame_workspace_layout(const mr_camera* cam, const mr_mask_params* mp, int effect,
                                     mr_frame_layout* out);

/* Batches: up to MR_MAX_BATCH frames of one effect (MR_EFFECT_SSAO or
 * MR_EFFECT_SSGI) with identical mask and effect parameters and input types
 * but any sizes, processed with one launch per stage for all frames (edges,
 * ranks and work lists, per-level evaluation over one item space of all
 * frames by a resident grid, merge), or in one persistent launch whose
 * blocks take the stages' tiles from one queue (mr_batch_config).  Every frame must take the compact path
 * (coarsest level <= 4, width divisible by 128, blur radii <= 8), have
 * multires = 1, level_map = NULL and no bilateral blur; stage_events are not
 * recorded.
 *
 * mr_batch_setup validates the frames, lays them out in ws (at least
 * mr_batch_workspace_bytes) and copies the kernel argument tables there; it
 * returns when the copy is complete.  It fills `plan` (caller-owned host
 * memory of MR_BATCH_PLAN_BYTES).  mr_batch_run enqueues the batch's kernels
 * on `stream` and nothing else (no copies, no allocation, no memset), so it
 * can be captured in a HIP graph; the frames' inputs may change between
 * runs, their addresses and sizes may not.  ws and the inputs must stay
 * valid while a run is in flight. */
#define MR_MAX_BATCH 64
#define MR_BATCH_PLAN_BYTES 512
MR_API size_t mr_batch_workspace_bytes(const mr_frame_desc* frames, int n);
MR_API int mr_batch_setup(const mr_frame_desc* frames, int n, void* ws, size_t ws_bytes, void* plan,
                          size_t plan_bytes, void* stream);
MR_API int mr_batch_run(const void* plan, void* stream);

/* mr_batch_setup that does not wait, for a loop that forms a new batch from
 * whatever requests are pending (continuous batching).  The argument tables
 * are written to `staging`, caller-owned host memory of at least
 * mr_batch_staging_bytes(frames, n) bytes (page-locked, so that the copy is
 * asynchronous), and copied into ws by hipMemcpyAsync on `stream`; staging
 * must stay unchanged until the stream has passed that copy (e.g. until an
 * event recorded after the batch's run has completed), and ws must not be in
 * use by an earlier batch still in flight.  Returns 0 from
 * mr_batch_staging_bytes for an invalid batch (mr_last_error says why). */
MR_API size_t mr_batch_staging_bytes(const mr_frame_desc* frames, int n);
MR_API int mr_batch_setup_async(const mr_frame_desc* frames, int n, void* ws, size_t ws_bytes, void* plan,
                                size_t plan_bytes, void* staging, size_t staging_bytes, void* stream);

/* A batch on resident mask pyramids (serving resident scenes): pyramids[k]
 * is frame k's pyramid, built by mr_frame_cached (build = 1) on the same
 * G-buffer contents, camera, mask parameters and effect -- the library
 * cannot check this -- and ordered before the run.  The batch evaluates and
 * merges only (its edge and ranking launches are skipped), so ws holds just
 * the frames' scratch: at least mr_batch_cached_workspace_bytes(frames, n).
 * Set up without waiting, as mr_batch_setup_async.  Its plan runs staged
 * with fixed evaluation strides: mr_batch_set_config refuses persistent = 1
 * and eval_queue = 1 for it. */
MR_API size_t mr_batch_cached_workspace_bytes(const mr_frame_desc* frames, int n);
MR_API int mr_batch_setup_cached(const mr_frame_desc* frames, void* const* pyramids, int n, void* ws,
                                 size_t ws_bytes, void* plan, size_t plan_bytes, void* staging,
                                 size_t staging_bytes, void* stream);

/* How a batch's launches are shaped.  mr_batch_setup puts the defaults (all
 * zero) in the plan.  Every choice gives bit-identical outputs; only the time
 * differs.
 *   edge_tile           0: 256x8-pixel edge tiles (frames of at most 4
 *                          levels; 64x32 otherwise), 1: 64x32
 *   eval_queue          0: each evaluation block takes a fixed stride of
 *                          chunks of its XCD's share of the item space;
 *                          1: the blocks of an XCD take chunks one at a time
 *                          from a counter in the workspace
 *   eval_blocks_per_cu  cap on evaluation blocks per CU, 0..64; 0: as many
 *                       as can be resident
 *   merge_generic       0: a merge with fixed tap geometry where one applies
 *                          (the levels 1, 2, 3, 4 or 1, 3, 4 enabled),
 *                       1: the general merge
 *   persistent          0: one launch per stage; 1: the whole batch in one
 *                          launch of resident blocks that take tickets from
 *                          one counter in stage order (edge tiles, then the
 *                          ranking tiles twice -- stencil, then list -- in
 *                          groups of 8, evaluation workers, merge tiles; frames
 *                          in order within a stage), a ticket first waiting
 *                          until the previous stage of its frame has
 *                          finished.  Needs
 *                          frames of at most 4 levels and at most 256
 *                          samples (else MR_E_PARAM); edge_tile,
 *                          eval_queue and eval_blocks_per_cu do not apply.
 *   eval_items          persistent launch: texels per evaluation thread and
 *                       chunk, 1, 2 or 4 (0: 1); the staged evaluation takes
 *                       one (a loop over more cost it a wave per SIMD)
 *   worker_pixels       persistent launch: one evaluation worker ticket per
 *                       this many pixels of a frame (4096 .. 2^24; 0: 8192);
 *                       a frame's workers share its chunks through per-XCD
 *                       counters
 *   tiles_per_ticket    persistent launch: edge and merge tiles per ticket
 *                       (1 .. 64; 0: 16)
 *   eval_halo           SSAO batches that build their masks, staged
 *                       launches with eval_queue = 0 and at most 256
 *                       samples: 0, or 8, 16 or 24 to evaluate every frame's
 *                       dense coarsest level in 16 x 16 texel tiles whose
 *                       depth, with a border of that many texels, is staged
 *                       in LDS (as mr_frame_desc.eval_halo) */
typedef struct mr_batch_config {
    int edge_tile;
    int eval_queue;
    int eval_blocks_per_cu;
    int merge_generic;
    int persistent;
    int eval_items;
    int worker_pixels;
    int tiles_per_ticket;
    int eval_halo;
} mr_batch_config;

/* Read or replace a filled plan's configuration (MR_E_PARAM for a plan not
 * filled by mr_batch_setup or a value out of range; the plan is unchanged
 * then). */
MR_API int mr_batch_get_config(const void* plan, mr_batch_config* cfg);
MR_API int mr_batch_set_config(void* plan, const mr_batch_config* cfg);

/* Autotuner: times the batch (one warm-up run, then `reps` runs, 1..1000) on
 * `stream` under candidate configurations, one choice at a time (the
 * evaluation's schedule and grid cap first, then the edge tile shape and
 * the merge kernel, then for SSAO the LDS depth-tile halo of 8, 16 or 24
 * texels, then the persistent launch with two worker sizes and one or two
 * texels per evaluation thread and, if it is the faster, its tiles per
 * ticket), keeps the
 * fastest in the plan and, when best is not NULL, in *best.  It runs the batch on its current inputs and waits for the
 * stream: not for use under graph capture.  Outputs after it are those of a
 * plain run. */
MR_API int mr_batch_tune(void* plan, int reps, mr_batch_config* best, void* stream);

/* The persistent launch bounds every wait for another stage (it cannot
 * deadlock: each ticket waits only for tickets taken earlier by running
 * blocks); a wait that runs out of polls sets an error word in the
 * workspace and the launch goes on, so it always ends.  mr_batch_check waits
 * for `stream`, reads and clears that word, and returns MR_E_DEVICE if it
 * was set (the outputs of the runs since the last check are then not
 * valid), else MR_OK.  Not for use under graph capture. */
MR_API int mr_batch_check(const void* plan, void* stream);


/* Host helpers. */
MR_API const char* mr_status_string(int status);
MR_API const char* mr_last_error(void);
MR_API int mr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MR_H */
