// Host side of libmr: argument validation, Gaussian taps, workspace layout
// and launch sequencing behind the C ABI declared in include/mr.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <limits>
#include <vector>

#include "mr_internal.hpp"

using namespace mr;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

// prefix the current error message with the frame index of a batch
int fail_frame(int code, int k) {
    char msg[sizeof(g_err)];
    snprintf(msg, sizeof(msg), "%s", g_err);
    return fail(code, "frame %d: %s", k, msg);
}

bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Level geometry of one frame.
struct Geo {
    int N = 0, W = 0, H = 0, L = 0;
    int Wi[kMaxLevels] = {}, Hi[kMaxLevels] = {};
    int levels[kMaxLevels] = {};  // enabled levels ascending (1-based)
    int nlev = 0;
    bool enabled(int i) const {
        for (int j = 0; j < nlev; ++j)
            if (levels[j] == i) return true;
        return false;
    }
    long long n(int i) const { return (long long)Wi[i - 1] * Hi[i - 1]; }
};

int check_geo(const mr_camera* cam, const mr_mask_params* mp, Geo& g) {
    if (!cam) return fail(MR_E_NULL, "camera is NULL");
    int N = 1;
    uint32_t en = 1;
    if (mp) {
        N = mp->num_levels;
        en = mp->level_enable;
        if (N < 1 || N > kMaxLevels) return fail(MR_E_PARAM, "num_levels %d not in [1, %d]", N, kMaxLevels);
        if (!(en & 1u) || !(en & (1u << (N - 1))))
            return fail(MR_E_PARAM, "level_enable 0x%x must contain levels 1 and %d", en, N);
        if (en >> N) return fail(MR_E_PARAM, "level_enable 0x%x names levels above %d", en, N);
    }
    const int W = cam->width, H = cam->height;
    if (W <= 0 || H <= 0 || W > MR_MAX_DIM || H > MR_MAX_DIM)
        return fail(MR_E_SHAPE, "image %dx%d outside [1, %d]", W, H, MR_MAX_DIM);
    const int div = 1 << (N - 1);
    if (W % div || H % div)
        return fail(MR_E_SHAPE, "image %dx%d not divisible by 2^(N-1) = %d", W, H, div);
    if (!(cam->focal_px > 0.0f) || !isfinite(cam->focal_px))
        return fail(MR_E_PARAM, "focal_px must be finite and > 0");
    g.N = N;
    g.W = W;
    g.H = H;
    g.nlev = 0;
    for (int i = 1; i <= N; ++i) {
        g.Wi[i - 1] = W >> (i - 1);
        g.Hi[i - 1] = H >> (i - 1);
        if (en & (1u << (i - 1))) g.levels[g.nlev++] = i;
    }
    g.L = g.levels[g.nlev - 1];
    return MR_OK;
}

// blur radius and normalised Gaussian taps of one level
int gauss(const mr_mask_params* mp, int i, float* taps, int& r) {
    const float s2f = mp->sigma2[i - 1];
    if (!(s2f >= 0.0f) || !isfinite(s2f)) return fail(MR_E_PARAM, "sigma2[%d] must be finite and >= 0", i - 1);
    const int rp = mp->radius[i - 1];
    if (rp < -1) return fail(MR_E_PARAM, "radius[%d] = %d must be >= -1", i - 1, rp);
    const double s2 = (double)s2f;
    if (rp >= 0)
        r = rp;
    else if (s2 <= 0.0)
        r = 0;
    else
        r = (int)ceil(3.0 * sqrt(s2));
    if (r > kMaxRadius) return fail(MR_E_PARAM, "blur radius %d of level %d exceeds %d", r, i, kMaxRadius);
    if (s2 <= 0.0) {
        for (int k = -r; k <= r; ++k) taps[k + r] = k == 0 ? 1.0f : 0.0f;
        return MR_OK;
    }
    double e[2 * kMaxRadius + 1];
    double tot = 0.0;
    for (int k = -r; k <= r; ++k) {
        e[k + r] = exp(-(double)(k * k) / (2.0 * s2));
        tot += e[k + r];
    }
    for (int k = -r; k <= r; ++k) taps[k + r] = (float)(e[k + r] / tot);
    return MR_OK;
}

int check_mask_params(const mr_mask_params* mp, const Geo& g) {
    if (!isfinite(mp->depth_ratio) || !(mp->depth_ratio >= 0.0f))
        return fail(MR_E_PARAM, "depth_ratio must be finite and >= 0");
    if (!(mp->normal_cos >= -1.0f && mp->normal_cos <= 1.0f))
        return fail(MR_E_PARAM, "normal_cos must be in [-1, 1]");
    if (mp->fovea.enable) {
        const mr_fovea& f = mp->fovea;
        if (!isfinite(f.gaze_x) || !isfinite(f.gaze_y) || !isfinite(f.r_inner) || !isfinite(f.r_outer) ||
            !(f.r_inner >= 0.0f) || !(f.r_outer >= 0.0f))
            return fail(MR_E_PARAM, "fovea: gaze and radii must be finite, radii >= 0");
    }
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        float taps[2 * kMaxRadius + 1];
        int r;
        int st = gauss(mp, i, taps, r);
        if (st) return st;
        const float w = mp->weight[i - 1];
        if (!(w > 0.0f) || !isfinite(w)) return fail(MR_E_PARAM, "weight[%d] must be finite and > 0", i - 1);
    }
    return MR_OK;
}

int check_gbuffer(const mr_gbuffer* g, bool need_normal, bool need_color) {
    if (!g) return fail(MR_E_NULL, "gbuffer is NULL");
    if (!g->depth) return fail(MR_E_NULL, "gbuffer.depth is NULL");
    if (misaligned(g->depth)) return fail(MR_E_PARAM, "gbuffer.depth is not 16-byte aligned");
    if (need_normal) {
        if (!g->normal) return fail(MR_E_NULL, "gbuffer.normal is NULL");
        if (misaligned(g->normal)) return fail(MR_E_PARAM, "gbuffer.normal is not 16-byte aligned");
        if (g->normal_dtype != MR_F32 && g->normal_dtype != MR_F16)
            return fail(MR_E_DTYPE, "normal_dtype %d unsupported", g->normal_dtype);
    }
    if (need_color) {
        if (!g->color) return fail(MR_E_NULL, "gbuffer.color is NULL");
        if (misaligned(g->color)) return fail(MR_E_PARAM, "gbuffer.color is not 16-byte aligned");
        if (g->color_dtype != MR_F32 && g->color_dtype != MR_F16)
            return fail(MR_E_DTYPE, "color_dtype %d unsupported", g->color_dtype);
    }
    return MR_OK;
}

// masks needed by the evaluators (need_alpha: also the merge)
int check_masks(const mr_masks* m, const Geo& g, bool need_alpha, bool need_lists) {
    if (!m) return fail(MR_E_NULL, "masks is NULL");
    if (need_lists) {
        if (!m->count) return fail(MR_E_NULL, "masks.count is NULL");
        if (misaligned(m->count)) return fail(MR_E_PARAM, "masks.count is not 16-byte aligned");
    }
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i >= 2 && m->level_depth[i - 1] && misaligned(m->level_depth[i - 1]))
            return fail(MR_E_PARAM, "masks.level_depth[%d] is not 16-byte aligned", i - 1);
        if (i == g.L) continue;
        if (!m->stencil[i - 1]) return fail(MR_E_NULL, "masks.stencil[%d] is NULL", i - 1);
        if (misaligned(m->stencil[i - 1])) return fail(MR_E_PARAM, "masks.stencil[%d] misaligned", i - 1);
        if (need_lists) {
            if (!m->worklist[i - 1]) return fail(MR_E_NULL, "masks.worklist[%d] is NULL", i - 1);
            if (misaligned(m->worklist[i - 1])) return fail(MR_E_PARAM, "masks.worklist[%d] misaligned", i - 1);
        }
        if (need_alpha) {
            if (!m->alpha[i - 1]) return fail(MR_E_NULL, "masks.alpha[%d] is NULL", i - 1);
            if (misaligned(m->alpha[i - 1])) return fail(MR_E_PARAM, "masks.alpha[%d] misaligned", i - 1);
        }
    }
    return MR_OK;
}

int check_outputs(float* const out[kMaxLevels], const Geo& g, bool plain) {
    if (!out) return fail(MR_E_NULL, "out is NULL");
    if (plain) {
        if (!out[0]) return fail(MR_E_NULL, "out[0] is NULL");
        if (misaligned(out[0])) return fail(MR_E_PARAM, "out[0] is not 16-byte aligned");
        return MR_OK;
    }
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (!out[i - 1]) return fail(MR_E_NULL, "out[%d] is NULL", i - 1);
        if (misaligned(out[i - 1])) return fail(MR_E_PARAM, "out[%d] is not 16-byte aligned", i - 1);
    }
    return MR_OK;
}

int check_samples(const float* k, int n, const char* what) {
    if (!k) return fail(MR_E_NULL, "%s is NULL", what);
    if (misaligned(k)) return fail(MR_E_PARAM, "%s is not 16-byte aligned", what);
    if (n < 1 || n > MR_MAX_SAMPLES) return fail(MR_E_PARAM, "%s count %d not in [1, %d]", what, n, MR_MAX_SAMPLES);
    return MR_OK;
}

int check_shadow(const mr_shadow_params* p) {
    if (!p) return fail(MR_E_NULL, "shadow params are NULL");
    if (!p->shadow_map) return fail(MR_E_NULL, "shadow_map is NULL");
    if (misaligned(p->shadow_map)) return fail(MR_E_PARAM, "shadow_map is not 16-byte aligned");
    if (p->sm_size < 1 || p->sm_size > MR_MAX_DIM) return fail(MR_E_SHAPE, "sm_size %d not in [1, %d]", p->sm_size, MR_MAX_DIM);
    for (int k = 0; k < 12; ++k)
        if (!isfinite(p->view_to_light[k])) return fail(MR_E_PARAM, "view_to_light must be finite");
    if (!(p->light_focal_px > 0.0f) || !isfinite(p->light_focal_px)) return fail(MR_E_PARAM, "light_focal_px must be finite and > 0");
    if (!(p->light_size >= 0.0f) || !isfinite(p->light_size)) return fail(MR_E_PARAM, "light_size must be finite and >= 0");
    if (!(p->light_near > 0.0f) || !isfinite(p->light_near)) return fail(MR_E_PARAM, "light_near must be finite and > 0");
    if (!isfinite(p->bias)) return fail(MR_E_PARAM, "bias must be finite");
    int st = check_samples(p->blocker_disk, p->n_blocker, "blocker_disk");
    if (st) return st;
    return check_samples(p->pcf_disk, p->n_pcf, "pcf_disk");
}

int check_sampling(const float* kernel, int S, float r, float b) {
    int st = check_samples(kernel, S, "kernel");
    if (st) return st;
    if (!(r > 0.0f) || !isfinite(r)) return fail(MR_E_PARAM, "radius must be finite and > 0");
    if (!(b >= 0.0f) || !isfinite(b)) return fail(MR_E_PARAM, "bias_rel must be finite and >= 0");
    return MR_OK;
}

// ---------------------------------------------------------------------------
// workspace layouts
// ---------------------------------------------------------------------------
struct MaskScratch {
    size_t Ei_off[kMaxLevels] = {};
    size_t chunk_count_off = 0, chunk_off_off = 0;
    unsigned nchunks = 0;
    size_t bytes = 0;
};

MaskScratch mask_scratch(const Geo& g) {
    MaskScratch s;
    size_t off = 0;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i < 2) continue;
        s.Ei_off[i - 1] = off;
        off += align256((size_t)g.n(i));
    }
    for (int j = 0; j + 1 < g.nlev; ++j) s.nchunks += (unsigned)((g.n(g.levels[j]) + kChunk - 1) / kChunk);
    s.chunk_count_off = off;
    off += align256((size_t)s.nchunks * 4 + 4);
    s.chunk_off_off = off;
    off += align256((size_t)s.nchunks * 4 + 4);
    s.bytes = off;
    return s;
}

struct FrameLayout {
    size_t edge = 0, alpha[kMaxLevels] = {}, stencil[kMaxLevels] = {}, worklist[kMaxLevels] = {};
    size_t level_depth[kMaxLevels] = {}, level_out[kMaxLevels] = {}, count = 0, hard = 0, scratch = 0;
    size_t bytes = 0;
};

FrameLayout frame_layout(const Geo& g, int effect) {
    FrameLayout f;
    const int C = effect == MR_EFFECT_SSGI ? 3 : 1;
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += align256(n);
        return o;
    };
    f.edge = take((size_t)g.W * g.H);
    f.count = take(4 * kMaxLevels);
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        const size_t n = (size_t)g.n(i);
        if (i != g.L) {
            f.alpha[i - 1] = take(4 * n);
            f.stencil[i - 1] = take(n);
            f.worklist[i - 1] = take(4 * n);
        }
        if (i >= 2) f.level_depth[i - 1] = take(4 * n);
        f.level_out[i - 1] = take(4 * n * C);
    }
    if (effect == MR_EFFECT_SHADOW) f.hard = take((size_t)g.W * g.H);
    f.scratch = off;
    off += mask_scratch(g).bytes;
    f.bytes = off;
    return f;
}

// ---------------------------------------------------------------------------
// lean frame path eligibility and layout
// ---------------------------------------------------------------------------
// The lean path stores the stencils as bits and a_i / sub-image values only at
// stencil texels.  It needs: the coarsest enabled level L <= 4 (bit outputs
// exist for levels 1..3), W divisible by 128 (whole bit words per row at
// levels 1..3), and for every enabled level below L a radius <= 8 whose
// Gaussian taps are all positive with no product of two taps underflowing
// (then a_i > 0 exactly on the Chebyshev dilation of the pooled edges), and
// radii for which the nesting step changes nothing (r_j >= ceil(r_i / k)).
// ranking tiles of a level with wpr words per row and H rows
unsigned lean_tiles(int wpr, int H) {
    return (unsigned)((wpr + kLeanTileWords - 1) / kLeanTileWords) * (unsigned)((H + kLeanTileRows - 1) / kLeanTileRows);
}

bool lean_ok(const Geo& g, const mr_mask_params* mp) {
    if (g.L > 4 || g.nlev < 2 || g.W % 128 != 0) return false;
    int radius[kMaxLevels] = {};
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        float taps[2 * kMaxRadius + 1];
        int r;
        if (gauss(mp, i, taps, r)) return false;
        if (r > kBlurFusedMaxRadius) return false;
        float gmin = 1.0f;
        for (int k = 0; k <= 2 * r; ++k) gmin = taps[k] < gmin ? taps[k] : gmin;
        // smallest positive binary32 (denormal) is 2^-149
        if (!(gmin > 0.0f) || (double)gmin * (double)gmin < ldexp(1.0, -149)) return false;
        radius[i - 1] = r;
    }
    for (int j = 0; j + 2 < g.nlev; ++j) {
        const int fi = g.levels[j], ci = g.levels[j + 1];
        const int k = 1 << (ci - fi);
        if (radius[ci - 1] < (radius[fi - 1] + k - 1) / k) return false;
    }
    return true;
}


// The compact layout in two parts.  The mask pyramid (counts, tile totals,
// edge and stencil bits, ranks, work lists and point-sampled level depth)
// depends only on the frame's inputs; the scratch part (a_i and sub-image
// values by rank, the coarsest level, hard-shadow bits, blurred values) is
// rewritten by every frame.  Offsets of the pyramid fields are from the
// pyramid's base, those of the scratch fields from the scratch's base;
// mr_frame places the scratch right after the pyramid.
struct LeanLayout {
    size_t count = 0, tot = 0, Eb[3] = {}, Sb[3] = {}, woff[3] = {}, list[3] = {}, zi[kMaxLevels] = {};
    size_t pyramid = 0;  // bytes of the pyramid part
    size_t ac[3] = {}, cc[3] = {}, cL = 0, hard = 0;
    size_t bc[3] = {}, bL = 0;  // SSAO: bilaterally blurred values
    size_t scratch = 0;  // bytes of the scratch part
    unsigned nblk = 0;
    size_t bytes = 0;    // pyramid + scratch
};

LeanLayout lean_layout(const Geo& g, int effect) {
    LeanLayout f;
    const int C = effect == MR_EFFECT_SSGI ? 3 : 1;
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += align256(n);
        return o;
    };
    for (int j = 0; j + 1 < g.nlev; ++j) f.nblk += lean_tiles(g.Wi[g.levels[j] - 1] / 32, g.Hi[g.levels[j] - 1]);
    f.count = take(4 * kMaxLevels);
    f.tot = take(4 * (size_t)f.nblk);  // per ranking tile: its stencil texels
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        const size_t n = (size_t)g.n(i);
        const size_t words = (size_t)(g.Wi[i - 1] / 32) * g.Hi[i - 1];
        f.Eb[i - 1] = take(4 * words);
        f.Sb[i - 1] = take(4 * words);
        f.woff[i - 1] = take(4 * words);
        f.list[i - 1] = take(4 * n);
    }
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i >= 2) f.zi[i - 1] = take(4 * (size_t)g.n(i));
    }
    f.pyramid = off;
    off = 0;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        const size_t n = (size_t)g.n(i);
        f.ac[i - 1] = take(4 * n);
        f.cc[i - 1] = take(4 * n * C);
    }
    f.cL = take(4 * (size_t)g.n(g.L) * C);
    if (effect == MR_EFFECT_SHADOW) f.hard = take((size_t)g.W * g.H);
    if (effect == MR_EFFECT_SSAO) {
        for (int j = 0; j + 1 < g.nlev; ++j) {
            const int i = g.levels[j];
            f.bc[i - 1] = take(4 * (size_t)g.n(i));
        }
        f.bL = take(4 * (size_t)g.n(g.L));
    }
    f.scratch = off;
    f.bytes = f.pyramid + f.scratch;
    return f;
}

// ---------------------------------------------------------------------------
// pipeline pieces (arguments already validated)
// ---------------------------------------------------------------------------
// importance mask of a gaze point: squared radii in FP32
void set_fovea(EdgeArgs& ea, const mr_mask_params* mp) {
    ea.fov = mp->fovea.enable ? 1 : 0;
    ea.fgx = mp->fovea.gaze_x;
    ea.fgy = mp->fovea.gaze_y;
    ea.fri2 = mp->fovea.r_inner * mp->fovea.r_inner;
    ea.fro2 = mp->fovea.r_outer * mp->fovea.r_outer;
}

int do_build_masks(const mr_gbuffer* gb, const Geo& g, const mr_mask_params* mp, const uint8_t* hard,
                   const mr_masks* m, void* ws, hipStream_t s) {
    const MaskScratch sc = mask_scratch(g);
    uint8_t* base = static_cast<uint8_t*>(ws);
    EdgeArgs ea{};
    ea.depth = gb->depth;
    ea.normal = gb->normal;
    ea.hard = hard;
    ea.W = g.W;
    ea.H = g.H;
    ea.depth_ratio = mp->depth_ratio;
    ea.normal_cos = mp->normal_cos;
    set_fovea(ea, mp);
    ea.E = m->edge;
    ea.num_levels = g.N;
    uint8_t* Ei[kMaxLevels] = {};
    for (int i = 1; i <= g.N; ++i) {
        ea.Wi[i - 1] = g.Wi[i - 1];
        ea.Hi[i - 1] = g.Hi[i - 1];
    }
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i >= 2) ea.zi[i - 1] = m->level_depth[i - 1];
        if (i == g.L) continue;
        Ei[i - 1] = i == 1 ? m->edge : base + sc.Ei_off[i - 1];
        if (i >= 2) ea.Ei[i - 1] = Ei[i - 1];
    }
    if (launch_edges(ea, gb->normal_dtype, s) != hipSuccess) return fail(MR_E_DEVICE, "edge kernel launch failed");
    int radius[kMaxLevels] = {};
    BlurArgs ba{};
    unsigned tiles = 0;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        BlurLevel bl{};
        int r;
        gauss(mp, i, bl.g, r);
        radius[i - 1] = r;
        bl.Ei = Ei[i - 1];
        bl.a = m->alpha[i - 1];
        bl.S = m->stencil[i - 1];
        bl.W = g.Wi[i - 1];
        bl.H = g.Hi[i - 1];
        bl.r = r;
        bl.tiles_x = (unsigned)((bl.W + 255) / 256);
        if (r > kBlurFusedMaxRadius) {
            if (launch_blur_wide(bl, s) != hipSuccess) return fail(MR_E_DEVICE, "blur kernel launch failed");
            continue;
        }
        bl.tile_base = tiles;
        tiles += bl.tiles_x * (unsigned)((bl.H + 31) / 32);
        ba.lv[ba.nlev++] = bl;
    }
    ba.ntiles = tiles;
    if (launch_blur(ba, s) != hipSuccess) return fail(MR_E_DEVICE, "blur kernel launch failed");
    // Nesting: S_j |= pool(S_i) for consecutive enabled i < j < L.  When every
    // earlier pair was a no-op, S_i is the Chebyshev dilation of E_i by r_i
    // and the pair is a no-op too if r_j >= ceil(r_i / k); only pairs that can
    // change anything are launched.
    bool dirty = false;
    for (int j = 0; j + 2 < g.nlev; ++j) {
        const int fi = g.levels[j], ci = g.levels[j + 1];
        const int k = 1 << (ci - fi);
        if (!dirty && radius[ci - 1] >= (radius[fi - 1] + k - 1) / k) continue;
        dirty = true;
        NestArgs na{m->stencil[fi - 1], m->stencil[ci - 1], g.Wi[fi - 1], g.Hi[fi - 1], g.Wi[ci - 1], g.Hi[ci - 1], k};
        if (launch_nest(na, s) != hipSuccess) return fail(MR_E_DEVICE, "nesting kernel launch failed");
    }
    if (m->level_map) {
        LevelMapArgs la{};
        la.nlev = g.nlev;
        for (int j = 0; j < g.nlev; ++j) {
            la.levels[j] = g.levels[j];
            la.S[j] = m->stencil[g.levels[j] - 1];
            la.Wi[j] = g.Wi[g.levels[j] - 1];
        }
        la.W = g.W;
        la.H = g.H;
        la.out = m->level_map;
        if (launch_level_map(la, s) != hipSuccess) return fail(MR_E_DEVICE, "level map kernel launch failed");
    }
    CompactArgs ca{};
    ca.nlev = g.nlev - 1;
    unsigned cb = 0;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        ca.S[j] = m->stencil[i - 1];
        ca.list[j] = m->worklist[i - 1];
        ca.n[j] = (uint32_t)g.n(i);
        ca.chunk_base[j] = cb;
        ca.count_idx[j] = i - 1;
        cb += (unsigned)((g.n(i) + kChunk - 1) / kChunk);
    }
    ca.chunk_base[ca.nlev] = cb;
    ca.chunk_count = reinterpret_cast<uint32_t*>(base + sc.chunk_count_off);
    ca.chunk_off = reinterpret_cast<uint32_t*>(base + sc.chunk_off_off);
    ca.count = m->count;
    if (launch_compact(ca, s) != hipSuccess) return fail(MR_E_DEVICE, "compaction kernel launch failed");
    return MR_OK;
}

// per-level views for an evaluation pass; returns the worst-case item count
unsigned make_eval_common(const mr_gbuffer* gb, const Geo& g, const mr_masks* m, float* const out[kMaxLevels],
                          int C, EvalCommon& c) {
    c.counts = m ? m->count : nullptr;
    c.normal = gb->normal;
    c.color = gb->color;
    c.plane = (long long)g.W * g.H;
    unsigned hint = 0;
    const int nl = m ? g.nlev : 1;
    c.nlev = nl;
    for (int j = 0; j < nl; ++j) {
        const int i = m ? g.levels[j] : 1;
        const int sft = i - 1, sc = 1 << sft;
        EvalLevel& L = c.lv[j];
        L.W = g.Wi[i - 1];
        L.H = g.Hi[i - 1];
        if (i == 1) {
            L.z = gb->depth;
            L.zpy = g.W;
            L.zpx = 1;
            L.goff = 0;
        } else {
            const long long off = (long long)(sc / 2) * g.W + sc / 2;
            if (m && m->level_depth[i - 1]) {
                L.z = m->level_depth[i - 1];
                L.zpy = L.W;
                L.zpx = 1;
            } else {
                L.z = gb->depth + off;
                L.zpy = sc * g.W;
                L.zpx = sc;
            }
            L.goff = off;
        }
        L.gpy = (long long)sc * g.W;
        L.gpx = sc;
        L.out = out[i - 1];
        L.out_plane = (long long)L.W * L.H;
        L.stream = m ? 0 : 1;  // without masks the output is the full-resolution image
        const bool dense = !m || i == g.L;
        L.list = dense ? nullptr : m->worklist[i - 1];
        L.count_idx = i - 1;
        L.dense_n = (unsigned)((long long)L.W * L.H);
        hint += L.dense_n;
        (void)C;
    }
    return hint;
}

void set_level_cameras(const mr_camera* cam, const Geo& g, EvalCommon& c, bool plain) {
    for (int j = 0; j < c.nlev; ++j) {
        const int i = plain ? 1 : g.levels[j];
        EvalLevel& L = c.lv[j];
        L.f = cam->focal_px / (float)(1 << (i - 1));
        L.cx = 0.5f * (float)L.W;
        L.cy = 0.5f * (float)L.H;
    }
}

// compact: list levels write their results at the list position; lean (with
// compact) also has the evaluators write a_i at the list position
// Kernel arguments of one evaluation launch (one effect).
struct EvalPlan {
    int effect = MR_EFFECT_SSAO;
    SsaoArgs sa{};
    ShadowArgs sh{};
    SsgiArgs gi{};
    unsigned hint = 0;
};

// compact: list levels write their results at the list position; lean (with
// compact) also has the evaluators write a_i at the list position
void build_eval(int effect, const mr_gbuffer* gb, const mr_camera* cam, const Geo& g, const mr_masks* m,
                const void* params, float* const out[kMaxLevels], bool compact, const LeanArgs* lean, bool out16,
                EvalPlan& E) {
    auto set_compact = [&](EvalCommon& c) {
        for (int j = 0; j < c.nlev; ++j) c.lv[j].out16 = out16 ? 1 : 0;
        if (!compact) return;
        for (int j = 0; j < c.nlev; ++j) {
            EvalLevel& L = c.lv[j];
            if (!L.list) continue;
            L.compact = 1;
            if (lean) {
                const LeanLevel& A = lean->lv[j];
                L.ac = A.ac;
                L.Eb = A.Eb;
                L.Ewpr = A.wpr;
                L.Er = A.r;
                for (int k = 0; k <= 2 * A.r; ++k) L.Eg[k] = A.g[k];
            }
        }
    };
    const int C = effect == MR_EFFECT_SSGI ? 3 : 1;
    E.effect = effect;
    if (effect == MR_EFFECT_SSAO) {
        const mr_ssao_params* p = static_cast<const mr_ssao_params*>(params);
        SsaoArgs& a = E.sa;
        E.hint = make_eval_common(gb, g, m, out, C, a.c);
        set_level_cameras(cam, g, a.c, !m);
        set_compact(a.c);
        a.kernel = p->kernel;
        a.S = p->samples;
        a.r = p->radius;
        a.b = p->bias_rel;
    } else if (effect == MR_EFFECT_SHADOW) {
        const mr_shadow_params* p = static_cast<const mr_shadow_params*>(params);
        ShadowArgs& a = E.sh;
        E.hint = make_eval_common(gb, g, m, out, C, a.c);
        set_level_cameras(cam, g, a.c, !m);
        set_compact(a.c);
        a.sm = p->shadow_map;
        a.size = p->sm_size;
        memcpy(a.M, p->view_to_light, sizeof(a.M));
        a.fL = p->light_focal_px;
        a.lsize = p->light_size;
        a.nL = p->light_near;
        a.bias = p->bias;
        a.bd = p->blocker_disk;
        a.pd = p->pcf_disk;
        a.nb = p->n_blocker;
        a.np = p->n_pcf;
    } else {
        const mr_ssgi_params* p = static_cast<const mr_ssgi_params*>(params);
        SsgiArgs& a = E.gi;
        E.hint = make_eval_common(gb, g, m, out, C, a.c);
        set_level_cameras(cam, g, a.c, !m);
        set_compact(a.c);
        a.kernel = p->kernel;
        a.S = p->samples;
        a.r = p->radius;
        a.b = p->bias_rel;
    }
}

int launch_eval(const EvalPlan& E, int normal_dtype, int color_dtype, hipStream_t s) {
    hipError_t e;
    if (E.effect == MR_EFFECT_SSAO)
        e = launch_ssao(E.sa, normal_dtype, E.hint, s);
    else if (E.effect == MR_EFFECT_SHADOW)
        e = launch_shadow(E.sh, E.hint, s);
    else
        e = launch_ssgi(E.gi, normal_dtype, color_dtype, E.hint, s);
    if (e != hipSuccess) return fail(MR_E_DEVICE, "evaluation kernel launch failed: %s", hipGetErrorString(e));
    return MR_OK;
}

int do_eval(int effect, const mr_gbuffer* gb, const mr_camera* cam, const Geo& g, const mr_masks* m,
            const void* params, float* const out[kMaxLevels], hipStream_t s, bool compact = false,
            const LeanArgs* lean = nullptr, bool out16 = false) {
    EvalPlan E;
    build_eval(effect, gb, cam, g, m, params, out, compact, lean, out16, E);
    return launch_eval(E, gb->normal_dtype, gb->color_dtype, s);
}

int do_merge(const Geo& g, const mr_mask_params* mp, const mr_masks* m, const float* const lo[kMaxLevels], int C,
             float* out, hipStream_t s) {
    MergeArgs a{};
    a.nlev = g.nlev;
    a.W = g.W;
    a.H = g.H;
    a.C = C;
    a.out = out;
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        MergeLevel& L = a.lv[j];
        L.c = lo[i - 1];
        L.c_plane = g.n(i);
        L.sh = i - 1;
        L.s = 1 << L.sh;
        L.W = g.Wi[i - 1];
        L.H = g.Hi[i - 1];
        L.w = mp->weight[i - 1];
        L.a = i == g.L ? nullptr : m->alpha[i - 1];
        L.S = i == g.L ? nullptr : m->stencil[i - 1];
        if (L.s >= 2) {
            // taps of a tile's columns x0 .. x0 + 63 lie in (x0 >> sh) - 1 ..
            // (x0 >> sh) + ceil(64 / s); rows likewise for 16 rows
            L.rw = (kMergeTW + L.s - 1) / L.s + 2;
            L.rh = (kMergeTH + L.s - 1) / L.s + 2;
            L.roff = a.staged;
            L.rmagic = (65536u + (unsigned)L.rw - 1) / (unsigned)L.rw;
            a.staged += L.rw * L.rh;
        }
    }
    if (launch_merge(a, s) != hipSuccess) return fail(MR_E_DEVICE, "merge kernel launch failed");
    return MR_OK;
}

int check_effect_params(int effect, const mr_ssao_params* ssao, const mr_shadow_params* sh, const mr_ssgi_params* gi) {
    if (effect == MR_EFFECT_SSAO) {
        if (!ssao) return fail(MR_E_NULL, "ssao params are NULL");
        return check_sampling(ssao->kernel, ssao->samples, ssao->radius, ssao->bias_rel);
    }
    if (effect == MR_EFFECT_SHADOW) return check_shadow(sh);
    if (effect == MR_EFFECT_SSGI) {
        if (!gi) return fail(MR_E_NULL, "ssgi params are NULL");
        return check_sampling(gi->kernel, gi->samples, gi->radius, gi->bias_rel);
    }
    return fail(MR_E_PARAM, "unknown effect %d", effect);
}

// records the caller's stage event k, if any, on the frame's stream
int mark(const mr_frame_desc* d, int k, hipStream_t s) {
    void* e = d->stage_events[k];
    if (!e) return MR_OK;
    const hipError_t r = hipEventRecord(static_cast<hipEvent_t>(e), s);
    if (r != hipSuccess) return fail(MR_E_DEVICE, "stage event %d: %s", k, hipGetErrorString(r));
    return MR_OK;
}

// eval_halo: 0, or an LDS halo for the SSAO evaluation of the dense coarsest
// level (multi-resolution SSAO frames of at most kTiledSamples samples)
constexpr int kTiledSamplesHost = 256;
constexpr int kFrameHalos = 4;  // eval_halo choices of mr_frame_tune
int check_halo(const mr_frame_desc* d) {
    const int h = d->eval_halo;
    if (h == 0) return MR_OK;
    if (h != 8 && h != 16 && h != 24) return fail(MR_E_PARAM, "eval_halo %d is not 0, 8, 16 or 24", h);
    if (d->effect != MR_EFFECT_SSAO || !d->multires)
        return fail(MR_E_PARAM, "eval_halo applies to multi-resolution MR_EFFECT_SSAO frames only");
    if (d->ssao->samples > kTiledSamplesHost)
        return fail(MR_E_PARAM, "eval_halo needs at most %d samples", kTiledSamplesHost);
    return MR_OK;
}

int check_bilateral(const mr_frame_desc* d, const Geo& g) {
    const mr_bilateral_params& p = d->bilateral;
    if (!p.levels) return MR_OK;
    if (d->effect != MR_EFFECT_SSAO) return fail(MR_E_PARAM, "the bilateral blur applies to MR_EFFECT_SSAO only");
    if (!lean_ok(g, &d->mp))
        return fail(MR_E_PARAM, "the bilateral blur needs the compact frame path (coarsest level <= 4, width "
                                "divisible by 128, blur radii <= 8)");
    uint32_t enabled = 0;
    for (int j = 0; j < g.nlev; ++j) enabled |= 1u << (g.levels[j] - 1);
    if (p.levels & ~enabled)
        return fail(MR_E_PARAM, "bilateral levels 0x%x name levels that are not enabled (0x%x)", p.levels, enabled);
    if (p.radius != 1 && p.radius != 2) return fail(MR_E_PARAM, "bilateral radius %d is not 1 or 2", p.radius);
    if (!(p.depth_rel > 0.0f) || !isfinite(p.depth_rel))
        return fail(MR_E_PARAM, "bilateral depth_rel %g is not finite and > 0", (double)p.depth_rel);
    return MR_OK;
}

// Kernel arguments of one frame on the compact path, laid out in the
// frame's workspace b.
struct LeanPlan {
    bool has_hard = false, has_map = false, has_bl = false;
    BilateralArgs bl{};
    HardArgs ha{};
    EdgeArgs ea{};
    LeanArgs la{};
    LeanMapArgs lm{};
    EvalPlan ev;
    LeanMergeArgs ma{};
};

// pyr: the mask pyramid; scr: the frame's scratch (see LeanLayout)
void build_lean(const mr_frame_desc* d, const Geo& g, const void* params, uint8_t* pyr, uint8_t* scr, LeanPlan& P) {
    const int effect = d->effect;
    const int C = effect == MR_EFFECT_SSGI ? 3 : 1;
    const LeanLayout f = lean_layout(g, effect);
    uint8_t* const b = pyr;
    uint32_t* count = reinterpret_cast<uint32_t*>(b + f.count);
    const uint8_t* hard = nullptr;
    if (effect == MR_EFFECT_SHADOW) {
        HardArgs& ha = P.ha;
        ha.depth = d->g.depth;
        ha.W = g.W;
        ha.H = g.H;
        ha.f = d->cam.focal_px;
        ha.sm = d->shadow->shadow_map;
        ha.size = d->shadow->sm_size;
        memcpy(ha.M, d->shadow->view_to_light, sizeof(ha.M));
        ha.fL = d->shadow->light_focal_px;
        ha.bias = d->shadow->bias;
        ha.hard = scr + f.hard;
        P.has_hard = true;
        hard = scr + f.hard;
    }
    // edges as bits, point-sampled level depth
    EdgeArgs& ea = P.ea;
    ea.depth = d->g.depth;
    ea.normal = d->g.normal;
    ea.hard = hard;
    ea.W = g.W;
    ea.H = g.H;
    ea.depth_ratio = d->mp.depth_ratio;
    ea.normal_cos = d->mp.normal_cos;
    set_fovea(ea, &d->mp);
    ea.num_levels = g.N;
    for (int i = 1; i <= g.N; ++i) {
        ea.Wi[i - 1] = g.Wi[i - 1];
        ea.Hi[i - 1] = g.Hi[i - 1];
    }
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i >= 2) ea.zi[i - 1] = reinterpret_cast<float*>(b + f.zi[i - 1]);
        if (i < g.L) {
            ea.Eb[i - 1] = reinterpret_cast<uint32_t*>(b + f.Eb[i - 1]);
            ea.wpr[i - 1] = g.Wi[i - 1] / 32;
        }
    }
    // the edge kernel zeroes the level counts (those of levels without a
    // list stay 0; the ranking writes the others)
    ea.zero = count;
    ea.zero_n = kMaxLevels;
    // stencils, ranks, lists (a_i at listed texels comes with the evaluation)
    LeanArgs& la = P.la;
    la.nlev = g.nlev - 1;
    la.count = count;
    la.tot = reinterpret_cast<uint32_t*>(b + f.tot);
    unsigned blk = 0;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        LeanLevel& L = la.lv[j];
        L.Eb = reinterpret_cast<uint32_t*>(b + f.Eb[i - 1]);
        L.Sb = reinterpret_cast<uint32_t*>(b + f.Sb[i - 1]);
        L.woff = reinterpret_cast<uint32_t*>(b + f.woff[i - 1]);
        L.list = reinterpret_cast<uint32_t*>(b + f.list[i - 1]);
        L.ac = reinterpret_cast<float*>(scr + f.ac[i - 1]);
        L.W = g.Wi[i - 1];
        L.H = g.Hi[i - 1];
        L.wpr = L.W / 32;
        gauss(&d->mp, i, L.g, L.r);
        L.nwords = (unsigned)L.wpr * (unsigned)L.H;
        L.tiles_x = (L.wpr + kLeanTileWords - 1) / kLeanTileWords;
        L.blk_base = blk;
        L.ntiles = lean_tiles(L.wpr, L.H);
        L.count_idx = i - 1;
        blk += L.ntiles;
    }
    la.nblk = blk;
    if (d->level_map) {
        LeanMapArgs& lm = P.lm;
        lm.nlev = g.nlev - 1;
        for (int j = 0; j + 1 < g.nlev; ++j) {
            lm.Sb[j] = la.lv[j].Sb;
            lm.wpr[j] = la.lv[j].wpr;
            lm.level[j] = g.levels[j];
        }
        lm.coarsest = g.L;
        lm.W = g.W;
        lm.H = g.H;
        lm.out = d->level_map;
        P.has_map = true;
    }
    // per-level evaluation, list levels written by rank
    mr_masks m{};
    m.count = count;
    float* lo[kMaxLevels] = {};
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i >= 2) m.level_depth[i - 1] = reinterpret_cast<float*>(b + f.zi[i - 1]);
        if (i < g.L) {
            m.worklist[i - 1] = reinterpret_cast<uint32_t*>(b + f.list[i - 1]);
            lo[i - 1] = reinterpret_cast<float*>(scr + f.cc[i - 1]);
        } else {
            lo[i - 1] = reinterpret_cast<float*>(scr + f.cL);
        }
    }
    build_eval(effect, &d->g, &d->cam, g, &m, params, lo, /*compact=*/true, &la, d->level_dtype == MR_F16, P.ev);
    if (effect == MR_EFFECT_SSAO && d->eval_halo) {
        P.ev.sa.halo = d->eval_halo;
        P.ev.sa.c.dense_tiles = 1;
    }
    // bilateral blur of chosen SSAO levels into their second buffers
    void* merged[kMaxLevels] = {};
    for (int j = 0; j < g.nlev; ++j) merged[g.levels[j] - 1] = lo[g.levels[j] - 1];
    if (effect == MR_EFFECT_SSAO && d->bilateral.levels) {
        BilateralArgs& bl = P.bl;
        bl.counts = count;
        bl.R = d->bilateral.radius;
        bl.drel = d->bilateral.depth_rel;
        bl.c16 = d->level_dtype == MR_F16 ? 1 : 0;
        for (int k = 0; k <= 2 * bl.R; ++k) {
            int binom = 1;  // C(2R, k)
            for (int q = 0; q < k; ++q) binom = binom * (2 * bl.R - q) / (q + 1);
            bl.wb[k] = (float)binom / (float)(1 << (2 * bl.R));
        }
        for (int j = 0; j < g.nlev; ++j) {
            const int i = g.levels[j];
            if (!((d->bilateral.levels >> (i - 1)) & 1u)) continue;
            BilateralLevel& B = bl.lv[bl.nlev++];
            B.z = i == 1 ? d->g.depth : reinterpret_cast<const float*>(b + f.zi[i - 1]);
            B.c = lo[i - 1];
            B.out = scr + (i < g.L ? f.bc[i - 1] : f.bL);
            B.W = g.Wi[i - 1];
            B.H = g.Hi[i - 1];
            B.dense_n = (unsigned)g.n(i);
            if (i < g.L) {
                B.list = la.lv[j].list;
                B.Sb = la.lv[j].Sb;
                B.woff = la.lv[j].woff;
                B.wpr = la.lv[j].wpr;
                B.count_idx = la.lv[j].count_idx;
            }
            merged[i - 1] = B.out;
        }
        P.has_bl = bl.nlev > 0;
    }
    // merge by rank
    LeanMergeArgs& ma = P.ma;
    ma.nlev = g.nlev;
    ma.W = g.W;
    ma.H = g.H;
    ma.C = C;
    ma.out = d->out;
    ma.fine1 = true;
    ma.c16 = d->level_dtype == MR_F16;
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        LeanMergeLevel& L = ma.lv[j];
        L.sh = i - 1;
        L.s = 1 << L.sh;
        L.W = g.Wi[i - 1];
        L.H = g.Hi[i - 1];
        L.w = d->mp.weight[i - 1];
        L.c = merged[i - 1];
        L.c_plane = g.n(i);
        if (i < g.L) {
            L.Sb = la.lv[j].Sb;
            L.woff = la.lv[j].woff;
            L.ac = la.lv[j].ac;
            L.wpr = la.lv[j].wpr;
        }
        if (L.s >= 2) {
            L.rw = (kMergeTW + L.s - 1) / L.s + 2;
            L.rh = (kMergeTH + L.s - 1) / L.s + 2;
            L.roff = ma.staged;
            L.rmagic = (65536u + (unsigned)L.rw - 1) / (unsigned)L.rw;
            // each level's region starts on a whole wave of staging slots,
            // so that a wave stages one level (its parameters are scalar)
            ma.staged += (L.rw * L.rh + 63) & ~63;
        }
    }
}

// build = false: the pyramid already holds this frame's masks; the mask
// kernels are skipped
int do_frame_lean(const mr_frame_desc* d, const Geo& g, const void* params, uint8_t* pyr, uint8_t* scr, bool build,
                  hipStream_t s) {
    LeanPlan P;
    build_lean(d, g, params, pyr, scr, P);
    int st = mark(d, 0, s);
    if (st) return st;
    if (build) {
        if (P.has_hard && launch_hard(P.ha, s) != hipSuccess)
            return fail(MR_E_DEVICE, "hard shadow kernel launch failed");
        if (launch_edges(P.ea, d->g.normal_dtype, s) != hipSuccess) return fail(MR_E_DEVICE, "edge kernel launch failed");
        if ((st = mark(d, 4, s))) return st;
        if (launch_lean_masks(P.la, s) != hipSuccess) return fail(MR_E_DEVICE, "lean mask kernels launch failed");
    } else if ((st = mark(d, 4, s))) {
        return st;
    }
    if (P.has_map && launch_lean_level_map(P.lm, s) != hipSuccess)
        return fail(MR_E_DEVICE, "level map kernel launch failed");
    if ((st = mark(d, 1, s))) return st;
    if ((st = launch_eval(P.ev, d->g.normal_dtype, d->g.color_dtype, s))) return st;
    if (P.has_bl && launch_bilateral(P.bl, P.ev.hint, s) != hipSuccess)
        return fail(MR_E_DEVICE, "bilateral blur kernel launch failed");
    if ((st = mark(d, 2, s))) return st;
    if (launch_lean_merge(P.ma, s) != hipSuccess) return fail(MR_E_DEVICE, "merge kernel launch failed");
    return mark(d, 3, s);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
constexpr uint32_t kBatchMagic = 0x3142524du;  // "MRB1"

struct BatchPlan {
    uint32_t magic;
    int n, effect, ndt, cdt, S, C;
    bool c16, m4_ok, wide_ok;
    int merge_geo;  // merge kernel of the frames (merge_geometry) when merge_generic = 0
    bool cached;  // evaluation and merge on resident mask pyramids only
    mr_batch_config cfg;
    const EdgeArgs* te;
    const LeanArgs* tl;
    const void* tv;  // SsaoArgs or SsgiArgs
    const LeanMergeArgs* tm;
    const unsigned *edge_base[2], *edge_tx[2], *rank_base, *merge_base, *merge_tx, *px;
    unsigned* queue;
    unsigned* fused_ctr;
    unsigned edge_total[2], rank_total, eval_hint, merge_total;
};
static_assert(sizeof(BatchPlan) <= MR_BATCH_PLAN_BYTES, "batch plan exceeds MR_BATCH_PLAN_BYTES");

// per-frame tables in the batch workspace: edge tile bases and tiles per row
// for both edge tile shapes, rank block bases, merge tile bases and tiles per
// row, pixel counts; then the evaluation's work-queue counters and the
// persistent launch's counters
constexpr int kBatchTables = 8;
// persistent launch defaults (the fastest measured on 24 uneven SSGI frames)
constexpr int kDefaultWorkerPixels = 8192;
constexpr int kDefaultTilesPerTicket = 16;
// polls of a persistent-launch wait before it gives up (tens of ms or more;
// a wait for another stage of the same frame normally lasts well under 1 ms)
constexpr unsigned kFusedSpinLimit = 1u << 18;

// the persistent launch: edge tiles of 256 x 8 pixels (at most 4 levels)
// and at most kFusedSamples samples
bool fused_ok(const BatchPlan& P) { return P.wide_ok && P.S <= kFusedSamples; }

struct BatchLayout {
    size_t te, tl, tv, tm, bases, frames[MR_MAX_BATCH], bytes;
};

int check_batch(const mr_frame_desc* fr, int n, Geo* geos) {
    if (!fr) return fail(MR_E_NULL, "frames are NULL");
    if (n < 1 || n > MR_MAX_BATCH) return fail(MR_E_PARAM, "batch size %d outside [1, %d]", n, MR_MAX_BATCH);
    const mr_frame_desc& f0 = fr[0];
    if (f0.effect != MR_EFFECT_SSAO && f0.effect != MR_EFFECT_SSGI)
        return fail(MR_E_PARAM, "batches take MR_EFFECT_SSAO or MR_EFFECT_SSGI frames");
    for (int k = 0; k < n; ++k) {
        const mr_frame_desc& d = fr[k];
        if (d.effect != f0.effect) return fail(MR_E_PARAM, "frame %d: effect differs from frame 0", k);
        if (!d.multires) return fail(MR_E_PARAM, "frame %d: batches are multi-resolution only", k);
        if (d.level_map) return fail(MR_E_PARAM, "frame %d: level_map is not produced in batches", k);
        if (d.bilateral.levels) return fail(MR_E_PARAM, "frame %d: batches do not apply the bilateral blur", k);
        if (d.eval_halo) return fail(MR_E_PARAM, "frame %d: eval_halo applies to single frames", k);
        const void* p = d.effect == MR_EFFECT_SSAO ? (const void*)d.ssao : (const void*)d.ssgi;
        const void* p0 = f0.effect == MR_EFFECT_SSAO ? (const void*)f0.ssao : (const void*)f0.ssgi;
        int st = check_effect_params(d.effect, d.ssao, d.shadow, d.ssgi);
        if (st) return fail_frame(st, k);
        if (memcmp(p, p0, d.effect == MR_EFFECT_SSAO ? sizeof(mr_ssao_params) : sizeof(mr_ssgi_params)) != 0)
            return fail(MR_E_PARAM, "frame %d: effect parameters differ from frame 0", k);
        if (memcmp(&d.mp, &f0.mp, sizeof(mr_mask_params)) != 0)
            return fail(MR_E_PARAM, "frame %d: mask parameters differ from frame 0", k);
        if (d.g.normal_dtype != f0.g.normal_dtype || (d.effect == MR_EFFECT_SSGI && d.g.color_dtype != f0.g.color_dtype))
            return fail(MR_E_DTYPE, "frame %d: input types differ from frame 0", k);
        if (d.level_dtype != f0.level_dtype || (d.level_dtype != MR_F32 && d.level_dtype != MR_F16))
            return fail(MR_E_DTYPE, "frame %d: level_dtype differs from frame 0 or is invalid", k);
        if (!d.out) return fail(MR_E_NULL, "frame %d: out is NULL", k);
        if (misaligned(d.out)) return fail(MR_E_PARAM, "frame %d: out is not 16-byte aligned", k);
        Geo& g = geos[k];
        st = check_geo(&d.cam, &d.mp, g);
        if (!st) st = check_mask_params(&d.mp, g);
        if (!st) st = check_gbuffer(&d.g, true, d.effect == MR_EFFECT_SSGI);
        if (st) return fail_frame(st, k);
        if (!lean_ok(g, &d.mp))
            return fail(MR_E_PARAM, "frame %d: not on the compact frame path (coarsest level <= 4, width "
                                    "divisible by 128, blur radii <= 8)", k);
    }
    return MR_OK;
}

// cached: the frames' mask pyramids live elsewhere (resident), the
// workspace holds only their per-frame scratch
BatchLayout batch_layout(const mr_frame_desc* fr, int n, const Geo* geos, bool cached = false) {
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t nb) {
        size_t o = off;
        off += align256(nb);
        return o;
    };
    L.te = take(sizeof(EdgeArgs) * n);
    L.tl = take(sizeof(LeanArgs) * n);
    L.tv = take((fr[0].effect == MR_EFFECT_SSAO ? sizeof(SsaoArgs) : sizeof(SsgiArgs)) * n);
    L.tm = take(sizeof(LeanMergeArgs) * n);
    L.bases = take(sizeof(unsigned) * (kBatchTables * (MR_MAX_BATCH + 1) + kBatchCounters + kFusedCounters));
    for (int k = 0; k < n; ++k) {
        const LeanLayout f = lean_layout(geos[k], fr[k].effect);
        L.frames[k] = take(cached ? f.scratch : f.bytes);
    }
    L.bytes = off;
    return L;
}

int load_plan(const void* plan, BatchPlan& P) {
    if (!plan) return fail(MR_E_NULL, "plan is NULL");
    memcpy(&P, plan, sizeof(P));
    if (P.magic != kBatchMagic || P.n < 1 || P.n > MR_MAX_BATCH)
        return fail(MR_E_PARAM, "plan was not filled by mr_batch_setup");
    return MR_OK;
}

int check_config(const BatchPlan& P, const mr_batch_config& c) {
    if (c.edge_tile != 0 && c.edge_tile != 1) return fail(MR_E_PARAM, "edge_tile %d not 0 or 1", c.edge_tile);
    if (c.eval_queue != 0 && c.eval_queue != 1) return fail(MR_E_PARAM, "eval_queue %d not 0 or 1", c.eval_queue);
    if (c.eval_blocks_per_cu < 0 || c.eval_blocks_per_cu > 64)
        return fail(MR_E_PARAM, "eval_blocks_per_cu %d outside [0, 64]", c.eval_blocks_per_cu);
    if (c.merge_generic != 0 && c.merge_generic != 1)
        return fail(MR_E_PARAM, "merge_generic %d not 0 or 1", c.merge_generic);
    if (c.persistent != 0 && c.persistent != 1) return fail(MR_E_PARAM, "persistent %d not 0 or 1", c.persistent);
    if (P.cached && (c.persistent || c.eval_queue))
        return fail(MR_E_PARAM, "a batch on resident mask pyramids runs staged with fixed evaluation strides "
                                "(persistent = 0, eval_queue = 0)");
    if (c.persistent && !fused_ok(P))
        return fail(MR_E_PARAM, "the persistent launch needs frames of at most 4 levels and at most %d samples",
                    kFusedSamples);
    if (c.eval_items != 0 && c.eval_items != 1 && c.eval_items != 2 && c.eval_items != 4)
        return fail(MR_E_PARAM, "eval_items %d not 0, 1, 2 or 4", c.eval_items);
    if (c.worker_pixels != 0 && (c.worker_pixels < 4096 || c.worker_pixels > (1 << 24)))
        return fail(MR_E_PARAM, "worker_pixels %d not 0 or in [4096, 2^24]", c.worker_pixels);
    if (c.tiles_per_ticket < 0 || c.tiles_per_ticket > 64)
        return fail(MR_E_PARAM, "tiles_per_ticket %d outside [0, 64]", c.tiles_per_ticket);
    if (c.eval_halo != 0) {
        if (c.eval_halo != 8 && c.eval_halo != 16 && c.eval_halo != 24)
            return fail(MR_E_PARAM, "eval_halo %d is not 0, 8, 16 or 24", c.eval_halo);
        if (P.effect != MR_EFFECT_SSAO || P.cached || c.persistent || c.eval_queue || P.S > kTiledSamplesHost)
            return fail(MR_E_PARAM, "eval_halo applies to SSAO batches that build their masks, with staged "
                                    "launches, eval_queue = 0 and at most %d samples", kTiledSamplesHost);
    }
    return MR_OK;
}

int run_fused(const BatchPlan& P, hipStream_t s) {
    const mr_batch_config& c = P.cfg;
    FusedArgs a{};
    a.te = P.te;
    a.tl = P.tl;
    a.tv = P.tv;
    a.tm = P.tm;
    a.base[0] = P.edge_base[0];  // 256 x 8 tiles (fused_ok)
    a.base[1] = P.rank_base;
    a.base[2] = P.rank_base;
    a.base[3] = nullptr;  // evaluation workers: from px in the kernel
    a.base[4] = P.merge_base;
    a.px = P.px;
    a.edge_tx = P.edge_tx[0];
    a.merge_tx = P.merge_tx;
    a.worker_px = (unsigned)(c.worker_pixels ? c.worker_pixels : kDefaultWorkerPixels);
    a.group = c.tiles_per_ticket ? c.tiles_per_ticket : kDefaultTilesPerTicket;
    a.ctr = P.fused_ctr;
    a.n = P.n;
    a.wide = 1;
    a.m4 = P.m4_ok && !c.merge_generic;
    a.items = c.eval_items ? c.eval_items : 1;
    a.spin_limit = kFusedSpinLimit;
    if (launch_batch_fused(a, P.effect, P.S, P.ndt, P.cdt, nullptr, s) != hipSuccess)
        return fail(MR_E_DEVICE, "persistent batch kernel launch failed");
    return MR_OK;
}

int run_plan(const BatchPlan& P, hipStream_t s) {
    const mr_batch_config& c = P.cfg;
    if (c.persistent) return run_fused(P, s);
    const int et = c.edge_tile;
    const bool wide = et == 0 && P.wide_ok;
    if (!P.cached) {
        if (launch_edges_batch(P.te, P.edge_base[et], P.edge_tx[et], P.n, P.edge_total[et], P.ndt, false, wide,
                               P.queue, s) != hipSuccess)
            return fail(MR_E_DEVICE, "batched edge kernel launch failed");
        if (launch_lean_masks_batch(P.tl, P.rank_base, P.n, P.rank_total, s) != hipSuccess)
            return fail(MR_E_DEVICE, "batched rank kernel launch failed");
    }
    const BatchSchedule bs{c.eval_queue != 0, c.eval_blocks_per_cu, P.queue};
    hipError_t e;
    if (P.effect == MR_EFFECT_SSAO && c.eval_halo)
        e = launch_ssao_batch_tiled(static_cast<const SsaoArgs*>(P.tv), P.n, P.S, P.ndt, c.eval_halo, P.eval_hint,
                                    s);
    else if (P.effect == MR_EFFECT_SSAO)
        e = launch_ssao_batch(static_cast<const SsaoArgs*>(P.tv), P.n, P.S, P.ndt, P.eval_hint, bs, s);
    else
        e = launch_ssgi_batch(static_cast<const SsgiArgs*>(P.tv), P.n, P.S, P.ndt, P.cdt, P.eval_hint, bs, s);
    if (e != hipSuccess) return fail(MR_E_DEVICE, "batched evaluation kernel launch failed");
    if (launch_lean_merge_batch(P.tm, P.merge_base, P.merge_tx, P.n, P.merge_total, P.C, P.c16,
                                c.merge_generic ? kMergeGeneral : P.merge_geo, s) != hipSuccess)
        return fail(MR_E_DEVICE, "batched merge kernel launch failed");
    return MR_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t mr_workspace_bytes(const mr_camera* cam, const mr_mask_params* mp, int purpose) {
    if (!mp) {
        fail(MR_E_NULL, "mask params are NULL");
        return 0;
    }
    Geo g;
    if (check_geo(cam, mp, g) || check_mask_params(mp, g)) return 0;
    if (purpose == MR_WS_MASKS) return mask_scratch(g).bytes;
    if (purpose != MR_EFFECT_SSAO && purpose != MR_EFFECT_SHADOW && purpose != MR_EFFECT_SSGI) {
        fail(MR_E_PARAM, "unknown workspace purpose %d", purpose);
        return 0;
    }
    const size_t dense = frame_layout(g, purpose).bytes, lean = lean_layout(g, purpose).bytes;
    return dense > lean ? dense : lean;
}

int mr_build_masks(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp, const uint8_t* hard,
                   const mr_masks* m, void* ws, size_t ws_bytes, void* stream) {
    if (!mp) return fail(MR_E_NULL, "mask params are NULL");
    Geo g;
    int st = check_geo(cam, mp, g);
    if (!st) st = check_mask_params(mp, g);
    if (!st) st = check_gbuffer(gb, true, false);
    if (!st) st = check_masks(m, g, true, true);
    if (st) return st;
    if (!m->edge) return fail(MR_E_NULL, "masks.edge is NULL");
    if (misaligned(m->edge) || (m->level_map && misaligned(m->level_map)) || (hard && misaligned(hard)))
        return fail(MR_E_PARAM, "edge, level_map and hard_shadow must be 16-byte aligned");
    const size_t need = mask_scratch(g).bytes;
    if (!ws || ws_bytes < need) return fail(MR_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (misaligned(ws)) return fail(MR_E_PARAM, "workspace is not 16-byte aligned");
    return do_build_masks(gb, g, mp, hard, m, ws, static_cast<hipStream_t>(stream));
}

static int eval_entry(int effect, const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp,
                      const mr_masks* m, const void* params, float* const out[kMaxLevels], void* stream) {
    Geo g;
    int st;
    if (m) {
        if (!mp) return fail(MR_E_NULL, "mask params are NULL (required with masks)");
        st = check_geo(cam, mp, g);
        if (!st) st = check_mask_params(mp, g);
    } else {
        st = check_geo(cam, nullptr, g);
    }
    if (!st) st = check_gbuffer(gb, effect != MR_EFFECT_SHADOW, effect == MR_EFFECT_SSGI);
    if (!st && m) st = check_masks(m, g, false, true);
    if (!st) st = check_outputs(out, g, !m);
    if (!st)
        st = check_effect_params(effect, static_cast<const mr_ssao_params*>(effect == MR_EFFECT_SSAO ? params : nullptr),
                                 static_cast<const mr_shadow_params*>(effect == MR_EFFECT_SHADOW ? params : nullptr),
                                 static_cast<const mr_ssgi_params*>(effect == MR_EFFECT_SSGI ? params : nullptr));
    if (st) return st;
    return do_eval(effect, gb, cam, g, m, params, out, static_cast<hipStream_t>(stream));
}

int mr_eval_ssao(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp, const mr_masks* m,
                 const mr_ssao_params* p, float* const out[MR_MAX_LEVELS], void* stream) {
    return eval_entry(MR_EFFECT_SSAO, gb, cam, mp, m, p, out, stream);
}

int mr_eval_shadow(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp, const mr_masks* m,
                   const mr_shadow_params* p, float* const out[MR_MAX_LEVELS], void* stream) {
    return eval_entry(MR_EFFECT_SHADOW, gb, cam, mp, m, p, out, stream);
}

int mr_eval_ssgi(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp, const mr_masks* m,
                 const mr_ssgi_params* p, float* const out[MR_MAX_LEVELS], void* stream) {
    return eval_entry(MR_EFFECT_SSGI, gb, cam, mp, m, p, out, stream);
}

int mr_shadow_hard(const mr_gbuffer* gb, const mr_camera* cam, const mr_shadow_params* p, uint8_t* hard,
                   void* stream) {
    Geo g;
    int st = check_geo(cam, nullptr, g);
    if (!st) st = check_gbuffer(gb, false, false);
    if (!st) st = check_shadow(p);
    if (st) return st;
    if (!hard) return fail(MR_E_NULL, "hard is NULL");
    if (misaligned(hard)) return fail(MR_E_PARAM, "hard is not 16-byte aligned");
    HardArgs a{};
    a.depth = gb->depth;
    a.W = g.W;
    a.H = g.H;
    a.f = cam->focal_px;
    a.sm = p->shadow_map;
    a.size = p->sm_size;
    memcpy(a.M, p->view_to_light, sizeof(a.M));
    a.fL = p->light_focal_px;
    a.bias = p->bias;
    a.hard = hard;
    if (launch_hard(a, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(MR_E_DEVICE, "hard shadow kernel launch failed");
    return MR_OK;
}

int mr_upsample_merge(const mr_camera* cam, const mr_mask_params* mp, const mr_masks* m,
                      const float* const level_out[MR_MAX_LEVELS], int channels, float* out, void* stream) {
    if (!mp) return fail(MR_E_NULL, "mask params are NULL");
    Geo g;
    int st = check_geo(cam, mp, g);
    if (!st) st = check_mask_params(mp, g);
    if (!st) st = check_masks(m, g, true, false);
    if (st) return st;
    if (channels != 1 && channels != 3) return fail(MR_E_PARAM, "channels %d not 1 or 3", channels);
    if (!level_out) return fail(MR_E_NULL, "level_out is NULL");
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (!level_out[i - 1]) return fail(MR_E_NULL, "level_out[%d] is NULL", i - 1);
        if (misaligned(level_out[i - 1])) return fail(MR_E_PARAM, "level_out[%d] misaligned", i - 1);
    }
    if (!out) return fail(MR_E_NULL, "out is NULL");
    if (misaligned(out)) return fail(MR_E_PARAM, "out is not 16-byte aligned");
    return do_merge(g, mp, m, level_out, channels, out, static_cast<hipStream_t>(stream));
}

int mr_eval_ssao_fullres(const mr_gbuffer* gb, const mr_camera* cam, const mr_mask_params* mp, const mr_masks* m,
                         const mr_ssao_params* const level_params[MR_MAX_LEVELS], float* out, void* stream) {
    if (!mp) return fail(MR_E_NULL, "mask params are NULL");
    if (!level_params) return fail(MR_E_NULL, "level_params is NULL");
    Geo g;
    int st = check_geo(cam, mp, g);
    if (!st) st = check_mask_params(mp, g);
    if (!st) st = check_gbuffer(gb, true, false);
    if (!st) st = check_masks(m, g, true, false);
    if (st) return st;
    if (!out) return fail(MR_E_NULL, "out is NULL");
    if (misaligned(out)) return fail(MR_E_PARAM, "out is not 16-byte aligned");
    FullresArgs A{};
    int koff = 0;
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        const mr_ssao_params* p = level_params[i - 1];
        if (!p) return fail(MR_E_NULL, "level_params[%d] is NULL (level %d is enabled)", i - 1, i);
        if ((st = check_effect_params(MR_EFFECT_SSAO, p, nullptr, nullptr))) return st;
        FullresLevel& V = A.lv[j];
        if (i != g.L) {
            V.a = m->alpha[i - 1];
            V.S = m->stencil[i - 1];
        }
        V.W = g.Wi[i - 1];
        V.H = g.Hi[i - 1];
        V.sh = i - 1;
        V.w = mp->weight[i - 1];
        V.p = SsaoSampling{p->kernel, p->samples, p->radius, p->bias_rel};
        V.koff = koff;
        koff += p->samples;
    }
    if (koff > kFullresMaxSamples)
        return fail(MR_E_PARAM, "%d samples over the levels > %d", koff, kFullresMaxSamples);
    A.nlev = g.nlev;
    // full-resolution geometry of the naive pass
    Geo gp;
    if ((st = check_geo(cam, nullptr, gp))) return st;
    EvalPlan E;
    float* o[kMaxLevels] = {out};
    build_eval(MR_EFFECT_SSAO, gb, cam, gp, nullptr, level_params[g.levels[0] - 1], o, false, nullptr, false, E);
    A.L = E.sa.c.lv[0];
    A.normal = E.sa.c.normal;
    A.plane = E.sa.c.plane;
    A.out = out;
    A.W = g.W;
    A.H = g.H;
    if (launch_ssao_fullres(A, gb->normal_dtype, static_cast<hipStream_t>(stream)) != hipSuccess)
        return fail(MR_E_DEVICE, "full-resolution level kernel launch failed");
    return MR_OK;
}

// The whole frame; `path_only`: the workspace need only hold the layout of
// the path these parameters take (the static-scratch entry point), else
// that of either path (what mr_workspace_bytes reports).  `check_only`:
// validate the arguments and return before anything is enqueued.
static int frame_run(const mr_frame_desc* d, void* ws, size_t ws_bytes, hipStream_t s, bool path_only,
                     bool check_only = false) {
    if (!d) return fail(MR_E_NULL, "frame descriptor is NULL");
    const int effect = d->effect;
    int st = check_effect_params(effect, d->ssao, d->shadow, d->ssgi);
    if (st) return st;
    const void* params = effect == MR_EFFECT_SSAO ? (const void*)d->ssao
                         : effect == MR_EFFECT_SHADOW ? (const void*)d->shadow : (const void*)d->ssgi;
    if (!d->out) return fail(MR_E_NULL, "out is NULL");
    if (misaligned(d->out)) return fail(MR_E_PARAM, "out is not 16-byte aligned");
    const int C = effect == MR_EFFECT_SSGI ? 3 : 1;
    if (d->level_dtype != MR_F32 && d->level_dtype != MR_F16)
        return fail(MR_E_DTYPE, "level_dtype %d is neither MR_F32 nor MR_F16", d->level_dtype);
    if ((st = check_halo(d))) return st;
    if (!d->multires) {
        if (d->bilateral.levels) return fail(MR_E_PARAM, "the bilateral blur needs multires = 1");
        Geo g;
        st = check_geo(&d->cam, nullptr, g);
        if (!st) st = check_gbuffer(&d->g, effect != MR_EFFECT_SHADOW, effect == MR_EFFECT_SSGI);
        if (st) return st;
        if (check_only) return MR_OK;
        float* out[kMaxLevels] = {d->out};
        if ((st = mark(d, 0, s)) || (st = mark(d, 4, s)) || (st = mark(d, 1, s))) return st;
        if ((st = do_eval(effect, &d->g, &d->cam, g, nullptr, params, out, s))) return st;
        if ((st = mark(d, 2, s))) return st;
        return mark(d, 3, s);
    }
    Geo g;
    st = check_geo(&d->cam, &d->mp, g);
    if (!st) st = check_mask_params(&d->mp, g);
    if (!st) st = check_gbuffer(&d->g, true, effect == MR_EFFECT_SSGI);
    if (st) return st;
    if (d->level_map && misaligned(d->level_map)) return fail(MR_E_PARAM, "level_map is not 16-byte aligned");
    if ((st = check_bilateral(d, g))) return st;
    const FrameLayout f = frame_layout(g, effect);
    const size_t lean_bytes = lean_layout(g, effect).bytes;
    const bool lean = lean_ok(g, &d->mp);
    if (d->eval_halo && !lean)
        return fail(MR_E_PARAM, "eval_halo needs the compact frame path (coarsest level <= 4, width divisible by 128, "
                                "blur radii <= 8)");
    const size_t need = path_only ? (lean ? lean_bytes : f.bytes) : (f.bytes > lean_bytes ? f.bytes : lean_bytes);
    if (!ws || ws_bytes < need) return fail(MR_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
    if (misaligned(ws)) return fail(MR_E_PARAM, "workspace is not 16-byte aligned");
    if (!lean && d->level_dtype == MR_F16)
        return fail(MR_E_DTYPE, "f16 sub-image storage needs the compact frame path (coarsest level <= 4, width "
                                "divisible by 128, blur radii <= 8 with positive taps)");
    if (check_only) return MR_OK;
    if (lean) {
        uint8_t* b = static_cast<uint8_t*>(ws);
        return do_frame_lean(d, g, params, b, b + lean_layout(g, effect).pyramid, true, s);
    }
    uint8_t* b = static_cast<uint8_t*>(ws);
    mr_masks m{};
    m.edge = b + f.edge;
    m.level_map = d->level_map;
    m.count = reinterpret_cast<uint32_t*>(b + f.count);
    float* lo[kMaxLevels] = {};
    for (int j = 0; j < g.nlev; ++j) {
        const int i = g.levels[j];
        if (i != g.L) {
            m.alpha[i - 1] = reinterpret_cast<float*>(b + f.alpha[i - 1]);
            m.stencil[i - 1] = b + f.stencil[i - 1];
            m.worklist[i - 1] = reinterpret_cast<uint32_t*>(b + f.worklist[i - 1]);
        }
        if (i >= 2) m.level_depth[i - 1] = reinterpret_cast<float*>(b + f.level_depth[i - 1]);
        lo[i - 1] = reinterpret_cast<float*>(b + f.level_out[i - 1]);
    }
    if ((st = mark(d, 0, s))) return st;
    const uint8_t* hard = nullptr;
    if (effect == MR_EFFECT_SHADOW) {
        HardArgs a{};
        a.depth = d->g.depth;
        a.W = g.W;
        a.H = g.H;
        a.f = d->cam.focal_px;
        a.sm = d->shadow->shadow_map;
        a.size = d->shadow->sm_size;
        memcpy(a.M, d->shadow->view_to_light, sizeof(a.M));
        a.fL = d->shadow->light_focal_px;
        a.bias = d->shadow->bias;
        a.hard = b + f.hard;
        if (launch_hard(a, s) != hipSuccess) return fail(MR_E_DEVICE, "hard shadow kernel launch failed");
        hard = b + f.hard;
    }
    st = do_build_masks(&d->g, g, &d->mp, hard, &m, b + f.scratch, s);
    if (st) return st;
    if ((st = mark(d, 4, s)) || (st = mark(d, 1, s))) return st;
    st = do_eval(effect, &d->g, &d->cam, g, &m, params, lo, s);
    if (st) return st;
    if ((st = mark(d, 2, s))) return st;
    const float* clo[kMaxLevels];
    for (int k = 0; k < kMaxLevels; ++k) clo[k] = lo[k];
    if ((st = do_merge(g, &d->mp, &m, clo, C, d->out, s))) return st;
    return mark(d, 3, s);
}

int mr_frame(const mr_frame_desc* d, void* ws, size_t ws_bytes, void* stream) {
    return frame_run(d, ws, ws_bytes, static_cast<hipStream_t>(stream), false);
}

int mr_frame_tune(mr_frame_desc* d, void* ws, size_t ws_bytes, int reps, float* ms, void* stream) {
    if (!d) return fail(MR_E_NULL, "frame descriptor is NULL");
    if (reps < 1 || reps > 1000) return fail(MR_E_PARAM, "reps %d outside [1, 1000]", reps);
    static const int kHalos[kFrameHalos] = {0, 8, 16, 24};
    // the descriptor as given must be valid; candidates it rejects are skipped
    mr_frame_desc c = *d;
    for (int k = 0; k < MR_FRAME_EVENTS; ++k) c.stage_events[k] = nullptr;  // the caller's events stay untouched
    hipStream_t s = static_cast<hipStream_t>(stream);
    int st = frame_run(&c, ws, ws_bytes, s, false, true);
    if (st) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(MR_E_DEVICE, "event creation failed");
    }
    int best = d->eval_halo;
    float best_ms = std::numeric_limits<float>::infinity();
    for (int k = 0; k < kFrameHalos && !st; ++k) {
        if (ms) ms[k] = -1.0f;
        c.eval_halo = kHalos[k];
        if (check_halo(&c) != MR_OK) continue;  // not a choice for this frame
        st = frame_run(&c, ws, ws_bytes, s, false);  // warm-up
        if (!st && hipEventRecord(e0, s) != hipSuccess) st = fail(MR_E_DEVICE, "event record failed");
        for (int i = 0; i < reps && !st; ++i) st = frame_run(&c, ws, ws_bytes, s, false);
        float t = 0.0f;
        if (!st && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess))
            st = fail(MR_E_DEVICE, "frame timing failed");
        if (st) break;
        t /= (float)reps;
        if (ms) ms[k] = t;
        if (t < best_ms) {
            best_ms = t;
            best = kHalos[k];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    d->eval_halo = best;
    return MR_OK;
}

int mr_pyramid_bytes(const mr_camera* cam, const mr_mask_params* mp, int effect, size_t* pyramid, size_t* scratch) {
    if (!cam || !mp || !pyramid || !scratch) return fail(MR_E_NULL, "an argument is NULL");
    if (effect != MR_EFFECT_SSAO && effect != MR_EFFECT_SHADOW && effect != MR_EFFECT_SSGI)
        return fail(MR_E_PARAM, "unknown effect %d", effect);
    Geo g;
    int st = check_geo(cam, mp, g);
    if (!st) st = check_mask_params(mp, g);
    if (st) return st;
    if (!lean_ok(g, mp))
        return fail(MR_E_PARAM, "the compact frame path does not apply (coarsest level <= 4, width divisible by 128, "
                                "blur radii <= 8)");
    const LeanLayout f = lean_layout(g, effect);
    *pyramid = f.pyramid;
    *scratch = f.scratch;
    return MR_OK;
}

int mr_frame_cached(const mr_frame_desc* d, void* pyramid, size_t pyramid_bytes, int build, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!d) return fail(MR_E_NULL, "frame descriptor is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int effect = d->effect;
    int st = check_effect_params(effect, d->ssao, d->shadow, d->ssgi);
    if (st) return st;
    const void* params = effect == MR_EFFECT_SSAO ? (const void*)d->ssao
                         : effect == MR_EFFECT_SHADOW ? (const void*)d->shadow : (const void*)d->ssgi;
    if (!d->multires) return fail(MR_E_PARAM, "a cached mask pyramid needs multires = 1");
    if (build != 0 && build != 1) return fail(MR_E_PARAM, "build %d is neither 0 nor 1", build);
    if (!d->out) return fail(MR_E_NULL, "out is NULL");
    if (misaligned(d->out)) return fail(MR_E_PARAM, "out is not 16-byte aligned");
    if (d->level_dtype != MR_F32 && d->level_dtype != MR_F16)
        return fail(MR_E_DTYPE, "level_dtype %d is neither MR_F32 nor MR_F16", d->level_dtype);
    Geo g;
    st = check_geo(&d->cam, &d->mp, g);
    if (!st) st = check_mask_params(&d->mp, g);
    if (!st) st = check_gbuffer(&d->g, true, effect == MR_EFFECT_SSGI);
    if (st) return st;
    if (d->level_map && misaligned(d->level_map)) return fail(MR_E_PARAM, "level_map is not 16-byte aligned");
    if ((st = check_bilateral(d, g)) || (st = check_halo(d))) return st;
    if (!lean_ok(g, &d->mp))
        return fail(MR_E_PARAM, "the compact frame path does not apply (coarsest level <= 4, width divisible by 128, "
                                "blur radii <= 8)");
    const LeanLayout f = lean_layout(g, effect);
    if (!pyramid || pyramid_bytes < f.pyramid)
        return fail(MR_E_WORKSPACE, "pyramid %zu bytes < %zu needed", pyramid_bytes, f.pyramid);
    if (!ws || ws_bytes < f.scratch) return fail(MR_E_WORKSPACE, "scratch %zu bytes < %zu needed", ws_bytes, f.scratch);
    if (misaligned(pyramid) || misaligned(ws)) return fail(MR_E_PARAM, "pyramid or scratch is not 16-byte aligned");
    return do_frame_lean(d, g, params, static_cast<uint8_t*>(pyramid), static_cast<uint8_t*>(ws), build != 0, s);
}

// ---------------------------------------------------------------------------
// mr_frame_static: mr_frame with its workspace in a file-scope device array,
// for callers that cannot allocate.  The array's name is only a host-side
// handle; its device address is looked up once per device (with that device
// current) and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[MR_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices] = {};

// device address of `scratch` on the device of `s` (which must be current)
int static_scratch(hipStream_t s, void** out) {
    int cur = -1, dev = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess) e = s ? hipStreamGetDevice(s, &dev) : hipSuccess;
    if (e != hipSuccess) return fail(MR_E_DEVICE, "device query failed: %s", hipGetErrorString(e));
    if (!s) dev = cur;
    if (dev != cur) return fail(MR_E_PARAM, "the stream belongs to device %d but device %d is current", dev, cur);
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(MR_E_DEVICE, "device %d beyond the %d devices with static scratch", dev, kMaxScratchDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MR_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MR_OK;
}
}  // namespace

int mr_frame_static(const mr_frame_desc* d, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!d) return fail(MR_E_NULL, "frame descriptor is NULL");
    // the size check first, so that an oversized frame is rejected with its
    // own message before any device query
    if (d->multires) {
        Geo g;
        int st = check_geo(&d->cam, &d->mp, g);
        if (!st) st = check_mask_params(&d->mp, g);
        if (st) return st;
        const size_t need = lean_ok(g, &d->mp) ? lean_layout(g, d->effect).bytes : frame_layout(g, d->effect).bytes;
        if (need > MR_STATIC_SCRATCH_BYTES)
            return fail(MR_E_WORKSPACE, "frame needs %zu bytes of scratch, more than the %u of MR_STATIC_SCRATCH_BYTES",
                        need, (unsigned)MR_STATIC_SCRATCH_BYTES);
    }
    void* ws = nullptr;
    const int st = static_scratch(s, &ws);
    if (st) return st;
    return frame_run(d, ws, MR_STATIC_SCRATCH_BYTES, s, true);
}

int mr_frame_workspace_layout(const mr_camera* cam, const mr_mask_params* mp, int effect, mr_frame_layout* out) {
    if (!cam || !mp || !out) return fail(MR_E_NULL, "camera, mask parameters or output is NULL");
    if (effect != MR_EFFECT_SSAO && effect != MR_EFFECT_SHADOW && effect != MR_EFFECT_SSGI)
        return fail(MR_E_PARAM, "unknown effect %d", effect);
    Geo g;
    int st = check_geo(cam, mp, g);
    if (!st) st = check_mask_params(mp, g);
    if (st) return st;
    *out = mr_frame_layout{};
    if (!lean_ok(g, mp)) return MR_OK;
    const LeanLayout f = lean_layout(g, effect);
    out->compact = 1;
    out->tile_words = kLeanTileWords;
    out->tile_rows = kLeanTileRows;
    out->count = f.count;
    for (int j = 0; j + 1 < g.nlev; ++j) {
        const int i = g.levels[j];
        out->worklist[i - 1] = f.list[i - 1];
        out->stencil_bits[i - 1] = f.Sb[i - 1];
        out->rank[i - 1] = f.woff[i - 1];
    }
    return MR_OK;
}

size_t mr_batch_workspace_bytes(const mr_frame_desc* frames, int n) {
    Geo geos[MR_MAX_BATCH];
    if (check_batch(frames, n, geos)) return 0;
    return batch_layout(frames, n, geos).bytes;
}

size_t mr_batch_staging_bytes(const mr_frame_desc* frames, int n) {
    Geo geos[MR_MAX_BATCH];
    if (check_batch(frames, n, geos)) return 0;
    return batch_layout(frames, n, geos).frames[0];
}

}  // extern "C"

namespace {
// mr_batch_setup and mr_batch_setup_async: the tables are built in `stage`
// (host memory of BL.frames[0] bytes) and copied to the start of ws on the
// stream; wait: the call returns after the copy (stage may be freed then)
int batch_setup(const mr_frame_desc* frames, void* const* pyramids, int n, void* ws, size_t ws_bytes, void* plan,
                size_t plan_bytes, uint8_t* stage, size_t stage_bytes, bool wait, hipStream_t s) {
    Geo geos[MR_MAX_BATCH];
    int st = check_batch(frames, n, geos);
    if (st) return st;
    if (!plan) return fail(MR_E_NULL, "plan is NULL");
    if (plan_bytes < MR_BATCH_PLAN_BYTES) return fail(MR_E_PARAM, "plan needs %d bytes", MR_BATCH_PLAN_BYTES);
    const bool cached = pyramids != nullptr;
    for (int k = 0; cached && k < n; ++k) {
        if (!pyramids[k]) return fail(MR_E_NULL, "frame %d: pyramid is NULL", k);
        if (misaligned(pyramids[k])) return fail(MR_E_PARAM, "frame %d: pyramid is not 16-byte aligned", k);
    }
    const BatchLayout BL = batch_layout(frames, n, geos, cached);
    if (!ws || ws_bytes < BL.bytes) return fail(MR_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, BL.bytes);
    if (misaligned(ws)) return fail(MR_E_PARAM, "workspace is not 16-byte aligned");
    if (!stage) return fail(MR_E_NULL, "staging is NULL");
    if (stage_bytes < BL.frames[0])
        return fail(MR_E_WORKSPACE, "staging %zu bytes < %zu needed", stage_bytes, BL.frames[0]);
    uint8_t* b = static_cast<uint8_t*>(ws);
    const int effect = frames[0].effect;
    // the tables region on the host, then one copy to the device
    uint8_t* const host = stage;
    memset(host, 0, BL.frames[0]);
    EdgeArgs* te = reinterpret_cast<EdgeArgs*>(host + BL.te);
    LeanArgs* tl = reinterpret_cast<LeanArgs*>(host + BL.tl);
    SsaoArgs* tsa = reinterpret_cast<SsaoArgs*>(host + BL.tv);
    SsgiArgs* tgi = reinterpret_cast<SsgiArgs*>(host + BL.tv);
    LeanMergeArgs* tm = reinterpret_cast<LeanMergeArgs*>(host + BL.tm);
    unsigned* bases = reinterpret_cast<unsigned*>(host + BL.bases);
    auto table = [&](int t) { return bases + t * (MR_MAX_BATCH + 1); };
    unsigned* edge_base[2] = {table(0), table(1)};
    unsigned* edge_tx[2] = {table(2), table(3)};
    unsigned* rank_base = table(4);
    unsigned* merge_base = table(5);
    unsigned* merge_tx = table(6);
    unsigned* px = table(7);  // the counters follow, zero
    BatchPlan P{};
    P.magic = kBatchMagic;
    P.cached = cached;
    P.n = n;
    P.effect = effect;
    P.ndt = frames[0].g.normal_dtype;
    P.cdt = frames[0].g.color_dtype;
    P.C = effect == MR_EFFECT_SSGI ? 3 : 1;
    P.c16 = frames[0].level_dtype == MR_F16;
    unsigned et[2] = {0, 0}, rt = 0, mt = 0, hint = 0;
    bool wide = false;
    for (int k = 0; k < n; ++k) {
        const mr_frame_desc& d = frames[k];
        const void* params = effect == MR_EFFECT_SSAO ? (const void*)d.ssao : (const void*)d.ssgi;
        LeanPlan L;
        uint8_t* const fb = b + BL.frames[k];
        if (cached)
            build_lean(&d, geos[k], params, static_cast<uint8_t*>(pyramids[k]), fb, L);
        else
            build_lean(&d, geos[k], params, fb, fb + lean_layout(geos[k], effect).pyramid, L);
        te[k] = L.ea;
        tl[k] = L.la;
        if (effect == MR_EFFECT_SSAO)
            tsa[k] = L.ev.sa;
        else
            tgi[k] = L.ev.gi;
        tm[k] = L.ma;
        // both tile shapes: table 0 the default one (wide with at most 4
        // levels: the same for all frames), table 1 the narrow one
        unsigned tx, nt;
        edges_grid(geos[k].W, geos[k].H, geos[k].N, wide, tx, nt);
        edge_base[0][k] = et[0];
        edge_tx[0][k] = tx;
        et[0] += nt;
        edges_tiles(geos[k].W, geos[k].H, false, tx, nt);
        edge_base[1][k] = et[1];
        edge_tx[1][k] = tx;
        et[1] += nt;
        rank_base[k] = rt;
        rt += L.la.nblk;
        const unsigned mx = (unsigned)((geos[k].W + kMergeTW - 1) / kMergeTW);
        merge_base[k] = mt;
        merge_tx[k] = mx;
        mt += mx * (unsigned)((geos[k].H + kMergeTH - 1) / kMergeTH);
        px[k] = (unsigned)geos[k].W * (unsigned)geos[k].H;
        hint += L.ev.hint + 1024u;  // + padding of the levels' and frame's item ranges
        if (k == 0) {
            P.m4_ok = merge4_applies(L.ma);
            P.merge_geo = merge_geometry(L.ma);
            P.S = effect == MR_EFFECT_SSAO ? L.ev.sa.S : L.ev.gi.S;
        }
    }
    edge_base[0][n] = et[0];
    edge_base[1][n] = et[1];
    rank_base[n] = rt;
    merge_base[n] = mt;
    P.edge_total[0] = et[0];
    P.edge_total[1] = et[1];
    P.rank_total = rt;
    P.merge_total = mt;
    P.eval_hint = hint;
    P.wide_ok = wide;
    P.cfg = mr_batch_config{};
    P.te = reinterpret_cast<const EdgeArgs*>(b + BL.te);
    P.tl = reinterpret_cast<const LeanArgs*>(b + BL.tl);
    P.tv = b + BL.tv;
    P.tm = reinterpret_cast<const LeanMergeArgs*>(b + BL.tm);
    unsigned* db = reinterpret_cast<unsigned*>(b + BL.bases);
    auto dtable = [&](int t) { return db + t * (MR_MAX_BATCH + 1); };
    P.edge_base[0] = dtable(0);
    P.edge_base[1] = dtable(1);
    P.edge_tx[0] = dtable(2);
    P.edge_tx[1] = dtable(3);
    P.rank_base = dtable(4);
    P.merge_base = dtable(5);
    P.merge_tx = dtable(6);
    P.px = dtable(7);
    P.queue = dtable(kBatchTables);
    P.fused_ctr = P.queue + kBatchCounters;
    hipError_t e = hipMemcpyAsync(b, host, BL.frames[0], hipMemcpyHostToDevice, s);
    if (e == hipSuccess && wait) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MR_E_DEVICE, "batch table copy failed: %s", hipGetErrorString(e));
    memcpy(plan, &P, sizeof(P));
    return MR_OK;
}
}  // namespace

extern "C" {

int mr_batch_setup(const mr_frame_desc* frames, int n, void* ws, size_t ws_bytes, void* plan, size_t plan_bytes,
                   void* stream) {
    Geo geos[MR_MAX_BATCH];
    const int st = check_batch(frames, n, geos);
    if (st) return st;
    std::vector<uint8_t> host(batch_layout(frames, n, geos).frames[0]);
    return batch_setup(frames, nullptr, n, ws, ws_bytes, plan, plan_bytes, host.data(), host.size(), true,
                       static_cast<hipStream_t>(stream));
}

int mr_batch_setup_async(const mr_frame_desc* frames, int n, void* ws, size_t ws_bytes, void* plan,
                         size_t plan_bytes, void* staging, size_t staging_bytes, void* stream) {
    return batch_setup(frames, nullptr, n, ws, ws_bytes, plan, plan_bytes, static_cast<uint8_t*>(staging),
                       staging_bytes, false, static_cast<hipStream_t>(stream));
}

size_t mr_batch_cached_workspace_bytes(const mr_frame_desc* frames, int n) {
    Geo geos[MR_MAX_BATCH];
    if (check_batch(frames, n, geos)) return 0;
    return batch_layout(frames, n, geos, true).bytes;
}

int mr_batch_setup_cached(const mr_frame_desc* frames, void* const* pyramids, int n, void* ws, size_t ws_bytes,
                          void* plan, size_t plan_bytes, void* staging, size_t staging_bytes, void* stream) {
    if (!pyramids) return fail(MR_E_NULL, "pyramids are NULL");
    return batch_setup(frames, pyramids, n, ws, ws_bytes, plan, plan_bytes, static_cast<uint8_t*>(staging),
                       staging_bytes, false, static_cast<hipStream_t>(stream));
}

int mr_batch_run(const void* plan, void* stream) {
    BatchPlan P;
    const int st = load_plan(plan, P);
    return st ? st : run_plan(P, static_cast<hipStream_t>(stream));
}

int mr_batch_get_config(const void* plan, mr_batch_config* cfg) {
    if (!cfg) return fail(MR_E_NULL, "config is NULL");
    BatchPlan P;
    const int st = load_plan(plan, P);
    if (st) return st;
    *cfg = P.cfg;
    return MR_OK;
}

int mr_batch_set_config(void* plan, const mr_batch_config* cfg) {
    if (!cfg) return fail(MR_E_NULL, "config is NULL");
    BatchPlan P;
    int st = load_plan(plan, P);
    if (!st) st = check_config(P, *cfg);
    if (st) return st;
    P.cfg = *cfg;
    memcpy(plan, &P, sizeof(P));
    return MR_OK;
}

int mr_batch_tune(void* plan, int reps, mr_batch_config* best, void* stream) {
    BatchPlan P;
    int st = load_plan(plan, P);
    if (st) return st;
    if (reps < 1 || reps > 1000) return fail(MR_E_PARAM, "reps %d outside [1, 1000]", reps);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(MR_E_DEVICE, "event creation failed");
    }
    // time of reps runs with configuration c after one warm-up run; a
    // persistent configuration whose runs gave up a wait is not a candidate
    // (its time is reported as infinite and the error word is cleared)
    auto time_of = [&](const mr_batch_config& c, float& ms) -> int {
        P.cfg = c;
        int r = run_plan(P, s);
        if (r) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(MR_E_DEVICE, "event record failed");
        for (int i = 0; i < reps && !r; ++i) r = run_plan(P, s);
        if (r) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return fail(MR_E_DEVICE, "batch timing failed");
        if (c.persistent) {
            unsigned err = 0;
            if (hipMemcpy(&err, P.fused_ctr + 2, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess)
                return fail(MR_E_DEVICE, "batch check failed");
            if (err) {
                const unsigned zero = 0;
                if (hipMemcpy(P.fused_ctr + 2, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
                    return fail(MR_E_DEVICE, "batch check failed");
                ms = std::numeric_limits<float>::infinity();
            }
        }
        return MR_OK;
    };
    // one choice at a time, the evaluation's schedule first (it dominates)
    mr_batch_config bc = P.cfg;
    float bt = 0.f;
    st = time_of(bc, bt);
    auto consider = [&](mr_batch_config c) {
        if (st || check_config(P, c) != MR_OK) return;
        float t = 0.f;
        st = time_of(c, t);
        if (!st && t < bt) {
            bt = t;
            bc = c;
        }
    };
    const mr_batch_config base = bc;
    for (int q = 0; q < 2; ++q)
        for (int bpc : {0, 8, 4, 2}) {
            mr_batch_config c = bc;
            c.eval_queue = q;
            c.eval_blocks_per_cu = bpc;
            if (c.eval_queue != base.eval_queue || c.eval_blocks_per_cu != base.eval_blocks_per_cu) consider(c);
        }
    for (int t = 0; t < 2; ++t) {
        mr_batch_config c = bc;
        c.edge_tile = t;
        if (t != bc.edge_tile) consider(c);
    }
    if (P.merge_geo != kMergeGeneral) {
        mr_batch_config c = bc;
        c.merge_generic = 1 - bc.merge_generic;
        consider(c);
    }
    // SSAO: the dense coarsest level in LDS depth tiles (fixed strides)
    for (int h : {8, 16, 24}) {
        mr_batch_config c = bc;
        c.eval_queue = 0;
        c.eval_halo = h;
        consider(c);  // check_config skips what does not apply
    }
    // the persistent launch, with the staged launches' merge choice
    if (fused_ok(P)) {
        const mr_batch_config staged = bc;
        for (int wp : {kDefaultWorkerPixels, 4 * kDefaultWorkerPixels})
            for (int it : {1, 2}) {
                mr_batch_config c = staged;
                c.persistent = 1;
                c.eval_halo = 0;
                c.worker_pixels = wp;
                c.eval_items = it;
                consider(c);
            }
        if (bc.persistent)
            for (int g : {4, 64}) {
                mr_batch_config c = bc;
                c.tiles_per_ticket = g;
                consider(c);
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    P.cfg = bc;
    memcpy(plan, &P, sizeof(P));
    if (best) *best = bc;
    return MR_OK;
}

int mr_batch_check(const void* plan, void* stream) {
    BatchPlan P;
    int st = load_plan(plan, P);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned err = 0;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipMemcpy(&err, P.fused_ctr + 2, sizeof(err), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(MR_E_DEVICE, "batch check failed: %s", hipGetErrorString(e));
    if (!err) return MR_OK;
    const unsigned zero = 0;
    e = hipMemcpy(P.fused_ctr + 2, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MR_E_DEVICE, "batch check failed: %s", hipGetErrorString(e));
    return fail(MR_E_DEVICE, "a persistent batch run gave up waiting for a stage (its outputs are not valid)");
}

const char* mr_status_string(int status) {
    switch (status) {
        case MR_OK: return "MR_OK";
        case MR_E_NULL: return "MR_E_NULL: a required pointer is NULL";
        case MR_E_SHAPE: return "MR_E_SHAPE: invalid image or map size";
        case MR_E_PARAM: return "MR_E_PARAM: parameter out of range or pointer misaligned";
        case MR_E_WORKSPACE: return "MR_E_WORKSPACE: workspace too small";
        case MR_E_DTYPE: return "MR_E_DTYPE: unsupported element type";
        case MR_E_DEVICE: return "MR_E_DEVICE: HIP launch failed";
        default: return "unknown status";
    }
}

const char* mr_last_error(void) { return g_err; }

int mr_version(void) { return MR_VERSION; }

}  // extern "C"
