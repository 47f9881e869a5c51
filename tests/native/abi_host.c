/* A C client of the library's boundary: includes mr.h as a C11 header,
 * links libmr.so and calls the entry points that run on the host (sizes,
 * layouts, argument validation, status strings).  No GPU is needed; the
 * test suite builds and runs it with gcc.  Prints one line per check and
 * exits 0 when every check holds. */
#include <stdio.h>
#include <string.h>

#include "mr.h"

static int failures = 0;

static void check(int ok, const char* what) {
    printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok) ++failures;
}

int main(void) {
    /* 3840 x 2160, four levels, Table 1's SSAO column (Sec. 3.1) */
    mr_camera cam = {3840, 2160, 1870.6149f};
    mr_mask_params mp;
    memset(&mp, 0, sizeof(mp));
    mp.num_levels = 4;
    mp.level_enable = 0xFu;
    mp.depth_ratio = 0.05f;
    mp.normal_cos = 0.9063078165054321f;
    const float s2[4] = {0.924f, 1.848f, 3.696f, 0.0f}, w[4] = {100.0f, 50.0f, 20.0f, 1.0f};
    for (int i = 0; i < 4; ++i) {
        mp.sigma2[i] = s2[i];
        mp.weight[i] = w[i];
        mp.radius[i] = -1;
    }

    const size_t ws = mr_workspace_bytes(&cam, &mp, MR_EFFECT_SSAO);
    check(ws > 0 && ws % 16 == 0, "mr_workspace_bytes of a 4K SSAO frame");
    check(mr_workspace_bytes(&cam, &mp, MR_WS_MASKS) > 0, "mr_workspace_bytes of the mask API");

    mr_frame_layout lay;
    check(mr_frame_workspace_layout(&cam, &mp, MR_EFFECT_SSAO, &lay) == MR_OK && lay.compact == 1 &&
              lay.tile_words == 16 && lay.tile_rows == 32,
          "mr_frame_workspace_layout: the compact path, 16 x 32 word ranking tiles");
    int inside = 1;
    for (int i = 0; i < 3; ++i)
        inside &= lay.worklist[i] < ws && lay.stencil_bits[i] < ws && lay.rank[i] < ws;
    check(inside, "every list level's regions start inside the workspace");

    size_t pyr = 0, scr = 0;
    check(mr_pyramid_bytes(&cam, &mp, MR_EFFECT_SSAO, &pyr, &scr) == MR_OK && pyr > 0 && scr > 0,
          "mr_pyramid_bytes: pyramid and scratch parts");

    /* argument validation: nothing is enqueued, a code and a message come back */
    check(mr_frame(NULL, NULL, 0, NULL) == MR_E_NULL && strlen(mr_last_error()) > 0,
          "mr_frame(NULL) is MR_E_NULL with a message");
    check(mr_frame_tune(NULL, NULL, 0, 3, NULL, NULL) == MR_E_NULL, "mr_frame_tune(NULL) is MR_E_NULL");
    mr_camera bad = {MR_MAX_DIM + 1, 64, 50.0f};
    check(mr_workspace_bytes(&bad, &mp, MR_EFFECT_SSAO) == 0 && strstr(mr_last_error(), "16384") != NULL,
          "a width above MR_MAX_DIM is refused");
    mr_camera odd = {1000, 1002, 50.0f};
    check(mr_workspace_bytes(&odd, &mp, MR_EFFECT_SSAO) == 0, "a size not divisible by 2^(N-1) is refused");

    check(mr_version() == MR_VERSION, "mr_version is the header's MR_VERSION");

    /* a frame whose parameters are out of range is refused before anything
     * is enqueued (the device pointers are never dereferenced) */
    mr_ssao_params sp = {(const float*)(void*)4096, 16, 0.5f, 0.02f};
    mr_frame_desc d;
    memset(&d, 0, sizeof(d));
    d.effect = MR_EFFECT_SSAO;
    d.multires = 1;
    d.g.depth = (const float*)(void*)4096;
    d.g.normal = (const void*)8192;
    d.g.normal_dtype = MR_F32;
    d.cam = cam;
    d.mp = mp;
    d.ssao = &sp;
    d.out = (float*)(void*)4096;
    d.mp.sigma2[0] = -1.0f;
    check(mr_frame(&d, (void*)4096, ws, NULL) == MR_E_PARAM, "sigma2 < 0 is MR_E_PARAM");
    d.mp = mp;
    d.mp.normal_cos = 2.0f;
    check(mr_frame(&d, (void*)4096, ws, NULL) == MR_E_PARAM, "normal_cos outside [-1, 1] is MR_E_PARAM");
    d.mp = mp;
    sp.samples = 0;
    check(mr_frame(&d, (void*)4096, ws, NULL) == MR_E_PARAM, "0 samples is MR_E_PARAM");
    sp.samples = 16;
    check(mr_frame(&d, (void*)4096, 100, NULL) == MR_E_WORKSPACE, "a small workspace is MR_E_WORKSPACE");

    int named = 1;
    const int codes[] = {MR_OK, MR_E_NULL, MR_E_SHAPE, MR_E_PARAM, MR_E_WORKSPACE, MR_E_DTYPE, MR_E_DEVICE};
    for (int i = 0; i < 7; ++i) named &= mr_status_string(codes[i]) != NULL && strlen(mr_status_string(codes[i])) > 0;
    check(named, "mr_status_string names every status code");

    printf("%d failure(s)\n", failures);
    return failures ? 1 : 0;
}
