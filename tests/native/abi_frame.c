/* A C client that runs frames on the GPU through the library's boundary:
 * device memory from hipMalloc, a 512 x 256 G-buffer of a fronto-parallel
 * plane (depth 10, normal +z toward the camera).  The plane has no edges, so
 * every pixel's owner level is the coarsest (Sec. 3.1), and every SSAO sample
 * of the normal hemisphere lies in front of the plane, so nothing occludes
 * (Sec. 2.4): the multi-resolution image, the naive image and the tuned frame
 * are all exactly 0.  Prints one line per check and exits 0 when all hold. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mr.h"

enum { W = 512, H = 256, S = 32 };

static int failures = 0;

static void check(int ok, const char* what) {
    printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok) ++failures;
}

static int all_equal(const float* d, size_t n, float v) {
    for (size_t i = 0; i < n; ++i)
        if (d[i] != v) return 0;
    return 1;
}

int main(void) {
    const size_t npx = (size_t)W * H;
    float* hz = malloc(npx * sizeof(float));
    float* hn = calloc(3 * npx, sizeof(float));
    float* hk = malloc(3 * S * sizeof(float));
    float* hout = malloc(npx * sizeof(float));
    unsigned char* hmap = malloc(npx);
    if (!hz || !hn || !hk || !hout || !hmap) return 2;
    for (size_t i = 0; i < npx; ++i) {
        hz[i] = 10.0f;
        hn[2 * npx + i] = 1.0f;
    }
    /* S points in the unit hemisphere around +z, lengths growing with the index */
    for (int s = 0; s < S; ++s) {
        const double a = 2.399963 * s, r = 0.1 + 0.9 * (s + 0.5) / S, c = (s + 0.5) / S;
        hk[3 * s] = (float)(r * sqrt(1.0 - c * c) * cos(a));
        hk[3 * s + 1] = (float)(r * sqrt(1.0 - c * c) * sin(a));
        hk[3 * s + 2] = (float)(r * c);
    }

    float *dz = NULL, *dn = NULL, *dk = NULL, *dout = NULL;
    unsigned char* dmap = NULL;
    if (hipMalloc((void**)&dz, npx * 4) != hipSuccess || hipMalloc((void**)&dn, 3 * npx * 4) != hipSuccess ||
        hipMalloc((void**)&dk, 3 * S * 4) != hipSuccess || hipMalloc((void**)&dout, npx * 4) != hipSuccess ||
        hipMalloc((void**)&dmap, npx) != hipSuccess) {
        printf("FAIL hipMalloc\n");
        return 2;
    }
    hipMemcpy(dz, hz, npx * 4, hipMemcpyHostToDevice);
    hipMemcpy(dn, hn, 3 * npx * 4, hipMemcpyHostToDevice);
    hipMemcpy(dk, hk, 3 * S * 4, hipMemcpyHostToDevice);

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
    mr_ssao_params sp = {dk, S, 1.0f, 0.02f};
    mr_frame_desc d;
    memset(&d, 0, sizeof(d));
    d.effect = MR_EFFECT_SSAO;
    d.multires = 1;
    d.g.depth = dz;
    d.g.normal = dn;
    d.g.normal_dtype = MR_F32;
    d.cam.width = W;
    d.cam.height = H;
    d.cam.focal_px = 221.7025f;
    d.mp = mp;
    d.ssao = &sp;
    d.out = dout;
    d.level_map = dmap;

    const size_t ws_bytes = mr_workspace_bytes(&d.cam, &d.mp, MR_EFFECT_SSAO);
    void* ws = NULL;
    check(ws_bytes > 0 && hipMalloc(&ws, ws_bytes) == hipSuccess, "workspace sized and allocated");

    hipMemset(dout, 0xFF, npx * 4);
    check(mr_frame(&d, ws, ws_bytes, NULL) == MR_OK, "mr_frame (multi-resolution) returns MR_OK");
    check(hipDeviceSynchronize() == hipSuccess, "the frame completes");
    hipMemcpy(hout, dout, npx * 4, hipMemcpyDeviceToHost);
    hipMemcpy(hmap, dmap, npx, hipMemcpyDeviceToHost);
    check(all_equal(hout, npx, 0.0f), "multi-resolution image is exactly 0");
    int coarsest = 1;
    for (size_t i = 0; i < npx; ++i) coarsest &= hmap[i] == 4;
    check(coarsest, "every pixel's owner level is the coarsest");

    d.multires = 0;
    d.level_map = NULL;
    hipMemset(dout, 0xFF, npx * 4);
    check(mr_frame(&d, ws, ws_bytes, NULL) == MR_OK && hipDeviceSynchronize() == hipSuccess,
          "mr_frame (naive) returns MR_OK and completes");
    hipMemcpy(hout, dout, npx * 4, hipMemcpyDeviceToHost);
    check(all_equal(hout, npx, 0.0f), "naive image is exactly 0");

    d.multires = 1;
    float ms[4] = {0, 0, 0, 0};
    check(mr_frame_tune(&d, ws, ws_bytes, 2, ms, NULL) == MR_OK, "mr_frame_tune returns MR_OK");
    check(d.eval_halo == 0 || d.eval_halo == 8 || d.eval_halo == 16 || d.eval_halo == 24,
          "the tuned halo is one of 0, 8, 16, 24");
    check(ms[0] > 0.0f && ms[1] > 0.0f && ms[2] > 0.0f && ms[3] > 0.0f, "every halo was timed");
    hipMemset(dout, 0xFF, npx * 4);
    check(mr_frame(&d, ws, ws_bytes, NULL) == MR_OK && hipDeviceSynchronize() == hipSuccess,
          "the tuned frame runs");
    hipMemcpy(hout, dout, npx * 4, hipMemcpyDeviceToHost);
    check(all_equal(hout, npx, 0.0f), "tuned image is exactly 0");

    hipFree(ws);
    hipFree(dz);
    hipFree(dn);
    hipFree(dk);
    hipFree(dout);
    hipFree(dmap);
    free(hz);
    free(hn);
    free(hk);
    free(hout);
    free(hmap);
    printf("%d failure(s)\n", failures);
    return failures ? 1 : 0;
}
