/* abi_render.c -- uses the library through its C ABI alone (no Python): loads a scene blob,
 * views and parameters from files, renders on the default stream, runs the backward pass with
 * dL/dI = 1 for every image element, and writes the image followed by every slot's gradient.
 *
 * usage: abi_render scene.blob views.bin params.bin seed max_depth out.bin
 *   views.bin   n x 88-byte ppt_view records
 *   params.bin  the float32 parameter slots, concatenated in slot order
 */
#include <stdio.h>
#include <stdlib.h>
#include <hip/hip_runtime_api.h>
#include "ppt.h"

static void* read_file(const char* path, size_t* n) {
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    long len = ftell(f);
    fseek(f, 0, SEEK_SET);
    void* p = malloc(len > 0 ? (size_t)len : 1);
    if (p && len > 0 && fread(p, 1, (size_t)len, f) != (size_t)len) { free(p); p = NULL; }
    fclose(f);
    *n = (size_t)len;
    return p;
}

#define PPT(call) do { int rc_ = (call); if (rc_ != PPT_OK) { \
    fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, ppt_last_error()); return 1; } } while (0)
#define HIP(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) { \
    fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_)); return 1; } } while (0)

int main(int argc, char** argv) {
    if (argc != 7) { fprintf(stderr, "usage: abi_render scene.blob views.bin params.bin seed max_depth out.bin\n"); return 2; }
    size_t nblob, nviews, nparams;
    void* blob = read_file(argv[1], &nblob);
    ppt_view* views = (ppt_view*)read_file(argv[2], &nviews);
    float* hparams = (float*)read_file(argv[3], &nparams);
    if (!blob || !views || !hparams || nviews % sizeof(ppt_view)) { fprintf(stderr, "bad input files\n"); return 2; }
    unsigned long long seed = strtoull(argv[4], NULL, 10);
    int max_depth = atoi(argv[5]);

    ppt_scene* scene = NULL;
    PPT(ppt_scene_create(blob, nblob, &scene));
    int32_t n_slots = 0;
    int64_t numel[64];
    PPT(ppt_scene_slots(scene, &n_slots, numel, 64));
    const float* dparams[64];
    float* dgrads[64];
    size_t at = 0;
    for (int s = 0; s < n_slots; ++s) {
        float* p = NULL;
        float* g = NULL;
        HIP(hipMalloc((void**)&p, (size_t)(numel[s] > 0 ? numel[s] : 1) * sizeof(float)));
        HIP(hipMalloc((void**)&g, (size_t)(numel[s] > 0 ? numel[s] : 1) * sizeof(float)));
        if ((at + (size_t)numel[s]) * sizeof(float) > nparams) { fprintf(stderr, "params.bin too short\n"); return 2; }
        HIP(hipMemcpy(p, hparams + at, (size_t)numel[s] * sizeof(float), hipMemcpyHostToDevice));
        at += (size_t)numel[s];
        dparams[s] = p;
        dgrads[s] = g;
    }

    ppt_plan* plan = NULL;
    PPT(ppt_plan_create(scene, views, (int32_t)(nviews / sizeof(ppt_view)), max_depth, 0u, NULL, &plan));
    int64_t n_img = ppt_plan_image_numel(plan);
    size_t ws_r = ppt_plan_workspace_bytes(plan, 0), ws_b = ppt_plan_workspace_bytes(plan, 1);
    size_t ws_bytes = ws_r > ws_b ? ws_r : ws_b;
    float *img = NULL, *dimg = NULL;
    void* ws = NULL;
    HIP(hipMalloc((void**)&img, (size_t)n_img * sizeof(float)));
    HIP(hipMalloc((void**)&dimg, (size_t)n_img * sizeof(float)));
    HIP(hipMalloc(&ws, ws_bytes));
    float* ones = (float*)malloc((size_t)n_img * sizeof(float));
    for (int64_t i = 0; i < n_img; ++i) ones[i] = 1.0f;
    HIP(hipMemcpy(dimg, ones, (size_t)n_img * sizeof(float), hipMemcpyHostToDevice));

    PPT(ppt_render(plan, dparams, n_slots, seed, img, ws, ws_bytes, NULL));
    PPT(ppt_backward(plan, dparams, n_slots, seed, dimg, dgrads, ws, ws_bytes, NULL));
    HIP(hipDeviceSynchronize());

    FILE* f = fopen(argv[6], "wb");
    if (!f) return 1;
    float* host = (float*)malloc((size_t)n_img * sizeof(float));
    HIP(hipMemcpy(host, img, (size_t)n_img * sizeof(float), hipMemcpyDeviceToHost));
    fwrite(host, sizeof(float), (size_t)n_img, f);
    for (int s = 0; s < n_slots; ++s) {
        float* hg = (float*)malloc((size_t)(numel[s] > 0 ? numel[s] : 1) * sizeof(float));
        HIP(hipMemcpy(hg, dgrads[s], (size_t)numel[s] * sizeof(float), hipMemcpyDeviceToHost));
        fwrite(hg, sizeof(float), (size_t)numel[s], f);
        free(hg);
    }
    fclose(f);
    printf("rendered %lld values, %d gradient slots\n", (long long)n_img, n_slots);
    ppt_plan_destroy(plan);
    ppt_scene_destroy(scene);
    return 0;
}
