/*
 * A plain C client of libnpm (include/npm.h): no Python, no torch.  It
 * creates the 4-level dense network of the small workload, queries a batch
 * of positions in the unit cube with directions, trains on it for three
 * steps, and writes its inputs and outputs as raw float32 files into the
 * directory given as argv[1]: pos.f32 [3][n], dir.f32 [3][n], rad.f32 [n],
 * spdf.f32 [n], params0.f32 [n_params] (before training), pdf.f32 [n],
 * sdir.f32 [3][n], loss.f64 [3].  Exit status 0 on success, 77 without a
 * device, 1 on any other failure.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <math.h>

#include <hip/hip_runtime_api.h>

#include "npm.h"

#define N 4099

static int check(npm_status st, const char *what)
{
    if (st != NPM_OK) {
        fprintf(stderr, "%s: status %d: %s\n", what, (int)st, npm_last_error());
        return 1;
    }
    return 0;
}

#define HIP_OK(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));        \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static int dump(const char *dir, const char *name, const void *p, size_t bytes)
{
    char path[1024];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(p, 1, bytes, f) != bytes) return 1;
    fclose(f);
    return 0;
}

/* xorshift64*: deterministic inputs without a library */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static float uniform01(void)
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (float)((rng_state * 0x2545f4914f6cdd1dull) >> 40) * (1.0f / 16777216.0f);
}

int main(int argc, char **argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s OUTDIR\n", argv[0]);
        return 1;
    }
    npm_config cfg;
    if (check(npm_config_default(&cfg), "config")) return 1;
    cfg.grid_kind = NPM_GRID_DENSE;
    cfg.n_levels = 4;
    cfg.feat_per_level = 4;
    cfg.base_resolution = 8;
    cfg.max_resolution = 64;
    cfg.mlp_width = 64;
    cfg.mlp_hidden_layers = 2;
    cfg.exec_mode = NPM_EXEC_FUSED;
    cfg.grid_init = NPM_INIT_NORMAL;
    cfg.grid_init_scale = 1e-2f;
    cfg.lr = 1e-2f;
    cfg.seed = 11;
    npm_ctx *ctx = NULL;
    npm_status st = npm_create(&cfg, &ctx);
    if (st == NPM_ERR_NO_DEVICE) return 77;
    if (check(st, "create")) return 1;
    npm_layout lay;
    if (check(npm_get_layout(&cfg, &lay), "layout")) return 1;

    float *h_pos = malloc(sizeof(float) * 3 * N), *h_dir = malloc(sizeof(float) * 3 * N);
    float *h_rad = malloc(sizeof(float) * N), *h_spdf = malloc(sizeof(float) * N);
    float *h_pdf = malloc(sizeof(float) * N), *h_sdir = malloc(sizeof(float) * 3 * N);
    float *h_par = malloc(sizeof(float) * lay.n_params);
    for (int i = 0; i < N; ++i) {
        for (int d = 0; d < 3; ++d) h_pos[d * N + i] = uniform01();
        /* a direction: normalised from three uniforms in [-1, 1] */
        float v[3], s = 0.0f;
        do {
            s = 0.0f;
            for (int d = 0; d < 3; ++d) { v[d] = 2.0f * uniform01() - 1.0f; s += v[d] * v[d]; }
        } while (s > 1.0f || s < 1e-4f);
        float inv = 1.0f / sqrtf(s);
        for (int d = 0; d < 3; ++d) h_dir[d * N + i] = v[d] * inv;
        h_rad[i] = 0.1f + uniform01();
        h_spdf[i] = 1.0f / (4.0f * 3.14159265f);
    }
    if (check(npm_get_state(ctx, NPM_STATE_PARAMS, h_par, lay.n_params), "get params")) return 1;

    float *pos, *dir, *rad, *spdf, *pdf, *sdir;
    double *stats;
    HIP_OK(hipMalloc((void **)&pos, sizeof(float) * 3 * N));
    HIP_OK(hipMalloc((void **)&dir, sizeof(float) * 3 * N));
    HIP_OK(hipMalloc((void **)&rad, sizeof(float) * N));
    HIP_OK(hipMalloc((void **)&spdf, sizeof(float) * N));
    HIP_OK(hipMalloc((void **)&pdf, sizeof(float) * N));
    HIP_OK(hipMalloc((void **)&sdir, sizeof(float) * 3 * N));
    HIP_OK(hipMalloc((void **)&stats, sizeof(double) * 2));
    HIP_OK(hipMemcpy(pos, h_pos, sizeof(float) * 3 * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dir, h_dir, sizeof(float) * 3 * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(rad, h_rad, sizeof(float) * N, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(spdf, h_spdf, sizeof(float) * N, hipMemcpyHostToDevice));

    if (check(npm_query(ctx, N, pos, dir, 5, 0, NULL, pdf, sdir, NULL, NULL), "query")) return 1;
    double loss[3];
    for (int step = 0; step < 3; ++step) {
        if (check(npm_train_step(ctx, N, pos, dir, rad, spdf, stats, NULL), "train step")) return 1;
        double st2[2];
        /* the library's calls run on the null stream: this copy waits */
        HIP_OK(hipMemcpy(st2, stats, sizeof st2, hipMemcpyDeviceToHost));
        loss[step] = st2[0];
    }
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(h_pdf, pdf, sizeof(float) * N, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(h_sdir, sdir, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    int bad = dump(argv[1], "pos.f32", h_pos, sizeof(float) * 3 * N) |
              dump(argv[1], "dir.f32", h_dir, sizeof(float) * 3 * N) |
              dump(argv[1], "rad.f32", h_rad, sizeof(float) * N) |
              dump(argv[1], "spdf.f32", h_spdf, sizeof(float) * N) |
              dump(argv[1], "params0.f32", h_par, sizeof(float) * lay.n_params) |
              dump(argv[1], "pdf.f32", h_pdf, sizeof(float) * N) |
              dump(argv[1], "sdir.f32", h_sdir, sizeof(float) * 3 * N) |
              dump(argv[1], "loss.f64", loss, sizeof loss);
    printf("n %d n_params %lld loss %.9f %.9f %.9f\n", N, (long long)lay.n_params, loss[0], loss[1],
           loss[2]);
    npm_destroy(ctx);
    HIP_OK(hipFree(pos));
    HIP_OK(hipFree(dir));
    HIP_OK(hipFree(rad));
    HIP_OK(hipFree(spdf));
    HIP_OK(hipFree(pdf));
    HIP_OK(hipFree(sdir));
    HIP_OK(hipFree(stats));
    free(h_pos); free(h_dir); free(h_rad); free(h_spdf); free(h_pdf); free(h_sdir); free(h_par);
    return bad ? 1 : 0;
}
