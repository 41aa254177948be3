/* A C program on the library's C ABI alone (no Python): a context created
 * from a launch-table file launches the stored geometry.
 *   1. a table holding APE geometries for 8x8x8x8 FP64 and 16x8x4x8 FP32-12
 *      is written;
 *   2. qdpx_create reads it: qdpx_tune_get reports that geometry, source 1
 *      (an entry without the LDS tile field gets the default tile);
 *   3. unit links are packed and smeared one step in that geometry: they
 *      stay unit links (a fixed point of the step), plaquette 1;
 *   4. a geometry set on another shape is saved into the table and a second
 *      context created through QDPX_TUNE_CACHE reads both;
 *   5. a malformed table makes qdpx_create fail with QDPX_EINVAL.
 * Usage: c_abi_check <scratch directory>.  Prints "ok" on success. */
#define _POSIX_C_SOURCE 200112L
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "../include/qdpx.h"

#define CHECK(cond, ...)                        \
    do {                                        \
        if (!(cond)) {                          \
            fprintf(stdout, "FAIL line %d: ", __LINE__); \
            fprintf(stdout, __VA_ARGS__);       \
            fprintf(stdout, " (%s)\n", qdpx_last_error()); \
            return 1;                           \
        }                                       \
    } while (0)

static int write_text(const char *path, const char *text) {
    FILE *f = fopen(path, "w");
    if (!f) return -1;
    fputs(text, f);
    return fclose(f);
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    char table[4096], bad[4096];
    snprintf(table, sizeof table, "%s/table.json", argv[1]);
    snprintf(bad, sizeof bad, "%s/bad.json", argv[1]);
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0) == hipSuccess, "no device");
    char text[8192];
    snprintf(text, sizeof text,
             "{\"device\": \"%s\", \"entries\": [\n"
             " {\"op\": \"APE\", \"prec\": \"F64\", \"fmt\": \"LINK18\", \"L\": [8, 8, 8, 8], "
             "\"launch\": [512, 2, 0, 2]},\n"
             " {\"op\": \"APE\", \"prec\": \"F32\", \"fmt\": \"LINK12\", \"L\": [16, 8, 4, 8], "
             "\"launch\": [256, 1, 2, 1, 1]}\n]}\n",
             prop.gcnArchName);
    CHECK(write_text(table, text) == 0, "cannot write %s", table);

    qdpx_ctx *ctx = NULL;
    CHECK(qdpx_create(&ctx, 0, table) == QDPX_OK, "qdpx_create with a table");
    const qdpx_geom g = {{8, 8, 8, 8}};
    int32_t b = 0, n = 0, x = 0, t = 0, d = -1, src = -1;
    CHECK(qdpx_tune_get(ctx, QDPX_OP_APE, &g, QDPX_F64, QDPX_LINK18, &b, &n, &x, &t, &d, &src) == QDPX_OK,
          "tune_get");
    CHECK(b == 512 && n == 2 && x == 0 && t == 2 && d == 0 && src == 1,
          "stored geometry not read: %d %d %d %d %d source %d", b, n, x, t, d, src);
    CHECK(qdpx_tune_get(ctx, QDPX_OP_APE, &g, QDPX_F32, QDPX_LINK12, &b, &n, &x, &t, &d, &src) == QDPX_OK &&
              src == 0 && b == 256 && d == 4,
          "an absent shape is not the default");
    const qdpx_geom g3 = {{16, 8, 4, 8}};
    CHECK(qdpx_tune_get(ctx, QDPX_OP_APE, &g3, QDPX_F32, QDPX_LINK12, &b, &n, &x, &t, &d, &src) == QDPX_OK &&
              b == 256 && n == 1 && x == 2 && t == 1 && d == 1 && src == 1,
          "stored LDS tile not read: %d %d %d %d %d source %d", b, n, x, t, d, src);

    /* unit links, one APE step in the stored geometry */
    const size_t V = 8 * 8 * 8 * 8, nreal = V * 4 * 18;
    double *host = (double *)calloc(nreal, sizeof(double));
    for (size_t l = 0; l < V * 4; ++l)
        for (int a = 0; a < 3; ++a) host[l * 18 + (a * 3 + a) * 2] = 1.0;
    void *aos = NULL, *soa = NULL, *out = NULL, *work = NULL, *plaq = NULL;
    const size_t lb = qdpx_links_bytes(&g, QDPX_F64, QDPX_LINK18);
    const size_t wb = qdpx_workspace_bytes(QDPX_OP_APE, &g, QDPX_F64, QDPX_LINK18, 1);
    CHECK(lb && wb, "sizes");
    CHECK(hipMalloc(&aos, nreal * 8) == hipSuccess && hipMalloc(&soa, lb) == hipSuccess &&
              hipMalloc(&out, lb) == hipSuccess && hipMalloc(&work, wb) == hipSuccess &&
              hipMalloc(&plaq, 6 * sizeof(double)) == hipSuccess,
          "hipMalloc");
    CHECK(hipMemcpy(aos, host, nreal * 8, hipMemcpyHostToDevice) == hipSuccess, "copy in");
    CHECK(qdpx_pack_links(ctx, &g, (const double *)aos, QDPX_F64, QDPX_LINK18, soa, NULL) == QDPX_OK, "pack");
    CHECK(qdpx_ape_smear(ctx, &g, QDPX_F64, QDPX_LINK18, soa, out, 0.5, 1, 0xFu, QDPX_PROJ_GRAM_SCHMIDT,
                         (double *)plaq, work, wb, NULL) == QDPX_OK,
          "ape_smear");
    CHECK(qdpx_unpack_links(ctx, &g, out, QDPX_F64, QDPX_LINK18, (double *)aos, NULL) == QDPX_OK, "unpack");
    double p[6];
    CHECK(hipMemcpy(host, aos, nreal * 8, hipMemcpyDeviceToHost) == hipSuccess &&
              hipMemcpy(p, plaq, sizeof p, hipMemcpyDeviceToHost) == hipSuccess,
          "copy out");
    double dev = 0.0;
    for (size_t l = 0; l < V * 4; ++l)
        for (int e = 0; e < 9; ++e) {
            const double re = host[l * 18 + e * 2], im = host[l * 18 + e * 2 + 1];
            const double want = (e % 4 == 0) ? 1.0 : 0.0;
            dev = fmax(dev, fmax(fabs(re - want), fabs(im)));
        }
    CHECK(dev < 1e-15, "unit links moved by %g", dev);
    for (int i = 0; i < 6; ++i) CHECK(fabs(p[i] - 1.0) < 1e-15, "plaquette %d = %.17g", i, p[i]);

    /* a geometry set on another shape, saved and read back through the environment */
    const qdpx_geom g2 = {{16, 8, 4, 8}};
    CHECK(qdpx_tune_set(ctx, QDPX_OP_SHIFT, &g2, QDPX_F32, QDPX_LINK12, 256, 4, 1, 2, 0) == QDPX_OK, "tune_set");
    CHECK(qdpx_tune_set(ctx, QDPX_OP_SHIFT, &g2, QDPX_F32, QDPX_LINK12, 256, 4, 1, 2, 1) == QDPX_EINVAL,
          "an LDS tile outside the FP32 APE step accepted");
    CHECK(qdpx_tune_save(ctx, NULL) == QDPX_OK, "tune_save");
    qdpx_destroy(ctx);
    setenv("QDPX_TUNE_CACHE", table, 1);
    qdpx_ctx *ctx2 = NULL;
    CHECK(qdpx_create(&ctx2, 0, NULL) == QDPX_OK, "qdpx_create through QDPX_TUNE_CACHE");
    CHECK(qdpx_tune_get(ctx2, QDPX_OP_SHIFT, &g2, QDPX_F32, QDPX_LINK12, &b, &n, &x, &t, &d, &src) == QDPX_OK &&
              b == 256 && n == 4 && x == 1 && t == 2 && d == 0 && src == 1,
          "saved geometry not read back");
    CHECK(qdpx_tune_get(ctx2, QDPX_OP_APE, &g, QDPX_F64, QDPX_LINK18, &b, &n, &x, &t, &d, &src) == QDPX_OK &&
              b == 512 && src == 1,
          "first geometry lost by the save");
    CHECK(qdpx_tune_get(ctx2, QDPX_OP_APE, &g3, QDPX_F32, QDPX_LINK12, &b, &n, &x, &t, &d, &src) == QDPX_OK &&
              d == 1 && src == 1,
          "LDS tile lost by the save");
    qdpx_destroy(ctx2);

    /* a malformed table, and an invalid geometry, are refused */
    CHECK(write_text(bad, "{\"device\": \"x\", \"entries\": [") == 0, "cannot write %s", bad);
    qdpx_ctx *ctx3 = NULL;
    CHECK(qdpx_create(&ctx3, 0, bad) == QDPX_EINVAL && ctx3 == NULL, "malformed table accepted");
    snprintf(text, sizeof text,
             "{\"device\": \"%s\", \"entries\": [{\"op\": \"APE\", \"prec\": \"F64\", \"fmt\": \"LINK18\", "
             "\"L\": [8, 8, 8, 8], \"launch\": [192, 1, 0, 1]}]}",
             prop.gcnArchName);
    CHECK(write_text(bad, text) == 0, "cannot write %s", bad);
    CHECK(qdpx_create(&ctx3, 0, bad) == QDPX_EINVAL && ctx3 == NULL, "invalid geometry accepted");

    (void)hipFree(aos);
    (void)hipFree(soa);
    (void)hipFree(out);
    (void)hipFree(work);
    (void)hipFree(plaq);
    free(host);
    printf("ok\n");
    return 0;
}
