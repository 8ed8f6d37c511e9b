#define _POSIX_C_SOURCE 200809L /* mkstemp, fdopen */
/* Host-only exercise of the C-ABI (test helper): every entry point that
 * needs no device, with valid and invalid arguments, for a build of the
 * library whose host code carries AddressSanitizer. Prints "ok" and exits 0
 * when every return code is the documented one. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

static int fails = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "line %d: %s\n", __LINE__, #cond);         \
            ++fails;                                                   \
        }                                                              \
    } while (0)

int main(void)
{
    double c[41 * 3], w[41], t0 = 0.0;
    EXPECT(lbm_lattice(c, w, &t0) == LBM_OK);
    EXPECT(lbm_lattice(NULL, NULL, NULL) == LBM_OK);
    EXPECT(t0 > 0.29 && t0 < 0.3);
    EXPECT(lbm_selftest() == LBM_OK);

    lbm_box box = {5, 3, 2, 0, 0.6};
    lbm_opts opts;
    memset(&opts, 0, sizeof(opts));
    opts.storage = LBM_F32;
    opts.tau_conv = LBM_TAU_LB;
    opts.rho0 = 1.0;
    opts.shift_exp = LBM_SHIFT_AUTO;
    uint64_t bytes = 0;
    EXPECT(lbm_workspace_size(&box, 1, &opts, &bytes) == LBM_OK && bytes > 0);
    EXPECT(lbm_workspace_size(&box, 1, &opts, NULL) == LBM_E_ARG);
    EXPECT(lbm_workspace_size(NULL, 1, &opts, &bytes) == LBM_E_ARG);
    EXPECT(lbm_workspace_size(&box, 0, &opts, &bytes) == LBM_E_ARG);
    lbm_box bad = box;
    bad.tau = 0.5;
    EXPECT(lbm_workspace_size(&bad, 1, &opts, &bytes) == LBM_E_ARG);
    bad = box;
    bad.nx = 0;
    EXPECT(lbm_workspace_size(&bad, 1, &opts, &bytes) == LBM_E_ARG);
    lbm_opts o2 = opts;
    o2.storage = (lbm_storage)9;
    EXPECT(lbm_workspace_size(&box, 1, &o2, &bytes) == LBM_E_ARG);
    o2 = opts;
    o2.flags = 0x80u;
    EXPECT(lbm_workspace_size(&box, 1, &o2, &bytes) == LBM_E_ARG);

    /* host collision of a perturbed rest state, both models and precisions */
    double f[41], g[41];
    for (int q = 0; q < 41; ++q) f[q] = w[q] * (1.0 + 1e-3 * sin(1.0 + q));
    for (int pr = 0; pr < 2; ++pr)
        for (uint32_t fl = 0; fl <= LBM_FLAG_ISOTHERMAL; fl += LBM_FLAG_ISOTHERMAL) {
            EXPECT(lbm_collide_host(pr, pr ? 1 : 3, fl, 1.0 / 0.6, f, g) == LBM_OK);
            double m0 = 0.0, m1 = 0.0;
            for (int q = 0; q < 41; ++q) {
                m0 += f[q];
                m1 += g[q];
            }
            EXPECT(fabs(m1 - m0) < 1e-6);
        }
    EXPECT(lbm_collide_host(2, 1, 0, 1.0, f, g) == LBM_E_ARG);
    EXPECT(lbm_collide_host(0, 9, 0, 1.0, f, g) == LBM_E_ARG);
    EXPECT(lbm_collide_host(0, 1, 0x10u, 1.0, f, g) == LBM_E_ARG);
    EXPECT(lbm_collide_host(0, 1, 0, 1.0, NULL, g) == LBM_E_ARG);

    int32_t blk = 0;
    uint32_t flags = 0;
    EXPECT(lbm_num_variants() > 0);
    EXPECT(lbm_variant_desc(0, &blk, &flags) == LBM_OK && blk > 0);
    EXPECT(lbm_variant_desc(-1, &blk, &flags) == LBM_E_ARG);
    EXPECT(lbm_variant_desc(lbm_num_variants(), &blk, &flags) == LBM_E_ARG);
    for (int code = 1; code >= -8; --code) EXPECT(lbm_strerror(code) != NULL && strlen(lbm_strerror(code)) > 0);

    /* lbm_init: argument and domain errors are found before device work */
    const int n = 2 * 5 * 3 * 2;
    double *rho = malloc(sizeof(double) * n), *ux = calloc(n, sizeof(double)), *uy = calloc(n, sizeof(double)),
           *uz = calloc(n, sizeof(double)), *th = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) {
        rho[i] = 1.0;
        th[i] = t0;
    }
    lbm_ctx *ctx = (lbm_ctx *)0x1;
    EXPECT(lbm_init(NULL, &box, 1, &opts, rho, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_ARG);
    EXPECT(lbm_init(&ctx, &box, 1, &opts, NULL, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_ARG && ctx == NULL);
    EXPECT(lbm_init(&ctx, &box, 0, &opts, rho, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_ARG);
    rho[n - 1] = -1.0;
    EXPECT(lbm_init(&ctx, &box, 1, &opts, rho, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_DOMAIN && ctx == NULL);
    rho[n - 1] = 1.0;
    th[3] = NAN;
    EXPECT(lbm_init(&ctx, &box, 1, &opts, rho, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_DOMAIN);
    EXPECT(lbm_init_device(NULL, &box, 1, &opts, rho, ux, uy, uz, th, NULL, NULL, 0) == LBM_E_ARG);
    free(rho);
    free(ux);
    free(uy);
    free(uz);
    free(th);

    /* NULL contexts */
    lbm_info info;
    lbm_tuning tun;
    double out5[5];
    EXPECT(lbm_step(NULL, 1) == LBM_E_ARG);
    EXPECT(lbm_get_info(NULL, &info) == LBM_E_ARG);
    EXPECT(lbm_get_tuning(NULL, &tun) == LBM_E_ARG);
    EXPECT(lbm_totals(NULL, out5) == LBM_E_ARG);
    EXPECT(lbm_status(NULL) == LBM_E_ARG);
    EXPECT(lbm_stream(NULL) == NULL);
    lbm_free(NULL);

    /* the tuning cache file: valid entries, a one-token line, extra tokens,
       out-of-range values and an over-long line */
    {
        char path[] = "/tmp/lbm_tune_asan_XXXXXX";
        int fd = mkstemp(path);
        EXPECT(fd >= 0);
        FILE *f = fdopen(fd, "w");
        fprintf(f, "keyA 0 1 0 0\nlonely\nkeyB 1 0 1 16\nkeyC 1 0 1 16 extra\nkeyD 99 0 0 0\nkeyE 0 1 0 3\n");
        for (int i = 0; i < 20000; ++i) fputc('x', f);
        fprintf(f, " 0 1 0 0\nkeyF 2 1 1 64\n");
        fclose(f);
        EXPECT(lbm_tune_cache_clear() == LBM_OK);
        EXPECT(lbm_tune_cache_file(path) == LBM_OK);
        EXPECT(lbm_tune_cache_count() == 3); /* keyA, keyB, keyF */
        EXPECT(lbm_tune_cache_file(NULL) == LBM_OK);
        EXPECT(lbm_tune_cache_clear() == LBM_OK && lbm_tune_cache_count() == 0);
        remove(path);
    }
    /* the allocation-free totals reject bad arguments before any device call */
    {
        double dev_out[5];
        lbm_box big = {65536, 65536, 2, 0, 0.6};
        EXPECT(lbm_totals_noalloc(NULL, LBM_F32, &box, 60, 1.0, 0, NULL, dev_out) == LBM_E_ARG);
        EXPECT(lbm_totals_noalloc(dev_out, 9, &box, 60, 1.0, 0, NULL, dev_out) == LBM_E_ARG);
        EXPECT(lbm_totals_noalloc(dev_out, LBM_F32, &box, 59, 1.0, 0, NULL, dev_out) == LBM_E_ARG);
        EXPECT(lbm_totals_noalloc(dev_out, LBM_F16_SHIFT, &big, (1ull << 33), 1.0, 0, NULL, dev_out) == LBM_E_ARG);
    }
    /* the plain copy rejects bad arguments before any launch; 0 bytes is a no-op */
    {
        _Alignas(16) unsigned char a[64], b[64];
        EXPECT(lbm_device_copy(NULL, b, 16, NULL) == LBM_E_ARG);
        EXPECT(lbm_device_copy(a, NULL, 16, NULL) == LBM_E_ARG);
        EXPECT(lbm_device_copy(a, b, 24, NULL) == LBM_E_ARG);       /* not a multiple of 16 */
        EXPECT(lbm_device_copy(a + 8, b, 16, NULL) == LBM_E_ARG);   /* misaligned */
        EXPECT(lbm_device_copy(a, a + 16, 32, NULL) == LBM_E_ARG);  /* overlapping */
        EXPECT(lbm_device_copy(a, b, 0, NULL) == LBM_OK);
    }

    if (fails) return 1;
    printf("ok\n");
    return 0;
}
