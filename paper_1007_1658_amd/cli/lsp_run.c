/*
 * lsp_run -- periodogram of one series from the command line, through the C
 * ABI of libmi355lsp only (no Python): the normalized periodogram of Eqs.
 * (5)-(8) on the grid f_k = f_min + k df, k < Nf (Eq. (9) when f_min = df).
 *
 *   lsp_run T.bin X.bin f_min df Nf OUT.bin [gls]
 *
 * T.bin: Nt little-endian FP64 times; X.bin: Nt FP32 values; OUT.bin receives
 * Nf FP32 powers.  With the optional word "gls" the generalized (floating-mean)
 * periodogram with equal weights is written instead.  Prints Nt, Nf, the peak
 * bin and its power, and the device time of the call.  Exit status 0 on
 * success, 1 on a usage or I/O error, 2 on a library error (its message is
 * printed).
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lsp.h"

static void *read_file(const char *path, size_t elem, long *n)
{
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    fseek(f, 0, SEEK_END);
    const long bytes = ftell(f);
    fseek(f, 0, SEEK_SET);
    if (bytes <= 0 || bytes % (long)elem) {
        fclose(f);
        return NULL;
    }
    void *p = malloc((size_t)bytes);
    if (p && fread(p, 1, (size_t)bytes, f) != (size_t)bytes) {
        free(p);
        p = NULL;
    }
    fclose(f);
    *n = bytes / (long)elem;
    return p;
}

static int lib_fail(const char *what, lsp_status st)
{
    fprintf(stderr, "%s: %s (%s)\n", what, lsp_status_string(st), lsp_last_error());
    return 2;
}

int main(int argc, char **argv)
{
    if (argc != 7 && argc != 8) {
        fprintf(stderr, "usage: %s T.bin X.bin f_min df Nf OUT.bin [gls]\n", argv[0]);
        return 1;
    }
    const int gls = (argc == 8 && strcmp(argv[7], "gls") == 0);
    long nt = 0, nx = 0;
    double *t = (double *)read_file(argv[1], sizeof(double), &nt);
    float *x = (float *)read_file(argv[2], sizeof(float), &nx);
    if (!t || !x || nt != nx) {
        fprintf(stderr, "cannot read matching T and X files\n");
        return 1;
    }
    const double f_min = atof(argv[3]), df = atof(argv[4]);
    const long long nf = atoll(argv[5]);
    if (nf < 1) {
        fprintf(stderr, "Nf must be >= 1\n");
        return 1;
    }
    double *dt = NULL;
    float *dx = NULL, *dp = NULL;
    if (hipMalloc((void **)&dt, sizeof(double) * (size_t)nt) != hipSuccess ||
        hipMalloc((void **)&dx, sizeof(float) * (size_t)nt) != hipSuccess ||
        hipMalloc((void **)&dp, sizeof(float) * (size_t)nf) != hipSuccess ||
        hipMemcpy(dt, t, sizeof(double) * (size_t)nt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dx, x, sizeof(float) * (size_t)nt, hipMemcpyHostToDevice) != hipSuccess) {
        fprintf(stderr, "device allocation or copy failed\n");
        return 2;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 2;
    /* one untimed call sets up the workspace and launch shape */
    lsp_status st = gls ? lsp_gls(dt, dx, NULL, nt, f_min, df, nf, dp, 0, 0, NULL)
                        : lsp_periodogram(dt, dx, nt, f_min, df, nf, dp, NULL);
    if (st != LSP_OK) return lib_fail(gls ? "lsp_gls" : "lsp_periodogram", st);
    if (hipEventRecord(e0, NULL) != hipSuccess) return 2;
    st = gls ? lsp_gls(dt, dx, NULL, nt, f_min, df, nf, dp, 0, 0, NULL)
             : lsp_periodogram(dt, dx, nt, f_min, df, nf, dp, NULL);
    if (st != LSP_OK) return lib_fail(gls ? "lsp_gls" : "lsp_periodogram", st);
    float ms = 0.f;
    if (hipEventRecord(e1, NULL) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return 2;
    float *p = (float *)malloc(sizeof(float) * (size_t)nf);
    if (!p || hipMemcpy(p, dp, sizeof(float) * (size_t)nf, hipMemcpyDeviceToHost) != hipSuccess) return 2;
    long long kmax = 0;
    for (long long k = 1; k < nf; ++k)
        if (p[k] > p[kmax]) kmax = k;
    FILE *f = fopen(argv[6], "wb");
    if (!f || fwrite(p, sizeof(float), (size_t)nf, f) != (size_t)nf) {
        fprintf(stderr, "cannot write %s\n", argv[6]);
        return 1;
    }
    fclose(f);
    printf("Nt=%ld Nf=%lld peak k=%lld f=%.9g power=%.6g device_ms=%.4f\n", nt, nf, kmax,
           f_min + (double)kmax * df, (double)p[kmax], ms);
    (void)hipFree(dt);
    (void)hipFree(dx);
    (void)hipFree(dp);
    free(p);
    free(t);
    free(x);
    return 0;
}
