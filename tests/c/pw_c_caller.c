/*
 * pw_c_caller.c -- TEST PROGRAM: a plain C99 caller of libpwadvect.
 *
 * Uses the library the way a C or Fortran host code would: device arrays from
 * hipMalloc, the C header include/pwadvect.h, no Python.  It fills the winds
 * and multipliers on the device with pw_fill_uniform and pw_halo_periodic,
 * runs pw_advect_fwd and pw_advect_fwd_adj (FP64) on the default stream, and
 * checks them against the FP64 oracle (oracle/libpworacle.so, test
 * infrastructure) on the same inputs:
 *   - su, sv, sw of both calls equal the oracle's forward (section 2.1,
 *     Listing 1) bit for bit on every interior cell;
 *   - gu, gv, gw are within 1e-12 of the oracle's scatter adjoint, normwise
 *     (largest difference over largest magnitude, per field).
 * Prints one line and exits 0 on success, 1 on a mismatch, 2 on an error.
 * Usage: pw_c_caller [nx ny nz halo]
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/pwadvect.h"

/* the oracle's entry points (oracle/pw_oracle.c) */
void pw_oracle_fwd(const double *u, const double *v, const double *w, const double *tzc1, const double *tzc2,
                   double tcx, double tcy, int nx, int ny, int nz, int h, double *su, double *sv, double *sw);
void pw_oracle_adj(const double *u, const double *v, const double *w, const double *lu, const double *lv,
                   const double *lw, const double *tzc1, const double *tzc2, double tcx, double tcy, int nx, int ny,
                   int nz, int h, double *gu, double *gv, double *gw);

#define HIP_OK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            printf("pw_c_caller: %s failed: %s\n", #call, hipGetErrorString(e_));        \
            return 2;                                                                     \
        }                                                                                 \
    } while (0)
#define PW_OK_(call)                                                                      \
    do {                                                                                  \
        int r_ = (call);                                                                  \
        if (r_ != PW_OK) {                                                                \
            printf("pw_c_caller: %s returned %d: %s\n", #call, r_, pw_last_error());      \
            return 2;                                                                     \
        }                                                                                 \
    } while (0)

enum { NF = 12 };   /* u v w lu lv lw | su sv sw | gu gv gw */

int main(int argc, char **argv)
{
    int nx = 19, ny = 13, nz = 64, h = 2, f, i, j, k, bad = 0;
    if (argc == 5) {
        nx = atoi(argv[1]);
        ny = atoi(argv[2]);
        nz = atoi(argv[3]);
        h = atoi(argv[4]);
    }
    if (nx < 1 || ny < 1 || nz < 2 || h < 1) {
        printf("pw_c_caller: bad shape\n");
        return 2;
    }
    const size_t sy = (size_t)(nz + 2 * h), sx = (size_t)(ny + 2 * h) * sy;
    const size_t n = (size_t)(nx + 2 * h) * sx, bytes = n * sizeof(double);
    double *d[NF], *hst[NF], *ref[3], *dt1, *dt2;
    double *t1 = malloc((size_t)nz * sizeof(double)), *t2 = malloc((size_t)nz * sizeof(double));
    const double tcx = -0.005, tcy = -0.004;
    if (!t1 || !t2) return 2;
    for (k = 0; k < nz; k++) {          /* any coefficient profile: both sides get the same */
        t1[k] = 0.5 / (1.0 + k);
        t2[k] = 0.25 / (2.0 + k);
    }
    for (f = 0; f < NF; f++) {
        HIP_OK(hipMalloc((void **)&d[f], bytes));
        HIP_OK(hipMemset(d[f], 0, bytes));
        hst[f] = malloc(bytes);
        if (!hst[f]) return 2;
    }
    for (f = 0; f < 3; f++) {
        ref[f] = calloc(n, sizeof(double));
        if (!ref[f]) return 2;
    }
    HIP_OK(hipMalloc((void **)&dt1, (size_t)nz * sizeof(double)));
    HIP_OK(hipMalloc((void **)&dt2, (size_t)nz * sizeof(double)));
    HIP_OK(hipMemcpy(dt1, t1, (size_t)nz * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dt2, t2, (size_t)nz * sizeof(double), hipMemcpyHostToDevice));

    /* inputs: winds of amplitude 10 (w zero at the lids), multipliers of amplitude 1 */
    for (f = 0; f < 6; f++) {
        PW_OK_(pw_fill_uniform(d[f], nx, ny, nz, h, 7ULL, f, f < 3 ? 10.0 : 1.0, f == 2, PW_F64, NULL));
        PW_OK_(pw_halo_periodic(d[f], nx, ny, nz, h, PW_F64, NULL));
    }
    /* the forward alone into gu, gv, gw's arrays (compared below), then the fused pass */
    PW_OK_(pw_advect_fwd(d[0], d[1], d[2], dt1, dt2, tcx, tcy, nx, ny, nz, h, d[9], d[10], d[11], PW_F64, NULL));
    HIP_OK(hipDeviceSynchronize());
    for (f = 9; f < 12; f++) HIP_OK(hipMemcpy(hst[f - 3], d[f], bytes, hipMemcpyDeviceToHost));
    for (f = 0; f < 3; f++) memcpy(ref[f], hst[6 + f], bytes);     /* hold the forward's su, sv, sw */
    PW_OK_(pw_advect_fwd_adj(d[0], d[1], d[2], d[3], d[4], d[5], dt1, dt2, tcx, tcy, nx, ny, nz, h, d[6], d[7],
                             d[8], d[9], d[10], d[11], PW_F64, NULL));
    HIP_OK(hipDeviceSynchronize());
    for (f = 0; f < NF; f++) HIP_OK(hipMemcpy(hst[f], d[f], bytes, hipMemcpyDeviceToHost));

    /* the forward of both calls against the oracle, bit for bit */
    double *os = malloc(3 * bytes), *og = malloc(3 * bytes);
    if (!os || !og) return 2;
    memset(os, 0, 3 * bytes);
    pw_oracle_fwd(hst[0], hst[1], hst[2], t1, t2, tcx, tcy, nx, ny, nz, h, os, os + n, os + 2 * n);
    pw_oracle_adj(hst[0], hst[1], hst[2], hst[3], hst[4], hst[5], t1, t2, tcx, tcy, nx, ny, nz, h, og, og + n,
                  og + 2 * n);
    for (f = 0; f < 3; f++)
        for (i = 0; i < nx; i++)
            for (j = 0; j < ny; j++)
                for (k = 0; k < nz; k++) {
                    const size_t c = (size_t)(i + h) * sx + (size_t)(j + h) * sy + (size_t)(k + h);
                    const double o = os[(size_t)f * n + c];
                    if (memcmp(&o, &hst[6 + f][c], sizeof o) || memcmp(&o, &ref[f][c], sizeof o)) {
                        if (bad < 5)
                            printf("forward field %d cell (%d,%d,%d): fused %.17g, fwd %.17g, oracle %.17g\n", f, i, j,
                                   k, hst[6 + f][c], ref[f][c], o);
                        bad++;
                    }
                }
    /* the adjoint, normwise */
    double worst = 0.0;
    for (f = 0; f < 3; f++) {
        double dmax = 0.0, rmax = 0.0;
        for (i = 0; i < nx; i++)
            for (j = 0; j < ny; j++)
                for (k = 0; k < nz; k++) {
                    const size_t c = (size_t)(i + h) * sx + (size_t)(j + h) * sy + (size_t)(k + h);
                    const double r = og[(size_t)f * n + c], g = hst[9 + f][c];
                    if (fabs(g - r) > dmax || g != g) dmax = g != g ? INFINITY : fabs(g - r);
                    if (fabs(r) > rmax) rmax = fabs(r);
                }
        const double rel = rmax > 0.0 ? dmax / rmax : dmax;
        if (rel > worst) worst = rel;
        if (!(rel <= 1e-12)) {
            printf("adjoint field %d: normwise difference %.3g\n", f, rel);
            bad++;
        }
    }
    for (f = 0; f < NF; f++) {
        HIP_OK(hipFree(d[f]));
        free(hst[f]);
    }
    for (f = 0; f < 3; f++) free(ref[f]);
    HIP_OK(hipFree(dt1));
    HIP_OK(hipFree(dt2));
    free(os);
    free(og);
    free(t1);
    free(t2);
    if (bad) {
        printf("pw_c_caller: %d mismatches at %dx%dx%d halo %d\n", bad, nx, ny, nz, h);
        return 1;
    }
    printf("pw_c_caller ok: %dx%dx%d halo %d, forward bitwise, adjoint within %.2g normwise (library version %d)\n",
           nx, ny, nz, h, worst, pw_version());
    return 0;
}
