"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

A small C driver links pw_oracle.c built with -fsanitize=address,undefined
and runs every entry point on exactly sized heap arrays for shapes at the
edges of the contract (halo 1, nz = 2, one-plane and one-column grids), so an
access outside a storage array or an undefined operation aborts the driver.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "pw_oracle.c")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>

void pw_oracle_fwd(const double*, const double*, const double*, const double*, const double*, double, double,
                   int, int, int, int, double*, double*, double*);
void pw_oracle_fwd_abs(const double*, const double*, const double*, const double*, const double*, double, double,
                       int, int, int, int, double*, double*, double*);
void pw_oracle_adj(const double*, const double*, const double*, const double*, const double*, const double*,
                   const double*, const double*, double, double, int, int, int, int, double*, double*, double*);
void pw_oracle_adj_abs(const double*, const double*, const double*, const double*, const double*, const double*,
                       const double*, const double*, double, double, int, int, int, int, double*, double*, double*);
void pw_oracle_fold_periodic(double*, int, int, int, int);

static double* field(size_t n, unsigned* seed)
{
    double* a = malloc(n * sizeof(double));
    for (size_t q = 0; q < n; q++) {
        *seed = *seed * 1103515245u + 12345u;
        a[q] = ((double)(*seed >> 8) / 16777216.0) * 20.0 - 10.0;
    }
    return a;
}

int main(void)
{
    const int shapes[][4] = {{1, 1, 2, 1}, {3, 2, 2, 1}, {1, 5, 3, 2}, {4, 1, 5, 1}, {5, 4, 7, 3}, {2, 3, 64, 2}};
    unsigned seed = 7;
    for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; s++) {
        const int nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2], h = shapes[s][3];
        const size_t n = (size_t)(nx + 2 * h) * (size_t)(ny + 2 * h) * (size_t)(nz + 2 * h);
        double *u = field(n, &seed), *v = field(n, &seed), *w = field(n, &seed);
        double *lu = field(n, &seed), *lv = field(n, &seed), *lw = field(n, &seed);
        double *t1 = field((size_t)nz, &seed), *t2 = field((size_t)nz, &seed);
        double *o[6];
        for (int q = 0; q < 6; q++) o[q] = field(n, &seed);
        pw_oracle_fwd(u, v, w, t1, t2, -0.005, -0.005, nx, ny, nz, h, o[0], o[1], o[2]);
        pw_oracle_fwd_abs(u, v, w, t1, t2, -0.005, -0.005, nx, ny, nz, h, o[3], o[4], o[5]);
        pw_oracle_adj(u, v, w, lu, lv, lw, t1, t2, -0.005, -0.005, nx, ny, nz, h, o[0], o[1], o[2]);
        pw_oracle_adj_abs(u, v, w, lu, lv, lw, t1, t2, -0.005, -0.005, nx, ny, nz, h, o[3], o[4], o[5]);
        pw_oracle_fold_periodic(o[0], nx, ny, nz, h);
        double acc = 0;
        for (int q = 0; q < 6; q++) {
            for (size_t k = 0; k < n; k++) acc += o[q][k];
            free(o[q]);
        }
        free(u); free(v); free(w); free(lu); free(lv); free(lw); free(t1); free(t2);
        printf("shape %d %d %d h%d ok %g\n", nx, ny, nz, h, acc);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_ubsan(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", str(drv), SRC, "-o", str(exe), "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok ") == 6
