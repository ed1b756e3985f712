"""Host sanitizers on the C oracle (CPU): fd6_oracle.c built by gcc with
AddressSanitizer and UndefinedBehaviorSanitizer (halting on the first report)
and driven by a small C program through every entry point -- ghost fill and
the operators on ragged boxes at the 6-cell minimum, both methods' steps and
right-hand sides, the force, the patch update at its minimum half-width, and
the reductions with non-finite values.  Any out-of-bounds access, use of
freed memory, leak or undefined arithmetic fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fd6_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
int orc_rk3(int, int, int, double*, double*, double*, double*, double, double, double, double,
            double, double, int, int, int);
int orc_rhs(int, int, int, const double*, const double*, const double*, const double*, double,
            double, double, double, double, int, double*, double*, double*, double*, int);
int orc_rk3_patch(int, const double*, const double*, const double*, const double*, double,
                  double, double, double, double, double, int, int, const double*,
                  const double*, const double*, double*);
int orc_reduce(int, int, int, const double*, const double*, const double*, const double*,
               double, double, double, double*);
void orc_fill_ghosts(int, int, int, double*);
int orc_apply_op_ghosted(int, int, int, const double*, int, double, double, double, double*);
int orc_set_forcing(const double*);

static double* field(size_t n, unsigned seed) {
    double* f = (double*)malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) f[i] = 1e-3 * sin(0.37 * (double)(i + 1) * (seed + 1));
    return f;
}

int main(void) {
    const int shapes[][3] = {{6, 6, 6}, {7, 9, 8}, {13, 6, 11}};
    for (int s = 0; s < 3; ++s) {
        const int nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
        const size_t n = (size_t)nx * ny * nz;
        const size_t ng = (size_t)(nx + 6) * (ny + 6) * (nz + 6);
        double* g = field(ng, 9);
        orc_fill_ghosts(nx, ny, nz, g);
        double* o = (double*)malloc(n * sizeof(double));
        for (int op = 0; op < 9; ++op)
            if (orc_apply_op_ghosted(nx, ny, nz, g, op, 0.1, 0.2, 0.3, o)) return 1;
        for (int v = 0; v < 2; ++v)
            for (int frc = 0; frc < 2; ++frc) {
                const double fin[10] = {1.0, 2.0, 0.0, 0.0, 0.0, 1.0, 0.02, 0.3, 1.0, 0.01};
                orc_set_forcing(frc ? fin : NULL);
                double *a = field(n, 1), *b = field(n, 2), *c = field(n, 3), *d = field(n, 4);
                if (orc_rk3(nx, ny, nz, a, b, c, d, 5e-3, 1.0, 0.1, 0.2, 0.3, 0.01, v, 2, 2))
                    return 2;
                double *r0 = field(n, 5), *r1 = field(n, 6), *r2 = field(n, 7), *r3 = field(n, 8);
                if (orc_rhs(nx, ny, nz, a, b, c, d, 5e-3, 1.0, 0.1, 0.2, 0.3, v, r0, r1, r2, r3, 1))
                    return 3;
                double red[5];
                b[0] = NAN;
                c[n - 1] = INFINITY;
                if (orc_reduce(nx, ny, nz, a, b, c, d, 0.1, 0.2, 0.3, red) || red[4] != 2.0)
                    return 4;
                free(a); free(b); free(c); free(d);
                free(r0); free(r1); free(r2); free(r3);
            }
        orc_set_forcing(NULL);
        free(g);
        free(o);
    }
    for (int v = 0; v < 2; ++v) {
        const int m = (v == 0 ? 9 : 18), w = 2 * m + 1;
        const size_t nn = (size_t)w * w * w;
        double *a = field(nn, 1), *b = field(nn, 2), *c = field(nn, 3), *d = field(nn, 4);
        double* px = (double*)malloc(w * sizeof(double));
        for (int i = 0; i < w; ++i) px[i] = 0.1 * i;
        double out[4];
        if (orc_rk3_patch(m, a, b, c, d, 5e-3, 1.0, 0.1, 0.1, 0.1, 0.01, v, 1, px, px, px, out))
            return 5;
        if (orc_rk3_patch(m - 1, a, b, c, d, 5e-3, 1.0, 0.1, 0.1, 0.1, 0.01, v, 1, px, px, px,
                          out) != -1)
            return 6;  /* too small a patch is refused */
        free(a); free(b); free(c); free(d); free(px);
    }
    puts("clean");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    flags = ["-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp"]
    r = subprocess.run(["gcc", *flags, str(drv), SRC, "-o", str(exe), "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0 and out.stdout.strip() == "clean", out.stdout + out.stderr
