"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host only) and driven through its C entry points over short runs: both
coupling schemes, the contact force, a rigid particle and the open channel.
Any out-of-bounds access, use after free, leak or undefined operation fails
the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "lbib_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include "lbib_oracle.c"

static void circle(double cx, double cy, double r, int n, double *xy)
{
    for (int k = 0; k < n; k++) {
        const double a = 2.0 * M_PI * (k + 0.5) / n;
        xy[2 * k] = cx + r * cos(a);
        xy[2 * k + 1] = cy + r * sin(a);
    }
}

static int run(orc_sim *s, int steps, int mode, const char *name)
{
    if (!s) { printf("%s: create failed\n", name); return 1; }
    if (orc_step(s, steps, mode) != 0) { printf("%s: step refused\n", name); return 1; }
    const int nx = s->nx, ny = s->ny;
    double *f = malloc(sizeof(double) * 9 * nx * ny), *m = malloc(sizeof(double) * 3 * nx * ny);
    double *F = malloc(sizeof(double) * 2 * nx * ny);
    orc_get_pops(s, f);
    orc_set_pops(s, f);
    orc_get_moments(s, m);
    orc_get_force(s, F);
    for (int c = 0; c < orc_num_capsules(s); c++) {
        const int nv = orc_capsule_nodes(s, c);
        double *x = malloc(sizeof(double) * 6 * nv), d[13];
        orc_get_capsule(s, c, x, x + 2 * nv, x + 4 * nv);
        orc_get_diag(s, c, d);
        free(x);
    }
    const int st = orc_status(s);
    free(f); free(m); free(F);
    orc_destroy(s);
    printf("%s: status %d\n", name, st);
    return st != 0;
}

int main(void)
{
    int bad = 0;
    double a[2 * 40], b[2 * 40], ks[40];
    for (int k = 0; k < 40; k++) ks[k] = 0.02;
    for (int mode = 0; mode < 2; mode++) {
        orc_sim *s = orc_create(70, 45, 0.8, 0, -0.01, 0.01, 1e-6, 0.0, 1, 0.0, 0.0, 1, 0.0, 1.0);
        circle(30.0, 22.0, 6.0, 40, a);
        orc_add_capsule(s, 40, a, ks, 40, mode ? 0.0 : 0.002, 1.0, 113.0);
        bad |= run(s, 30, mode, mode ? "channel dynamic" : "channel kinematic");
    }
    {   /* two capsules in contact range and a rigid disc, Dynamic */
        orc_sim *s = orc_create(80, 50, 0.9, 0, 0.0, 0.0, 2e-6, 0.0, 2, 0.0, 0.0, 1, 0.0, 1.0);
        circle(25.0, 25.0, 6.0, 40, a);
        circle(38.6, 25.0, 6.0, 40, b);
        orc_add_capsule(s, 40, a, ks, 1, 0.0, 1.0, 113.0);
        orc_add_capsule(s, 40, b, ks, 1, 0.0, 1.0, 113.0);
        circle(60.0, 20.0, 5.0, 32, a);
        orc_add_rigid(s, 32, a, 78.0, 975.0);
        orc_set_contact(s, 2.0);
        bad |= run(s, 25, 1, "contact and rigid");
    }
    {   /* open channel: velocity inlet, pressure outlet */
        orc_sim *s = orc_create(90, 40, 0.8, 0, 0.0, 0.0, 0.0, 0.0, 4, 0.0, 0.0, 0, 0.02, 1.0);
        circle(40.0, 20.0, 6.0, 40, a);
        orc_add_capsule(s, 40, a, ks, 1, 0.0, 1.0, 113.0);
        bad |= run(s, 25, 1, "open channel");
    }
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-Wno-unknown-pragmas",
                           "-I", os.path.dirname(ORACLE), "-o", str(exe), str(src), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ERROR" not in r.stderr and "runtime error" not in r.stderr, r.stderr
