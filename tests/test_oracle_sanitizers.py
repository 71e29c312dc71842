"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) runs its step in every mode on a small system without a
report: fixed steps with direct gravity, the static host with the reflecting
sphere, block time steps and tree gravity; plus the tree force on its own and
the event search with an event buffer too small (the capacity path).  The
test program builds its inputs with a fixed linear congruential generator (inputs
only, no arithmetic of the method)."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "sidm_oracle.h"

static uint64_t lcg = 12345u;
static double uni(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int run(int mode)
{
    const int64_t n = 700;
    double *buf = calloc((size_t)n * 13, sizeof(double));
    double *x = buf, *y = x + n, *z = y + n, *vx = z + n, *vy = vx + n, *vz = vy + n;
    double *m = vz + n, *ax = m + n, *ay = ax + n, *az = ay + n, *pot = az + n, *h = pot + n;
    uint32_t *id = malloc(sizeof(uint32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        x[i] = uni() - 0.5; y[i] = uni() - 0.5; z[i] = uni() - 0.5;
        vx[i] = uni() - 0.5; vy[i] = uni() - 0.5; vz[i] = uni() - 0.5;
        m[i] = 1.0 / (double)n;
        id[i] = (uint32_t)(3 * i + 1);
    }
    orc_params p;
    memset(&p, 0, sizeof p);
    p.G = 1.0; p.eps = 0.02; p.sigma_m = 200.0; p.dt = 2e-3; p.k = 16; p.seed = 7;
    if (mode == 1) {
        p.host_kind = 1; p.host_rho_s = 1.0; p.host_r_s = 2.0;
        p.boundary_r = 0.45;
    }
    if (mode == 2) { p.eta = 0.025; p.max_bin = 3; p.dt = 1.0 / 64; p.dt_min = 1.0 / 256; }
    if (mode == 3) { p.tree_alpha = 5e-4; p.eta = 0.025; p.max_bin = 2; p.dt = 1.0 / 64; }
    orc_gravity(n, x, y, z, m, 1.0, p.eps, n, NULL, ax, ay, az, pot, NULL);
    const int64_t cap = 1 << 16;
    orc_event *ev = malloc(sizeof(orc_event) * (size_t)cap);
    int64_t total = 0;
    for (uint32_t s = 0; s < 3; ++s) {
        const int64_t k = orc_kdk_step(n, x, y, z, vx, vy, vz, m, id, ax, ay, az, pot, h, &p, s,
                                       ev, cap);
        if (k < 0) return 10 + mode;
        total += k;
    }
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i] + vx[i] + ax[i] + pot[i] + h[i])) return 20 + mode;
    if (mode == 0) {
        /* the event search with a buffer of one: reports the count it needed */
        int64_t pairs = 0, pg = 0;
        const int64_t need = orc_find_events(n, x, y, z, vx, vy, vz, m, id, h, p.sigma_m, 0.0,
                                             p.dt, p.seed, 9, NULL, ev, 1, &pairs, &pg);
        if (need < 0 || pairs <= 0) return 30;
        int64_t terms = 0;
        /* previous accelerations in, forces out into the (no longer needed) velocities */
        orc_tree_gravity(n, x, y, z, m, ax, ay, az, 1.0, p.eps, 5e-4, n, NULL, vx, vy, vz, pot,
                         &terms);
        if (terms <= 0) return 31;
    }
    printf("mode %d: %lld events\n", mode, (long long)total);
    free(ev); free(id); free(buf);
    return 0;
}

int main(void)
{
    for (int mode = 0; mode < 4; ++mode) {
        const int r = run(mode);
        if (r) return r;
    }
    puts("ok");
    return 0;
}
'''


def test_oracle_under_sanitizers():
    d = tempfile.mkdtemp(prefix="orc_san_")
    drv = os.path.join(d, "drv.c")
    exe = os.path.join(d, "drv")
    with open(drv, "w") as f:
        f.write(_DRIVER)
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "oracle"), drv, os.path.join(ROOT, "oracle", "sidm_oracle.c"),
           "-o", exe, "-lm"]
    try:
        subprocess.run(cmd, check=True, capture_output=True, text=True)
    except (OSError, subprocess.CalledProcessError) as e:  # pragma: no cover
        pytest.skip(f"no sanitizer build here: {e}")
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr
    assert "AddressSanitizer" not in r.stderr
    assert r.stdout.strip().endswith("ok")
