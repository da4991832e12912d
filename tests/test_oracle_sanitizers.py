"""The FP64 oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
a host-only build of oracle/lbref.c (gcc, no OpenMP) steps a droplet with periodic
and wall boundaries, both interaction stencils and both collision forms, and calls
the moment, stream and one-site collision entry points at the lattice corners; any
out-of-bounds access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HARNESS = r"""
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <math.h>
#include "lbref.c"
int main(void)
{
    for (int bc = 0; bc < 2; ++bc)
        for (int st = 0; st < 2; ++st)
            for (int form = 0; form < 2; ++form) {
                lbref_params p = {0};
                p.nx = 37; p.ny = 29; p.bc = bc; p.a = 0.5; p.b = 4.0; p.R = 1.0; p.T = 0.6 * 0.047;
                p.G = -1.0; p.sigma = 0.11; p.s_rho = 1.0; p.s_e = 1.1; p.s_zeta = 1.1; p.s_j = 1.0;
                p.s_q = 1.1; p.nu_l = 0.1; p.nu_g = 0.3; p.rho_switch = 0.13045; p.stencil = st;
                const int n = p.nx * p.ny;
                double *rho = malloc(sizeof(double) * n), *f = malloc(sizeof(double) * 9 * n);
                double *w = malloc(sizeof(double) * 9 * n), *o[7];
                for (int k = 0; k < 7; ++k) o[k] = malloc(sizeof(double) * 9 * n);
                for (int y = 0; y < p.ny; ++y)
                    for (int x = 0; x < p.nx; ++x) {
                        const double d = sqrt((x - 18.0) * (x - 18.0) + (y - 14.0) * (y - 14.0));
                        rho[y * p.nx + x] = 0.205 - 0.202 * tanh(2.0 * (d - 8.0) / 5.0);
                    }
                int64_t done = 0, sites[5] = {0, 1, p.nx - 1, (int64_t)p.nx * (p.ny - 1), (int64_t)n - 1};
                double out[45];
                int s = lbref_init(&p, rho, NULL, NULL, f);
                s = s ? s : lbref_step(&p, f, w, 20, form, &done);
                s = s ? s : lbref_moments(&p, f, o[0], o[1], o[2], o[3], o[4], o[5]);
                s = s ? s : lbref_stream(&p, f, o[6]);
                s = s ? s : lbref_collide_at(&p, f, 5, sites, out);
                printf("%d %d %d %d %lld\n", bc, st, form, s, (long long)done);
                free(rho); free(f); free(w);
                for (int k = 0; k < 7; ++k) free(o[k]);
                if (s || done != 20) return 1;
            }
    return 0;
}
"""


def test_oracle_is_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "harness.c"
    src.write_text(HARNESS)
    exe = tmp_path / "harness"
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), str(src), "-o", str(exe), "-lm"],
                   check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert len(r.stdout.split("\n")) >= 8
