"""The double-precision deposit computes R = sqrt(|d|^2) with its own sequence
(canon_sqrt in radio_kernels.hip): a reciprocal-square-root seed, one coupled
Goldschmidt step and two residual corrections, each step one fused multiply-add.
Arrival times must match the oracle bit for bit, so R must be the correctly
rounded square root.  This test replays the same steps on the CPU with C's fma,
seeding them with 1/sqrt(x) cut to 23 bits and perturbed by up to 1e-6 (the
hardware seed is good to about 2^-22), and checks every result against the
correctly rounded sqrt: random magnitudes, rounded squares of random values, and
the doubles next to exact squares, for x = 0 and 2^-767 <= x < inf, plus the
reciprocal it returns beside R to within two ulps."""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static uint64_t s = 88172645463325252ull;
static uint64_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double unif(void) { return (rnd() >> 11) * (1.0 / 9007199254740992.0); }
static double seed(double x, double maxerr) {
    double y = 1.0 / sqrt(x);
    uint64_t b;
    memcpy(&b, &y, 8);
    b &= ~((1ull << 29) - 1);
    memcpy(&y, &b, 8);
    return y * (1.0 + maxerr * (2.0 * unif() - 1.0));
}
static double steps(double x, double y, double* rinv) {
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    double q = 2.0 * h;
    *rinv = fma(q, fma(-g, q, 1.0), q);
    return x == 0.0 ? 0.0 : g;
}
int main(void) {
    const double errs[] = {1e-9, 2.4e-7, 1e-6};
    long bad = 0, n = 0;
    double worst = 0.0;
    for (int e = 0; e < 3; ++e) {
        for (long i = 0; i < 700000; ++i) {
            double x;
            if (i % 3 == 0) {
                x = ldexp(1.0 + unif(), (int)(rnd() % 1500) - 750);
            } else if (i % 3 == 1) {
                const double a = ldexp(1.0 + unif(), (int)(rnd() % 80) - 40);
                x = a * a;
            } else {
                const double a = floor(unif() * 1e7) + 1.0;
                x = nextafter(a * a, (rnd() & 1) ? 0.0 : INFINITY);
            }
            if (x < ldexp(1.0, -767))
                continue;
            double ri;
            const double g = steps(x, seed(x, errs[e]), &ri);
            const double ref = sqrt(x);
            ++n;
            if (g != ref)
                ++bad;
            const double rel = fabs(ri * ref - 1.0);
            if (rel > worst)
                worst = rel;
        }
    }
    double ri0;
    const double z = steps(0.0, INFINITY, &ri0);
    printf("%ld %ld %.3e %.17g\n", n, bad, worst, z);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_sqrt_steps_round_correctly(tmp_path):
    src = tmp_path / "steps.c"
    exe = tmp_path / "steps"
    src.write_text(SRC)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True,
                         env=dict(os.environ, LC_ALL="C")).stdout.split()
    n, bad, worst, zero = int(out[0]), int(out[1]), float(out[2]), float(out[3])
    assert n > 1_500_000
    assert bad == 0
    assert worst <= 2.3e-16  # 1/R within about two ulps
    assert zero == 0.0
