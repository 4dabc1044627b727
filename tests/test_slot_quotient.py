"""The double-precision deposit forms the slot coordinate (t_det - t0) / dt_det
without a division per state (canon_slot in radio_kernels.hip): from the host's
correctly rounded reciprocal y = RN(1/dt_det) it takes q0 = x y and two
residual corrections q <- q + (x - dt_det q) y, each one fused multiply-add.
Slot coordinates decide which slots a segment covers and its overlaps, so they
must be the correctly rounded quotient the oracle's division gives.  The
argument for the two corrections holds for divisors that pass a host check
(|dt_det y - 1| B < 1 - 2^-45, B the divisor's integer significand); the
library divides for the others.

This test replays the steps on the CPU with C's fma and checks every result
against the division: random divisors and numerators over wide ranges,
numerators built to put the quotient within an ulp of a rounding midpoint (the
hard cases), and divisors whose significand is all ones or nearly so (where the
check is tight).  It also checks that the host check rejects only divisors with
a significand within 64 units of the next power of two.
"""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double unif(void) { return (rnd() >> 11) * (1.0 / 9007199254740992.0); }
/* the host check of the library */
static int corrects(double b) {
    if (!(b >= 0x1p-900 && b <= 0x1p900)) return 0;
    const double y = 1.0 / b;
    const double e = fma(b, y, -1.0);
    int ex;
    const double B = ldexp(frexp(b, &ex), 53);
    return fabs(e) * B < 1.0 - 0x1p-45;
}
/* the kernel's steps */
static double quotient(double x, double b, double y) {
    double q = x * y;
    double r = fma(-q, b, x);
    q = fma(r, y, q);
    r = fma(-q, b, x);
    return fma(r, y, q);
}
static double rand_divisor(int kind) {
    if (kind == 0)                      /* any significand, wide exponent */
        return ldexp(1.0 + unif(), (int)(rnd() % 120) - 60);
    if (kind == 1) {                    /* significand within 4096 units of 2 */
        uint64_t bits = 0x3FFFFFFFFFFFFFFFull - (rnd() % 4096);
        double b;
        memcpy(&b, &bits, 8);
        return ldexp(b, (int)(rnd() % 40) - 20);
    }
    /* slot widths of the workloads: 1e-6 .. 1 */
    return pow(10.0, -6.0 * unif());
}
int main(void) {
    long n = 0, bad = 0, rejected = 0, rejected_far = 0, divisors = 0;
    for (int kind = 0; kind < 3; ++kind) {
        for (int i = 0; i < 3000; ++i) {
            const double b = rand_divisor(kind);
            ++divisors;
            if (!corrects(b)) {
                ++rejected;
                int ex;
                const double B = ldexp(frexp(b, &ex), 53);
                if (B < 0x1p53 - 64.0) ++rejected_far;
                continue;
            }
            const double y = 1.0 / b;
            for (int j = 0; j < 400; ++j) {
                double x;
                const int m = j % 4;
                if (m == 0) {                       /* any numerator */
                    x = ldexp(1.0 + unif(), (int)(rnd() % 200) - 100);
                } else if (m == 1) {                /* times of the workloads */
                    x = (unif() - 0.25) * 2e5;
                } else {                            /* quotient next to a midpoint */
                    const double q = ldexp(1.0 + unif(), (int)(rnd() % 80) - 40);
                    const double h = 0.5 * (nextafter(q, INFINITY) - q);
                    x = fma(b, q, b * h);           /* RN(b (q + h)) */
                    if (m == 3) {
                        const int k = (int)(rnd() % 5) - 2;
                        for (int t = 0; t < k; ++t) x = nextafter(x, INFINITY);
                        for (int t = 0; t > k; --t) x = nextafter(x, -INFINITY);
                    }
                }
                if (rnd() & 1) x = -x;
                ++n;
                if (quotient(x, b, y) != x / b) ++bad;
            }
            /* exact quotients and zero */
            const double q = ldexp(1.0 + unif(), (int)(rnd() % 60) - 30);
            const double xq = b * q;
            ++n;
            if (quotient(xq, b, y) != xq / b) ++bad;
            ++n;
            if (quotient(0.0, b, y) != 0.0) ++bad;
        }
    }
    /* every divisor of an all-ones significand and its neighbours */
    for (int e = -30; e <= 30; ++e) {
        for (int k = 0; k < 80; ++k) {
            uint64_t bits = 0x3FFFFFFFFFFFFFFFull - (uint64_t)k;
            double b;
            memcpy(&b, &bits, 8);
            b = ldexp(b, e);
            ++divisors;
            if (!corrects(b)) { ++rejected; continue; }
            const double y = 1.0 / b;
            for (int j = 0; j < 200; ++j) {
                const double q = ldexp(1.0 + unif(), (int)(rnd() % 80) - 40);
                const double h = 0.5 * (nextafter(q, INFINITY) - q);
                double x = fma(b, q, b * h);
                if (j & 1) x = nextafter(x, (j & 2) ? INFINITY : -INFINITY);
                ++n;
                if (quotient(x, b, y) != x / b) ++bad;
            }
        }
    }
    printf("%ld %ld %ld %ld %ld\n", n, bad, divisors, rejected, rejected_far);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_slot_quotient_steps_round_correctly(tmp_path):
    src = tmp_path / "quotient.c"
    exe = tmp_path / "quotient"
    src.write_text(SRC)
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-o", str(exe), str(src),
                    "-lm"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True,
                         env=dict(os.environ, LC_ALL="C")).stdout.split()
    n, bad, divisors, rejected, rejected_far = (int(v) for v in out)
    print(f"{n} quotients over {divisors} divisors, {rejected} divisors sent to division")
    assert n > 3_000_000
    assert bad == 0
    # only significands next to the power of two above fail the check
    assert rejected_far == 0
    assert 0 < rejected < 0.05 * divisors
