"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

1. The oracle (oracle/radio_oracle.c), built with gcc -fsanitize=address,undefined
   and driven by a small C program through every option, clipped and
   non-monotone segments, empty chunks, NaN and infinite inputs and invalid
   arguments.
2. The library's host code (paper_2302_14812_amd/csrc), its host pass built by
   hipcc with the sanitizers (device code is not instrumented), driven through
   the C interface's argument checks, the detector-geometry builders and the
   tuning calls.  There is no GPU here, so calls that pass validation stop at
   the first device call (RADIO_EDEVICE) -- which is the point: everything
   before it is host validation.

Any sanitizer report aborts the program (halt_on_error, no recovery), and the
test checks the exit status and the program's own summary line.
"""
import os
import shutil
import subprocess

import pytest

from paper_2302_14812_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", LC_ALL="C")

ORACLE_DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
int radio_oracle_deposit(const double*, int64_t, double, double, int64_t, double, int64_t,
                         int64_t, double, int64_t, double, const double*, const double*,
                         const double*, int, double*, int64_t*, int);
void radio_oracle_field_opts(const double*, const double*, const double*, double,
                             const double*, double, double, int, double*, double*);
double radio_oracle_arrival(const double*, const double*, double, double);
double radio_oracle_arrival_far(const double*, const double*, double, double);
double radio_oracle_slot_of(double, double, double);
static uint64_t st = 7;
static double rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (st >> 11) * 0x1p-53; }
int main(void) {
    const int np = 5, ns = 40, nc = 6, nt = 50;
    double* x = malloc(sizeof(double) * 3 * (ns + 1) * np);
    double* u = malloc(sizeof(double) * 3 * (ns + 1) * np);
    double q[5] = {-1, 1, -2, 0.5, -1};
    double cells[18];
    for (int c = 0; c < nc; ++c) {
        cells[3 * c] = 10.0 * rnd() - 5; cells[3 * c + 1] = 10.0 * rnd() - 5; cells[3 * c + 2] = 40.0;
    }
    for (int k = 0; k < 3; ++k)
        for (int s = 0; s <= ns; ++s)
            for (int p = 0; p < np; ++p) {
                const int i = (k * (ns + 1) + s) * np + p;
                u[i] = (k == 2 ? 3.0 : 0.5) * sin(0.3 * s + p + k);
                /* particle 4 jumps faster than light at step 20: a backward segment */
                x[i] = 0.05 * s * (k == 2) + 0.3 * p + ((p == 4 && s >= 20) ? -3.0 * (k == 2) : 0.0);
            }
    double* D = calloc((size_t)nc * nt * 6, sizeof(double));
    int64_t cnt[2] = {0, 0};
    int bad = 0;
    const int opts[] = {0, 1, 2, 3, 4, 5, 8, 9, 10, 16, 17, 20, 24};
    for (unsigned o = 0; o < sizeof(opts) / sizeof(opts[0]); ++o) {
        /* window cutting both ends of the arrivals */
        bad |= radio_oracle_deposit(cells, nc, 40.5, 0.03, nt, 1.0, np, ns, 0.0, 3, 0.05, x, u,
                                    (o & 1) ? q : NULL, opts[o], D, cnt, 2) != 0;
    }
    bad |= radio_oracle_deposit(cells, nc, 40.5, 0.03, nt, 1.0, 0, ns, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != 0;
    bad |= radio_oracle_deposit(cells, nc, 40.5, 0.03, nt, 1.0, np, 0, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != 0;
    bad |= radio_oracle_deposit(cells, -1, 40.5, 0.03, nt, 1.0, np, ns, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != -1;
    bad |= radio_oracle_deposit(cells, nc, 40.5, 0.0, nt, 1.0, np, ns, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != -1;
    bad |= radio_oracle_deposit(NULL, nc, 40.5, 0.03, nt, 1.0, np, ns, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != -1;
    /* NaN and infinite positions deposit non-finite values or nothing, in bounds */
    x[7] = NAN;
    x[11] = INFINITY;
    bad |= radio_oracle_deposit(cells, nc, 40.5, 0.03, nt, 1.0, np, ns, 0.0, 0, 0.05, x, u, q, 0, D, cnt, 1) != 0;
    double E[3], B[3], beta[3] = {0.1, 0.2, 0.3}, bd[3] = {1, 0, 0}, xp[3] = {0, 0, 0};
    radio_oracle_field_opts(cells, xp, beta, 0.86, bd, -1.0, 1.0, 0, E, B);
    radio_oracle_field_opts(cells, cells, beta, 0.86, bd, -1.0, 1.0, 0, E, B); /* R = 0 */
    double t = radio_oracle_arrival(cells, xp, 1.0, 1.0) + radio_oracle_arrival_far(cells, xp, 1.0, 1.0);
    t += radio_oracle_slot_of(t, 1.0, 0.01);
    printf("oracle ok bad=%d clipped=%lld back=%lld t=%d\n", bad, (long long)cnt[0],
           (long long)cnt[1], isfinite(t));
    free(x); free(u); free(D);
    return bad;
}
"""

RUNTIME_DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "radio.h"
static int fails = 0;
#define EXPECT(call, want) do { int r_ = (call); if (r_ != (want)) { \
    printf("unexpected %d from %s (want %d)\n", r_, #call, (want)); ++fails; } } while (0)
int main(void) {
    radio_detector* h = NULL;
    radio_detector_desc d;
    memset(&d, 0, sizeof d);
    d.geometry = RADIO_GEOM_PLANE;
    d.n1 = 7; d.n2 = 5; d.e1[0] = 1; d.e2[1] = 1; d.half1 = 2; d.half2 = 3;
    d.origin[2] = 100; d.t0 = 90; d.dt_det = 0.1; d.n_t = 64; d.c = 1;
    EXPECT(radio_detector_create(NULL, NULL, &h), RADIO_EINVAL);
    d.dt_det = 0; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.dt_det = 0.1;
    d.dt_det = 1e-310; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.dt_det = 0.1;
    d.n_t = 0; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.n_t = 64;
    d.c = NAN; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.c = 1;
    d.precision = 3; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.precision = 1;
    d.options = RADIO_HOLD_PREVIOUS | RADIO_HOLD_LINEAR;
    EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    d.options = RADIO_POTENTIALS | RADIO_ACCEL_ONLY;
    EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    d.options = 64; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.options = 0;
    d.e1[0] = 0; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.e1[0] = 1;
    d.n1 = -3; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.n1 = 7;
    d.n3 = 2; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL); d.n3 = 0;
    /* valid plane: validated and built on the host, then the first device call */
    EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EDEVICE);
    /* spheres, with shells; an axis parallel to e1 is invalid */
    d.geometry = RADIO_GEOM_SPHERE; d.radius = 1e4; d.axis[2] = 1; d.e1[0] = 1; d.n3 = 3;
    d.radius_step = 100; d.half1 = 0.1; d.half2 = 0.05;
    EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EDEVICE);
    d.axis[0] = 1; d.axis[2] = 0; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    d.axis[0] = 0; d.axis[2] = 1;
    d.radius_step = -1e4; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    d.radius_step = 100;
    double cells[9] = {1, 2, 3, 4, 5, 6, 7, 8, 9};
    d.geometry = RADIO_GEOM_EXPLICIT; d.n_cells = 3; d.cells = cells; d.n3 = 0;
    EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EDEVICE);
    cells[4] = INFINITY; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    d.cells = NULL; EXPECT(radio_detector_create(&d, NULL, &h), RADIO_EINVAL);
    /* chunk and batch arguments */
    radio_chunk k;
    memset(&k, 0, sizeof k);
    k.n_particles = 4; k.n_steps = 3; k.dt = 0.1;
    EXPECT(radio_deposit_trajectory_chunk(NULL, &k, NULL), RADIO_EINVAL);
    EXPECT(radio_deposit_trajectory_chunk_noalloc(NULL, &k, NULL), RADIO_EINVAL);
    EXPECT(radio_deposit_batch(NULL, NULL, -1, NULL), RADIO_EINVAL);
    EXPECT(radio_deposit_batch(NULL, NULL, 0, NULL), RADIO_OK);
    radio_detector* none[2] = {NULL, NULL};
    radio_chunk ks[2];
    memcpy(&ks[0], &k, sizeof k); memcpy(&ks[1], &k, sizeof k);
    EXPECT(radio_deposit_batch(none, ks, 2, NULL), RADIO_EDEVICE);
    EXPECT(radio_read_detector(NULL, NULL, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_detector_reset(NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_detector_load(NULL, cells, cells, NULL), RADIO_EINVAL);
    EXPECT(radio_detector_destroy(NULL), RADIO_OK);
    radio_stats s;
    EXPECT(radio_detector_stats(NULL, &s), RADIO_EINVAL);
    EXPECT(radio_detector_shape(NULL, NULL, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_detector_cells(NULL, cells), RADIO_EINVAL);
    EXPECT(radio_spectrum(NULL, 0, NULL, NULL, NULL, NULL, NULL), RADIO_EINVAL);
    /* tuning */
    radio_tuning t0, t;
    EXPECT(radio_get_tuning(&t0), RADIO_OK);
    t = t0; t.items_per_workgroup = 0; EXPECT(radio_set_tuning(&t), RADIO_EINVAL);
    t = t0; t.max_grid = 1 << 23; EXPECT(radio_set_tuning(&t), RADIO_EINVAL);
    t = t0; t.order_budget_mib = -1; EXPECT(radio_set_tuning(&t), RADIO_EINVAL);
    t = t0; t.target_blocks = 1000; EXPECT(radio_set_tuning(&t), RADIO_OK);
    EXPECT(radio_set_tuning(&t0), RADIO_OK);
    EXPECT(radio_set_tuning(NULL), RADIO_EINVAL);
    /* arrival times, slot coordinates, push */
    EXPECT(radio_arrival_times(NULL, NULL, NULL, 4, 1.0, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_arrival_times(NULL, NULL, NULL, 0, 1.0, NULL, NULL), RADIO_OK);
    EXPECT(radio_slot_coordinates(NULL, NULL, NULL, 0, 1.0, 0.0, -1.0, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_slot_coordinates(NULL, NULL, NULL, 2, 1.0, 0.0, 0.1, NULL, NULL), RADIO_EINVAL);
    radio_push_desc p;
    memset(&p, 0, sizeof p);
    p.qm = -1; p.dt = 0.1;
    EXPECT(radio_push(NULL, 1, 1, 0.0, 0, NULL, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_push(&p, 1, 1, 0.0, 0, NULL, NULL, NULL), RADIO_EINVAL);
    EXPECT(radio_push(&p, 0, 1, 0.0, 0, NULL, NULL, NULL), RADIO_OK);
    p.dt = -1; EXPECT(radio_push(&p, 1, 1, 0.0, 0, NULL, NULL, NULL), RADIO_EINVAL);
    int64_t bytes = 0;
    EXPECT(radio_noalloc_scratch_bytes(&bytes), RADIO_OK);
    EXPECT(radio_noalloc_scratch_bytes(NULL), RADIO_EINVAL);
    for (int c = -6; c <= 1; ++c)
        if (!radio_status_string(c) || !radio_status_string(c)[0]) ++fails;
    printf("runtime ok fails=%d scratch=%lld\n", fails, (long long)bytes);
    return fails;
}
"""


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    drv = tmp_path / "oracle_driver.c"
    exe = tmp_path / "oracle_driver"
    drv.write_text(ORACLE_DRIVER)
    subprocess.run(["gcc", "-O1", "-g", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", str(exe), str(drv),
                    os.path.join(ROOT, "oracle", "radio_oracle.c"), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.startswith("oracle ok bad=0")
    clipped = int(r.stdout.split("clipped=")[1].split()[0])
    back = int(r.stdout.split("back=")[1].split()[0])
    assert clipped > 0 and back > 0


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_runtime_under_address_and_undefined_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2302_14812_amd", "csrc")
    # the host pass only is instrumented (each -fsanitize behind -Xarch_host)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics", "-I",
              os.path.join(ROOT, "include"), "-I", csrc]
    objs = []
    procs = []
    # every source of the library, as its build compiles them
    for src in build_lib.SOURCES:
        obj = tmp_path / (src.split(".")[0] + ".o")
        procs.append(subprocess.Popen([HIPCC] + common + san + ["-x", "hip", "-c",
                                                                os.path.join(csrc, src), "-o",
                                                                str(obj)],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(str(obj))
    for p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, out.decode()[-3000:]
    drv = tmp_path / "runtime_driver.cpp"
    drv.write_text(RUNTIME_DRIVER)
    drv_obj = tmp_path / "runtime_driver.o"
    exe = tmp_path / "runtime_driver"
    subprocess.run([HIPCC] + common + san + ["-x", "hip", "-c", str(drv), "-o", str(drv_obj)],
                   check=True, capture_output=True)
    subprocess.run([HIPCC, "--offload-arch=gfx950"] + san + [str(drv_obj)] + objs +
                   ["-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=SAN_ENV, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.strip().endswith("scratch=268435456")
