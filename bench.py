"""Throughput of the radiation deposit on one MI355X.

A step is one pass of the whole hot path over the planar-undulator ensemble
(10^4 electrons, gamma ~ N(50, 0.5), K = 1, 20 periods in 4096 steps; a
128 x 128 spherical-cap detector at 1e5 with 2048 time slots): zero the
detector, deposit every (particle, segment, cell) triple, read E and B back.
Inputs are resident in HBM before the timed region.  Prints one JSON line.

The timed path is the mixed-precision deposit (`value`); the double-precision
deposit is timed in the same run and reported under "fp64".  The CPU oracle
is timed on a bounded sample of cells on the host cores (cpu_baseline).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic work of one (particle segment, cell) interaction, counting an FMA as
# two flops and a sqrt or divide as one: arrival time 16, n - beta and kappa 9,
# cross products 18, 1/kappa^3 and the two coefficients 7, E 9, B 9, one slot 16
FLOPS_PER_INTERACTION = 84
PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3, "mixed_twosum": 157.3}  # MI355X vector FP64 / FP32


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["mixed", "fp64", "mixed_twosum"], default="mixed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the double-precision leg")
    ap.add_argument("--no-twosum", action="store_true",
                    help="skip the compensated single-precision accumulation leg")
    ap.add_argument("--cpu-cells", type=int, default=0,
                    help="cells in the oracle sample (default: six per host thread)")
    ap.add_argument("--no-atomics", action="store_true",
                    help="skip the device measurement programs (atomic-add throughput, "
                         "vector instruction issue costs)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-launch leg (64 uneven sets, one persistent launch "
                         "vs 64 separate launches)")
    ap.add_argument("--batch-scale", type=float, default=0.02,
                    help="particle counts of the batched leg as a fraction of the recipe's")
    ap.add_argument("--no-serve", action="store_true", help="skip the streaming-service leg")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the detector-options leg (far field, hold rules)")
    ap.add_argument("--no-spectrum", action="store_true",
                    help="skip the spectral post-processing leg")
    ap.add_argument("--no-runtime", action="store_true",
                    help="skip the run-time (push and deposit) leg")
    ap.add_argument("--serve-chunks", type=int, default=30,
                    help="timed chunks of the streaming leg (after a fifth as many warm-up)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="bound on the streaming leg's offered stream (fewer chunks when "
                         "the device is slow)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="offered load as a fraction of the measured single-chunk throughput")
    ap.add_argument("--no-plasma", action="store_true",
                    help="skip the plasma-mirror configuration (2e5 electrons, 1000 steps, "
                         "256 x 256 cells, 4096 slots)")
    ap.add_argument("--plasma-particles", type=int, default=200_000,
                    help="electrons of the plasma-mirror leg (the configuration has 2e5)")
    ap.add_argument("--plasma-steps", type=int, default=1000,
                    help="steps of the plasma-mirror leg (the configuration has 1000 over ten "
                         "laser periods; fewer keep the same motion over a shorter time)")
    ap.add_argument("--plasma-fp64-steps", type=int, default=500,
                    help="steps of the plasma-mirror leg's double-precision run (the first "
                         "five laser periods by default, so that the benchmark fits its time)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def time_precision(radio, wl, chunk_dev, precision, steps, warmup, options=0, keep=False):
    import torch
    det = radio.Detector.from_spec(wl.detector, precision=precision, options=options)
    E = torch.empty((det.n_cells, det.n_t, 3), dtype=torch.float64, device="cuda")
    B = torch.empty_like(E)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        det.reset(stream)
        if ev is not None:
            ev[0].record(stream)
        det.deposit(chunk_dev, stream)
        if ev is not None:
            ev[1].record(stream)
        det.read(E, B, stream)

    for i in range(warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] {precision} warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in evs) / steps
    # deposit launches in the last step (a long chunk runs as time slices)
    time_precision.launches = det.stats()["slices"]
    det.close()
    if keep:
        return wall / steps * 1e3, kernel_ms, (E, B)
    del E, B
    return wall / steps * 1e3, kernel_ms


def options_leg(radio, wl, chunk_dev, precision, steps, warmup):
    """Detector options on the benchmark workload: far field (Eq. 3 arrival time, cell
    direction and distance in Eq. 1), far field with the acceleration term alone, the
    previous state's field held, and the linear interpolation.  Throughput of each and
    its departure from the default deposit (a property of the option, not of the
    kernel: every option matches the oracle with the same option in the tests)."""
    import torch
    out = {"precision": precision}
    fields = {}
    legs = (("default", 0), ("far_field", radio.FAR_FIELD),
            ("far_field_accel_only", radio.FAR_FIELD | radio.ACCEL_ONLY),
            ("hold_previous", radio.HOLD_PREVIOUS), ("hold_linear", radio.HOLD_LINEAR))
    for name, opt in legs:
        ms, kms, EB = time_precision(radio, wl, chunk_dev, precision, steps if opt else 1,
                                     warmup if opt else 0, options=opt, keep=True)
        fields[name] = EB[0]
        del EB
        inter = wl.interactions
        if opt:
            out[name] = {"options": opt, "ms_per_step": ms, "deposit_kernel_ms": kms,
                         "value": inter / (ms * 1e-3)}
        print(f"[bench] {precision} options={opt}: {ms:.1f} ms/step, "
              f"{inter / (ms * 1e-3):.3e} interactions/s", file=sys.stderr, flush=True)
    Ee = fields.pop("default")
    for name, Ef in fields.items():
        out[name]["rel_l2_vs_default"] = float(torch.linalg.vector_norm(Ef - Ee) /
                                               torch.linalg.vector_norm(Ee))
    del fields, Ee
    torch.cuda.synchronize()
    return out


def _alu_roofline(interactions, ms, precision):
    """The ALU roofline of a leg's deposits: FLOPS_PER_INTERACTION per interaction over
    its time (deposits with whatever else the leg's timed region holds) against the
    vector peak of its precision."""
    achieved = interactions * FLOPS_PER_INTERACTION / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS[precision],
            "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[precision], "traffic": None}


def batch_leg(radio, W, precision, steps, warmup, scale=0.02):
    """64 independent uneven sets of the batched-launch recipe (detectors of 32^2 to
    256^2 cells with 256 to 4096 slots, 500-4000 steps, helical or planar motion),
    particle counts times `scale`: one persistent batched launch vs 64 launches."""
    import torch

    from paper_2302_14812_amd import autotune
    sets = W.batched_sets(n_sets=64, scale=scale)
    chunks = [radio.Chunk.from_numpy(wl.chunk) for wl in sets]
    dets = [radio.Detector.from_spec(wl.detector, precision=precision) for wl in sets]
    total = sum(wl.interactions for wl in sets)
    defaults = radio.get_tuning()
    tuned = autotune.apply_batch([wl.detector for wl in sets], chunks)
    shape = radio.get_tuning()["shape"]
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            for d in dets:
                d.reset(stream)
            fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            for d in dets:
                d.reset(stream)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        return sum(ms) / len(ms)

    ms_batch = timed(lambda: radio.deposit_batch(dets, chunks, stream))
    print(f"[bench] batch ({precision}): one launch {ms_batch:.1f} ms", file=sys.stderr, flush=True)

    def separate():
        for d, c in zip(dets, chunks):
            d.deposit(c, stream)

    ms_sep = timed(separate)
    print(f"[bench] batch ({precision}): 64 launches {ms_sep:.1f} ms", file=sys.stderr, flush=True)
    sizes = [wl.interactions for wl in sets]
    radio.set_tuning(**defaults)
    for d in dets:
        d.close()
    det_bytes = sum(wl.detector.n_cells * wl.detector.n_t * 48 for wl in sets)
    return {"workload": f"64 uneven sets (batched-launch recipe: sides 32-256, 256-4096 slots, "
                        f"500-4000 steps; particle counts x {scale:g})",
            "detector_bytes": det_bytes,
            "interactions": total, "precision": precision,
            "smallest_set": min(sizes), "largest_set": max(sizes),
            "one_launch_ms": ms_batch, "separate_launches_ms": ms_sep,
            "one_launch_value": total / (ms_batch * 1e-3),
            "separate_value": total / (ms_sep * 1e-3),
            "speedup": ms_sep / ms_batch, "autotuned": tuned,
            "workgroup_shape": list(radio.SHAPES[shape]),
            "roofline": _alu_roofline(total, ms_batch, precision)}


def plasma_leg(radio, W, precisions, n_particles, n_steps=1000, fp64_steps=1000):
    """The plasma-mirror configuration at its stated size: 2 x 10^5 electrons on a
    20 lambda x 20 lambda sheet driven at 45 degrees (peak gamma 10, 1% momentum
    jitter), 1000 steps over 10 laser periods, a 256 x 256 cap about the specular
    direction at 1e5 with 4096 slots (1.31e13 interactions).  Per precision: a
    warm-up deposit of the chunk's first 32 steps, then one timed step (reset,
    deposit, read E and B), with the deposit kernel time from events around the
    deposit call.  The relative L2 of the single-precision result against the
    double path is taken over the whole detector."""
    import torch
    t = time.perf_counter()
    wl = W.plasma_mirror_workload(n_particles=n_particles)
    if n_steps < wl.chunk.n_steps:
        wl.chunk = wl.chunk.slice_steps(0, n_steps)
    chunk_dev = radio.Chunk.from_numpy(wl.chunk)
    inter_all = wl.chunk.n_particles * wl.chunk.n_steps * wl.detector.n_cells
    torch.cuda.synchronize()
    spec, inter, spec_name = wl.detector, inter_all, wl.name
    name = wl.name if n_steps >= 1000 else f"{wl.name} (first {n_steps} steps)"
    del wl
    print(f"[bench] plasma: {name} generated and copied in {time.perf_counter() - t:.1f} s "
          f"({inter:.3e} interactions)", file=sys.stderr, flush=True)
    warm = chunk_dev.slice_steps(0, 32)
    stream = torch.cuda.current_stream()
    out = {"workload": name, "n_particles": n_particles, "n_steps": chunk_dev.n_steps,
           "n_cells": spec.n_cells, "n_t": spec.n_t, "interactions": inter}
    fields = {}
    full = chunk_dev
    from paper_2302_14812_amd import autotune
    defaults = radio.get_tuning()
    for prec in precisions:
        # the double run may take the first fp64_steps steps only (same motion, shorter)
        chunk = full
        if prec == "fp64" and fp64_steps < full.n_steps:
            chunk = full.slice_steps(0, fp64_steps)
        inter = chunk.n_particles * chunk.n_steps * spec.n_cells
        radio.set_tuning(**defaults)
        tuned = autotune.apply_single(spec, chunk, prec)
        shape = radio.get_tuning()["shape"]
        print(f"[bench] plasma ({prec}): {chunk.n_steps} steps, {inter:.3e} interactions, "
              f"shape {radio.SHAPES[shape]}{' (tuned)' if tuned else ''}",
              file=sys.stderr, flush=True)
        det = radio.Detector.from_spec(spec, precision=prec)
        det.deposit(warm, stream)
        torch.cuda.synchronize()
        det.reset(stream)
        E = torch.empty((det.n_cells, det.n_t, 3), dtype=torch.float64, device="cuda")
        B = torch.empty_like(E)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        det.reset(stream)
        a.record(stream)
        det.deposit(chunk, stream)
        b.record(stream)
        det.read(E, B, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        kms = a.elapsed_time(b)
        st = det.stats()
        det.close()
        radio.set_tuning(**defaults)
        flops = inter * FLOPS_PER_INTERACTION
        # roofline.traffic is per launch: bytes per interaction x the mean launch's interactions
        bpi = measured_traffic_per_interaction(prec, spec_name, radio.SHAPES[shape])
        traffic = None if bpi is None else bpi * inter / max(1, st["slices"])
        out[prec] = {"value": inter / (ms * 1e-3), "ms_per_step": ms, "deposit_kernel_ms": kms,
                     "n_steps": chunk.n_steps, "interactions": inter, "autotuned": tuned,
                     "workgroup_shape": list(radio.SHAPES[shape]),
                     "deposit_launches_per_step": st["slices"],
                     "bypassed_per_interaction": st["bypassed"] / max(1, st["interactions"]),
                     "large_ring_fraction": st["large_ring"] / max(1, st["interactions"]),
                     "roofline": {"bound": "alu", "achieved": flops / (kms * 1e-3) / 1e12,
                                  "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                                  "frac": flops / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                                  "traffic": traffic}}
        if chunk is full:
            fields[prec] = (E, B)
        else:
            del E, B
        print(f"[bench] plasma ({prec}): {ms:.0f} ms, deposit {kms:.0f} ms in {st['slices']} "
              f"launches, {inter / (ms * 1e-3):.3e} interactions/s", file=sys.stderr, flush=True)
    if "fp64" in fields:
        E64, B64 = fields["fp64"]
        for prec, (E, B) in fields.items():
            if prec != "fp64":
                out[prec]["rel_l2_vs_fp64_path"] = max(
                    float(torch.linalg.vector_norm(E - E64) / torch.linalg.vector_norm(E64)),
                    float(torch.linalg.vector_norm(B - B64) / torch.linalg.vector_norm(B64)))
    if "fp64" in out and "mixed" in out:
        out["mixed_vs_fp64_speedup"] = out["mixed"]["value"] / out["fp64"]["value"]
    out["interactions"] = full.n_particles * full.n_steps * spec.n_cells
    del fields, chunk_dev, warm, full, chunk
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def serve_leg(radio, W, precisions, n_chunks, load, seconds=60.0):
    """Streaming service: 8 plasma-mirror detectors (256 x 256 cells, 4096 slots each)
    resident in HBM, fed by a Poisson stream of chunks of 1-64 steps x 10^3-10^5
    fresh particles.  The arrival rate is load x X / E[work], where X is the
    throughput measured on chunks deposited one at a time; p50/p99 latency is
    device completion minus host arrival, over the chunks after the warm-up."""
    import torch

    from paper_2302_14812_amd.serving import DepositServer, poisson_arrivals, replay
    n_det, side, n_t = 8, 256, 4096
    specs = {d: W.plasma_mirror_detector(n_side=side, n_t=n_t, seed=W.BASE_SEED + 3 + d)
             for d in range(n_det)}
    n_warm = max(1, n_chunks // 5)
    n_all = n_warm + n_chunks
    rows = list(W.stream_schedule(n_all, n_det, seed=W.BASE_SEED + 500, min_steps=1,
                                  max_steps=64, min_log_particles=3.0, max_log_particles=5.0))
    t = time.perf_counter()
    host = [(d, W.plasma_mirror_chunk(n, s0, st, seed=W.BASE_SEED + 1000 + k))
            for k, (d, s0, st, n) in enumerate(rows)]
    items = [(d, radio.Chunk.from_numpy(c)) for d, c in host]
    torch.cuda.synchronize()
    del host
    print(f"[bench] serve: {n_all} chunks generated in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    cells = side * side
    # E[work] of the recipe: E[S] = 32.5 steps, E[n] = (1e5 - 1e3) / ln(100) particles
    mean_work = 32.5 * (1e5 - 1e3) / math.log(100.0) * cells
    out = {}
    for prec in precisions:
        # X: chunks deposited one at a time on one resident detector
        det = radio.Detector.from_spec(specs[0], precision=prec)
        probe = [c for _, c in items[:6]]
        det.deposit(probe[0])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for c in probe:
            det.deposit(c)
        torch.cuda.synchronize()
        x_rate = sum(c.n_particles * c.n_steps * cells for c in probe) / (time.perf_counter() - t)
        det.close()
        rate = load * x_rate / mean_work
        # keep the stream to about `seconds`: fewer chunks when the device is slow
        n_use = int(min(n_all, max(10, rate * seconds)))
        n_skip = max(1, n_use * n_warm // n_all)
        offsets = poisson_arrivals(rate, n_use, seed=W.BASE_SEED + 501)
        print(f"[bench] serve ({prec}): X = {x_rate:.3e} I/s, {rate:.2f} chunks/s, "
              f"{n_use} chunks", file=sys.stderr, flush=True)

        def progress(k):
            if (k + 1) % 10 == 0:
                print(f"[bench] serve ({prec}): {k + 1} chunks submitted", file=sys.stderr,
                      flush=True)

        t = time.perf_counter()
        with DepositServer(specs, precision=prec) as srv:
            replay(srv, items[:n_use], offsets, progress=progress)
            srv.drain(timeout=600)
            st = srv.summary(skip=n_skip)
            for d in specs:
                srv.finish(d, read="none")
        print(f"[bench] serve ({prec}): {time.perf_counter() - t:.1f} s, p50 {st['p50_ms']:.0f} ms"
              f", p99 {st['p99_ms']:.0f} ms, {st['interactions_per_s']:.3e} I/s",
              file=sys.stderr, flush=True)
        st["single_chunk_rate"] = x_rate
        st["offered_chunks_per_s"] = rate
        st["warmup_chunks"] = n_skip
        st["timed_chunks"] = st.get("chunks", 0)
        if st["timed_chunks"] < 100:
            # too few chunks for a 99th percentile: it is the largest latency of the sample
            st["p99_note"] = f"max of {st['timed_chunks']} timed chunks"
        out[prec] = st
    del items
    torch.cuda.synchronize()
    return {"workload": f"{n_det} plasma-mirror detectors of {side}x{side} cells x {n_t} slots; "
                        f"Poisson chunks of 1-64 steps x 10^3-10^5 particles",
            "load": load, **out}


def spectrum_leg(radio, W, steps):
    """The paper's spectral benchmark at its size: one electron on a sinusoidal orbit
    (gamma 50, K 10, dt 0.01, six betatron periods) seen by a line of 512 cells at 1e5
    spanning +-0.1 rad with 131072 slots; deposit, then the spectral post-processing
    (per-cell transform in time, d2I/domega dOmega, dI/domega, dI/dOmega)."""
    import torch
    chunk = W.sinusoidal_orbit(37699)
    n_c, n_t = 512, 131072
    cells = W.line_cells(1e5, n_c, 0.1)
    t0, dtd = W.arrival_window(cells, chunk, n_t, pad_frac=0.01)
    dch = radio.Chunk.from_numpy(chunk)
    det = radio.Detector(cells, t0=t0, dt_det=dtd, n_t=n_t, precision="fp64")
    stream = torch.cuda.current_stream()
    det.deposit(dch)
    det.spectrum()  # warm: code objects, workspace path
    torch.cuda.synchronize()
    dep_ms, spec_ms = [], []
    for _ in range(steps):
        det.reset(stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        det.deposit(dch, stream)
        b.record(stream)
        torch.cuda.synchronize()
        dep_ms.append(a.elapsed_time(b))
        t = time.perf_counter()
        det.spectrum(stream=stream)  # returns after its stream work has finished
        spec_ms.append((time.perf_counter() - t) * 1e3)
    det.close()
    N = n_t
    # bytes the kernels move (two-step transform, both signals of a cell per
    # tile, Parseval's sums taken in the column step): E in and the column
    # transforms out, the column transforms in and the row-major |Z1|^2 + |Z2|^2
    # out, that in again for the power, d2I out
    fft_bytes = n_c * n_t * 24 + n_c * N * (32 + 32 + 8 + 8) + n_c * (N // 2 + 1) * 8
    alg_bytes = n_c * n_t * 24 + n_c * (N // 2 + 1) * 8       # E in, d2I out
    sms = min(spec_ms)
    print(f"[bench] spectrum: deposit {min(dep_ms):.1f} ms, spectrum {sms:.1f} ms "
          f"({alg_bytes / (sms * 1e-3) / 1e9:.0f} GB/s algorithmic)", file=sys.stderr, flush=True)
    return {"workload": "sinusoidal orbit gamma 50 K 10, 37699 steps; line of 512 cells x 131072 "
                        "slots at 1e5", "deposit_ms": min(dep_ms), "spectrum_ms": sms,
            "interactions": chunk.n_steps * n_c,
            "spectrum_roofline": {"bound": "hbm", "achieved": alg_bytes / (sms * 1e-3) / 1e9,
                                  "peak": 8000.0, "unit": "GB/s",
                                  "frac": alg_bytes / (sms * 1e-3) / 1e9 / 8000.0,
                                  "algorithmic_bytes": alg_bytes, "pass_bytes": fft_bytes}}


def runtime_leg(radio, W, precision):
    """The run-time mode: 10^4 electrons in a plane wave (a = 1.5, omega = 1, along +x)
    pushed on the device by radio_push 16 steps at a time (dt = 0.05, 1024 steps) and
    each block deposited right away into a 128 x 128 cap at 1e4 about +x with 2048
    slots; nothing leaves device memory.  Each block is a one-pair batched deposit,
    with the launch settings the tuning cache holds for such blocks."""
    import torch

    from paper_2302_14812_amd import autotune
    from paper_2302_14812_amd.runtime import RunTimeDiagnostic, plane_wave_electrons
    n_p, block, n_blocks, dt = 10000, 16, 64, 0.05
    cells, t0, dtd, n_t, x0, u0, wave = plane_wave_electrons(n_p, block, n_blocks, dt)
    det = radio.Detector(cells, t0=t0, dt_det=dtd, n_t=n_t, precision=precision)
    defaults = radio.get_tuning()
    tuned = autotune.apply_runtime(det, n_p, block, precision)
    shape = radio.get_tuning()["shape"]
    rt = RunTimeDiagnostic([det], x0, u0, None, dt=dt, block_steps=block, fields=wave)
    rt.advance(1)  # warm
    torch.cuda.synchronize()
    det.reset()
    rt = RunTimeDiagnostic([det], x0, u0, None, dt=dt, block_steps=block, fields=wave)
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    rt.advance(n_blocks)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    # the push alone, same blocks
    c, d = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c.record(stream)
    for _ in range(n_blocks):
        radio.push(rt.chunk, **wave)
    d.record(stream)
    torch.cuda.synchronize()
    push_ms = c.elapsed_time(d)
    inter = n_p * block * n_blocks * det.n_cells
    det.close()
    radio.set_tuning(**defaults)
    print(f"[bench] runtime ({precision}): {ms:.1f} ms for {n_blocks} push-deposit blocks, "
          f"push {push_ms:.1f} ms, {inter / (ms * 1e-3):.3e} interactions/s, shape "
          f"{radio.SHAPES[shape]}{' (tuned)' if tuned else ''}", file=sys.stderr, flush=True)
    return {"workload": "1e4 electrons in a plane wave (a 1.5), 1024 steps in blocks of 16; "
                        "128x128 cap at 1e4, 2048 slots", "precision": precision,
            "total_ms": ms, "push_ms": push_ms, "interactions": inter,
            "value": inter / (ms * 1e-3), "autotuned": tuned,
            "workgroup_shape": list(radio.SHAPES[shape]),
            "roofline": _alu_roofline(inter, ms, precision)}


def _traffic_record(name, workload):
    """A committed rocprofv3 counter summary (profiles/<name>), or None when it was
    taken on another workload or on a different kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2302_14812_amd", "csrc", "radio_kernels.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()[:16]
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256_16") != sha or rec.get("workload") != workload:
        return None
    return rec


def measured_traffic(precision, workload):
    """HBM bytes per deposit launch of the undulator benchmark from its counter summary."""
    rec = _traffic_record("deposit_traffic_undulator_10000e_4096steps.json", workload)
    leg = None if rec is None else rec.get("per_launch", {}).get(precision)
    return None if leg is None else leg["hbm_bytes"]


def measured_traffic_per_interaction(precision, workload, shape):
    """HBM bytes per interaction of the plasma-mirror deposit from its counter summary
    (taken on equal time slices, so it carries over to any launch of the same slicing),
    or None when the summary was taken with another workgroup shape."""
    rec = _traffic_record("deposit_traffic_plasma_mirror_200000e_256x256_4096bins.json", workload)
    leg = None if rec is None else rec.get("per_interaction", {}).get(precision)
    if leg is None or tuple(leg["workgroup_shape"]) != tuple(shape):
        return None
    return leg["hbm_bytes_per_interaction"]


def measurement_program(name):
    """Run one of the device measurement programs built with the library and return
    its JSON line.  Runs as a child process, so it is called before this process
    touches the GPU, and not at all under a profiler (whose preloaded library has
    touched it already)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2302_14812_amd", name)
    if not os.path.exists(exe):
        return {"skipped": "measurement program not built"}
    if "rocprof" in os.environ.get("LD_PRELOAD", "") or any(k.startswith("ROCPROF")
                                                             for k in os.environ):
        return {"skipped": "under a profiler"}
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return {"failed": r.returncode, "stderr": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def atomics_leg():
    """Floating-point atomic-add throughput of the GPU, the rates the deposit's ring
    flushes and slot emissions run against."""
    res = measurement_program("radio_atomics_bench")
    if "global_f64_spread" in res:
        print(f"[bench] atomics: global f64 {res['global_f64_spread']:.3e}/s coalesced, "
              f"{res['global_f64_wave']:.3e}/s one address per wave; LDS f64 "
              f"{res['lds_f64_spread']:.3e}/s", file=sys.stderr, flush=True)
    return res


def valu_leg():
    """Issue cost of the vector instructions the deposit is made of (cycles one
    wavefront instruction occupies a SIMD): with the deposit's instruction counts by
    type, the time its VALU work takes on this GPU."""
    res = measurement_program("radio_valu_bench")
    if "fma_f64" in res:
        print("[bench] valu cycles per wavefront instruction: " +
              ", ".join(f"{k} {v:.2f}" for k, v in res.items() if k not in ("unit", "clock_ghz")),
              file=sys.stderr, flush=True)
    return res


def cpu_baseline(wl, n_cells):
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    threads = max(1, min(threads, os.cpu_count() or 1))
    if n_cells <= 0:
        n_cells = 6 * threads  # about 15 s of oracle work on the benchmark workload
    n_c = wl.detector.n_cells
    idx = np.linspace(0, n_c - 1, n_cells).round().astype(np.int64)
    t0 = time.perf_counter()
    oracle.deposit_workload(wl.detector, wl.chunk, cell_index=idx, n_threads=threads)
    el = time.perf_counter() - t0
    inter = wl.chunk.n_particles * wl.chunk.n_steps * len(idx)
    # the same on one thread, over two of those cells
    idx1 = idx[[0, len(idx) // 2]] if len(idx) > 1 else idx
    t1 = time.perf_counter()
    oracle.deposit_workload(wl.detector, wl.chunk, cell_index=idx1, n_threads=1)
    el1 = time.perf_counter() - t1
    inter1 = wl.chunk.n_particles * wl.chunk.n_steps * len(idx1)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": inter / el, "unit": "interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(idx)} evenly spaced cells x all {wl.chunk.n_particles} particles x "
                      f"all {wl.chunk.n_steps} segments ({inter:.3e} interactions, {el:.1f} s)",
            "value_1thread": inter1 / el1,
            "sample_1thread": f"{len(idx1)} of those cells on one thread ({inter1:.3e} "
                              f"interactions, {el1:.1f} s)",
            "nproc": os.cpu_count(), "cpu_model": model}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the deposit is measured on a single MI355X "
              "(see the sharding paragraph of the design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    # the measurement programs run first, as child processes, while this one has
    # not touched the GPU yet
    atomics = None if args.no_atomics else atomics_leg()
    valu = None if args.no_atomics else valu_leg()
    import torch

    import paper_2302_14812_amd as radio
    from paper_2302_14812_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    wl = W.undulator_workload()
    gen_s = time.perf_counter() - t_gen
    print(f"[bench] generated {wl.name} in {gen_s:.1f} s ({wl.interactions:.3e} interactions "
          "per step)", file=sys.stderr, flush=True)
    chunk_dev = radio.Chunk.from_numpy(wl.chunk)
    torch.cuda.synchronize()
    inter = wl.interactions

    if args.calibrate_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] copied 1 GiB device to device (counter calibration)", file=sys.stderr,
              flush=True)
        del src, dst

    legs = {}
    fields = {}  # each leg's E, B (device) for the relative L2 against the double path
    order = [args.precision] + ([] if args.no_fp64 or args.precision == "fp64" else ["fp64"])
    if not args.no_twosum and args.precision != "mixed_twosum":
        order.append("mixed_twosum")
    # the headline leg takes the requested steps; the others three (after one warm-up),
    # so that every leg fits the run
    sec_steps, sec_warm = min(args.steps, 3), min(args.warmup, 1)
    from paper_2302_14812_amd import autotune
    defaults = radio.get_tuning()
    tuned = {}
    for prec in order:
        main = prec == args.precision
        # the tuned workgroup shape and split for this workload, where the cache has them
        radio.set_tuning(**defaults)
        tuned[prec] = autotune.apply_single(wl.detector, wl.chunk, prec)
        ms, kms, fields[prec] = time_precision(radio, wl, chunk_dev, prec,
                                               args.steps if main else sec_steps,
                                               args.warmup if main else sec_warm, keep=True)
        shape = radio.get_tuning()["shape"]
        radio.set_tuning(**defaults)
        flops = inter * FLOPS_PER_INTERACTION
        # the deposit call of a step is `launches` deposit-kernel launches of equal
        # work (time slices); flops / time is the same per launch and per step, and
        # roofline.traffic is per launch
        legs[prec] = {
            "value": inter / (ms * 1e-3), "ms_per_step": ms, "deposit_kernel_ms": kms,
            "steps": args.steps if main else sec_steps,
            "autotuned": tuned[prec], "shape": radio.SHAPES[shape],
            "deposit_launches_per_step": time_precision.launches,
            "roofline": {"bound": "alu", "achieved": flops / (kms * 1e-3) / 1e12,
                         "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                         "frac": flops / (kms * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                         "traffic": measured_traffic(prec, wl.name)},
        }
        print(f"[bench] {prec}: {ms:.1f} ms/step, deposit kernel {kms:.1f} ms, "
              f"{legs[prec]['value']:.3e} interactions/s", file=sys.stderr, flush=True)
    # error of each single-precision result, as relative L2 over the whole detector
    # against the double path (which the parity tests hold within 5e-14 of the
    # oracle); the larger of E and B
    if "fp64" in fields:
        E64, B64 = fields["fp64"]
        for prec, (E, B) in fields.items():
            if prec != "fp64":
                err = max(float(torch.linalg.vector_norm(E - E64) / torch.linalg.vector_norm(E64)),
                          float(torch.linalg.vector_norm(B - B64) / torch.linalg.vector_norm(B64)))
                legs[prec]["rel_l2_vs_fp64_path"] = err
                print(f"[bench] {prec}: relative L2 against the double path {err:.2e}",
                      file=sys.stderr, flush=True)
    del fields

    main_leg = legs[args.precision]
    opts = None if args.no_options else options_leg(radio, wl, chunk_dev, args.precision, 1, 1)
    del chunk_dev
    batch = None if args.no_batch else batch_leg(radio, W, args.precision, sec_steps, sec_warm,
                                                 args.batch_scale)
    out = {
        "metric": "LW interactions/s (particle-step x cell)",
        "value": main_leg["value"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "n_particles": wl.chunk.n_particles,
                   "n_steps": wl.chunk.n_steps, "n_cells": wl.detector.n_cells,
                   "n_t": wl.detector.n_t, "precision": args.precision,
                   "interactions_per_step": inter},
        "roofline": main_leg["roofline"],
        "deposit_launches_per_step": main_leg["deposit_launches_per_step"],
        "rel_l2_vs_fp64_path": main_leg.get("rel_l2_vs_fp64_path"),
        "autotuned": main_leg["autotuned"],
        "workgroup_shape": {"cells_per_tile": main_leg["shape"][0],
                            "particles_per_batch": main_leg["shape"][1],
                            "segments_per_run": main_leg["shape"][2]},
    }
    # ceilings of the interaction rate at F_int flops per interaction: double at the FP64
    # vector peak; mixed as its 25 double + 59 single flops at the two vector peaks
    # (single at the packed rate), and with every flop at 78.6 (the library is compiled without
    # packed single-precision instructions)
    fp64_ceiling = PEAK_TFLOPS["fp64"] * 1e12 / FLOPS_PER_INTERACTION
    blended = 1.0 / (25.0 / (PEAK_TFLOPS["fp64"] * 1e12) + 59.0 / (PEAK_TFLOPS["mixed"] * 1e12))
    out["ceilings"] = {"unit": "interactions/s", "fp64": fp64_ceiling, "mixed_blended": blended,
                       "mixed_unpacked": fp64_ceiling}
    if args.precision == "fp64":
        out["ceilings"]["frac_fp64"] = main_leg["value"] / fp64_ceiling
    else:
        out["ceilings"]["frac_mixed_blended"] = main_leg["value"] / blended
        out["ceilings"]["frac_mixed_unpacked"] = main_leg["value"] / fp64_ceiling
        if "fp64" in legs:
            out["ceilings"]["frac_fp64"] = legs["fp64"]["value"] / fp64_ceiling
    if "fp64" in legs and args.precision != "fp64":
        out["fp64"] = legs["fp64"]
        out["mixed_vs_fp64_speedup"] = legs["fp64"]["ms_per_step"] / main_leg["ms_per_step"]
    if "mixed_twosum" in legs and args.precision != "mixed_twosum":
        out["mixed_twosum"] = legs["mixed_twosum"]
    if opts is not None:
        out["options"] = opts
    if batch is not None:
        out["batch"] = batch
    if not args.no_plasma:
        precs = [args.precision] + (["fp64"] if args.precision != "fp64" and not args.no_fp64 else [])
        out["plasma_mirror"] = plasma_leg(radio, W, precs, args.plasma_particles,
                                          args.plasma_steps, args.plasma_fp64_steps)
    if not args.no_spectrum:
        out["spectrum"] = spectrum_leg(radio, W, sec_steps)
    if not args.no_runtime:
        out["runtime"] = runtime_leg(radio, W, args.precision)
    if not args.no_serve:
        precs = [args.precision] + (["fp64"] if args.precision != "fp64" and not args.no_fp64 else [])
        out["serve"] = serve_leg(radio, W, precs, args.serve_chunks, args.serve_load,
                                 args.serve_seconds)
    if atomics is not None:
        out["atomics"] = atomics
    if valu is not None:
        out["valu_issue_cycles"] = valu
    if not args.no_cpu_baseline:
        cb = cpu_baseline(wl, args.cpu_cells)
        out["cpu_baseline"] = cb
        print(f"[bench] cpu oracle: {cb['value']:.3e} interactions/s on {cb['cores']} threads",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
