"""Launch-parameter autotuner for the deposit.

Times candidate launch configurations on the device for a given workload and
keeps the fastest per size bucket in a JSON cache, so later calls with similar
sizes reuse the choice without timing again.  Tunables (see `radio_tuning` in
include/radio.h):

  shape                the deposit's workgroup shape (SHAPES: cells per tile,
                       particles per batch, segments per run), for detectors
                       with the default options
  target_blocks        workgroups aimed at by one deposit: how finely the
                       runs of a chunk are split across workgroups
  items_per_workgroup  work items per resident workgroup in a batched
                       deposit: finer items balance uneven jobs, coarser
                       ones pay less per-item overhead

Timing uses HIP events on the current stream around the library's own
deposit calls on scratch detectors, so it measures exactly what a caller
gets; the caller's detectors are never touched.

The package ships a cache (tuning_cache.json, written by `python -m
paper_2302_14812_amd.autotune --ship` on the GPU) for the benchmark's
workloads; a user cache (RADIO_TUNE_CACHE or ~/.cache/radio_mi355x) adds to
it and wins where both have an entry.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Sequence

import paper_2302_14812_amd as radio

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "radio_mi355x", "tuning.json")
SHIPPED_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def cache_path() -> str:
    return os.environ.get("RADIO_TUNE_CACHE", DEFAULT_CACHE)


def _bucket(v: float) -> int:
    return int(round(math.log2(max(float(v), 1.0))))


# chunks of this many steps or more share a bucket: past a few particle-order groups
# (two runs each) a deposit's cost per interaction no longer depends on its length
LONG_STEPS_BUCKET = 7


def single_key(n_particles: int, n_steps: int, n_cells: int, precision: str) -> str:
    s = min(_bucket(n_steps), LONG_STEPS_BUCKET)
    return f"single/{precision}/p{_bucket(n_particles)}/s{s}/c{_bucket(n_cells)}"


def batch_key(n_pairs: int, total_interactions: float, spread: float) -> str:
    return f"batch/n{_bucket(n_pairs)}/i{_bucket(total_interactions)}/r{_bucket(spread)}"


def _read(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def load_cache(path: Optional[str] = None, shipped: bool = True) -> Dict[str, dict]:
    """The tuning cache: the shipped entries (unless shipped=False) updated with
    those of `path` (default: the user cache)."""
    out = _read(SHIPPED_CACHE) if shipped else {}
    out.update(_read(path or cache_path()))
    return out


def save_cache(cache: Dict[str, dict], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(fn, repeats: int) -> float:
    import torch
    s = torch.cuda.current_stream()
    fn()  # warm: workspaces, code objects
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def _shapes_for(specs, shapes: Iterable[int]) -> List[int]:
    """Shapes worth timing: all of them when every detector has the default
    options, else the default (the library uses it for detectors with options)."""
    shapes = [int(s) for s in shapes]
    if any(getattr(s, "options", 0) for s in specs):
        return [0]
    return shapes


def tune_single(spec, chunk: "radio.Chunk", precision: str = "mixed",
                candidates: Iterable[int] = (0, 768, 1536, 3072, 6144, 12288), repeats: int = 2,
                cache: Optional[Dict[str, dict]] = None,
                shapes: Iterable[int] = tuple(radio.SHAPES),
                progress: Optional[Callable[[str], None]] = None) -> dict:
    """Pick the workgroup shape and target_blocks for deposits like (spec, chunk):
    the shapes at the first candidate, then the candidates at the best shape.
    progress, if given, receives a line per timed configuration."""
    det = radio.Detector.from_spec(spec, precision=precision)
    saved = radio.get_tuning()
    candidates = [int(c) for c in candidates]
    results = {}

    def timed(shape, tb):
        radio.set_tuning(shape=shape, target_blocks=tb)
        key = f"{shape}/{tb}"
        if key not in results:
            results[key] = _time_ms(lambda: (det.reset(), det.deposit(chunk)), repeats)
            if progress:
                progress(f"shape {shape} target_blocks {tb}: {results[key]:.1f} ms")
        return results[key]

    try:
        best_shape = min(_shapes_for([spec], shapes), key=lambda sh: timed(sh, candidates[0]))
        for tb in candidates:
            timed(best_shape, tb)
    finally:
        radio.set_tuning(**saved)
        det.close()
    best = min(results, key=results.get)
    shape, tb = (int(v) for v in best.split("/"))
    rec = {"shape": shape, "target_blocks": tb, "ms": results[best], "timings_ms": results}
    if cache is not None:
        cache[single_key(chunk.n_particles, chunk.n_steps, spec.n_cells, precision)] = rec
    return rec


def tune_batch(specs: Sequence, chunks: Sequence["radio.Chunk"], precision: str = "mixed",
               candidates: Iterable[int] = (1, 2, 4, 8, 16), repeats: int = 2,
               cache: Optional[Dict[str, dict]] = None,
               shapes: Iterable[int] = tuple(radio.SHAPES),
               progress: Optional[Callable[[str], None]] = None) -> dict:
    """Pick the workgroup shape and items_per_workgroup for batches like (specs,
    chunks): the shapes at the current items_per_workgroup, then the candidates at
    the best shape.  progress, if given, receives a line per timed configuration."""
    dets = [radio.Detector.from_spec(s, precision=precision) for s in specs]
    saved = radio.get_tuning()
    results = {}

    def run():
        for d in dets:
            d.reset()
        radio.deposit_batch(dets, list(chunks))

    def timed(shape, k):
        radio.set_tuning(shape=shape, items_per_workgroup=k)
        key = f"{shape}/{k}"
        if key not in results:
            results[key] = _time_ms(run, repeats)
            if progress:
                progress(f"shape {shape} items_per_workgroup {k}: {results[key]:.1f} ms")
        return results[key]

    try:
        k0 = saved["items_per_workgroup"]
        best_shape = min(_shapes_for(specs, shapes), key=lambda sh: timed(sh, k0))
        for k in candidates:
            timed(best_shape, int(k))
    finally:
        radio.set_tuning(**saved)
        for d in dets:
            d.close()
    best = min(results, key=results.get)
    shape, k = (int(v) for v in best.split("/"))
    rec = {"shape": shape, "items_per_workgroup": k, "ms": results[best], "timings_ms": results}
    if cache is not None:
        work = [s.n_cells * c.n_particles * c.n_steps for s, c in zip(specs, chunks)]
        cache[batch_key(len(work), sum(work), max(work) / max(1, min(work)))] = rec
    return rec


def apply_single(spec, chunk, precision: str, cache: Optional[Dict[str, dict]] = None) -> bool:
    """Set the shape and target_blocks from the cache if deposits like this were
    tuned; True if they were."""
    cache = load_cache() if cache is None else cache
    rec = cache.get(single_key(chunk.n_particles, chunk.n_steps, spec.n_cells, precision))
    if rec:
        radio.set_tuning(target_blocks=rec["target_blocks"], shape=rec.get("shape", 0))
    return bool(rec)


def apply_batch(specs: Sequence, chunks: Sequence, cache: Optional[Dict[str, dict]] = None) -> bool:
    """Set the shape and items_per_workgroup from the cache if batches like this
    were tuned; True if they were."""
    cache = load_cache() if cache is None else cache
    work = [s.n_cells * c.n_particles * c.n_steps for s, c in zip(specs, chunks)]
    rec = cache.get(batch_key(len(work), sum(work), max(work) / max(1, min(work))))
    if rec:
        radio.set_tuning(items_per_workgroup=rec["items_per_workgroup"], shape=rec.get("shape", 0))
    return bool(rec)


def runtime_key(n_particles: int, block_steps: int, n_cells: int, precision: str) -> str:
    return (f"runtime/{precision}/p{_bucket(n_particles)}/s{_bucket(block_steps)}"
            f"/c{_bucket(n_cells)}")


def tune_runtime(spec, block: "radio.Chunk", precision: str = "mixed",
                 cache: Optional[Dict[str, dict]] = None, **kw) -> dict:
    """Pick the workgroup shape and items_per_workgroup for run-time deposits: one
    block of pushed steps into one detector per call, a one-pair batch."""
    rec = tune_batch([spec], [block], precision, cache=None, **kw)
    if cache is not None:
        cache[runtime_key(block.n_particles, block.n_steps, spec.n_cells, precision)] = rec
    return rec


def apply_runtime(det, n_particles: int, block_steps: int, precision: str,
                  cache: Optional[Dict[str, dict]] = None) -> bool:
    """Set the shape and items_per_workgroup for run-time blocks like these from the
    cache; True if such blocks were tuned."""
    cache = load_cache() if cache is None else cache
    rec = cache.get(runtime_key(n_particles, block_steps, det.n_cells, precision))
    if rec:
        radio.set_tuning(items_per_workgroup=rec["items_per_workgroup"], shape=rec.get("shape", 0))
    return bool(rec)


def ship(path: str = SHIPPED_CACHE, repeats: int = 2) -> Dict[str, dict]:
    """Tune the benchmark's workloads and write the shipped cache: the planar
    undulator ensemble (single deposits, both precisions), the plasma-mirror sheet
    (2e5 electrons; its first 200 steps, which share the bucket of the whole run;
    both precisions), the 64 uneven sets of the batched-launch benchmark (mixed) and the
    run-time mode's 16-step blocks of plane-wave electrons (mixed)."""
    import sys

    import torch

    from paper_2302_14812_amd import workloads as W
    cache: Dict[str, dict] = {}

    def note(line):
        print(f"[tune]   {line}", file=sys.stderr, flush=True)

    wl = W.undulator_workload()
    chunk = radio.Chunk.from_numpy(wl.chunk)
    for prec in ("mixed", "fp64"):
        rec = tune_single(wl.detector, chunk, prec, candidates=(0,), repeats=repeats, cache=cache,
                          progress=note)
        print(f"[tune] {wl.name} {prec}: {rec}", file=sys.stderr, flush=True)
    del chunk
    pm = W.plasma_mirror_workload(n_particles=200_000)
    chunk = radio.Chunk.from_numpy(pm.chunk.slice_steps(0, 200))
    for prec in ("mixed", "fp64"):
        rec = tune_single(pm.detector, chunk, prec, candidates=(0,), repeats=1, cache=cache,
                          progress=note)
        print(f"[tune] {pm.name} (first 200 steps) {prec}: {rec}", file=sys.stderr, flush=True)
    del chunk, pm
    sets = W.batched_sets(n_sets=64, scale=0.02)
    chunks = [radio.Chunk.from_numpy(s.chunk) for s in sets]
    rec = tune_batch([s.detector for s in sets], chunks, "mixed", candidates=(2, 4, 8, 16),
                     repeats=repeats, cache=cache, progress=note)
    print(f"[tune] 64 batched sets mixed: {rec}", file=sys.stderr, flush=True)
    del chunks
    # run-time blocks: a 16-step block from the middle of the plane-wave run
    from paper_2302_14812_amd.runtime import plane_wave_electrons
    cells, t0, dtd, n_t, x0, u0, wave = plane_wave_electrons()
    xs = torch.zeros((3, 1025, x0.shape[1]), dtype=torch.float64, device="cuda")
    us = torch.zeros_like(xs)
    xs[:, 0] = torch.from_numpy(x0).cuda()
    us[:, 0] = torch.from_numpy(u0).cuda()
    run = radio.push(radio.Chunk(xs, us, None, 0.0, 0.05), **wave)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t)
    rec = tune_runtime(spec, run.slice_steps(512, 528), "mixed", candidates=(2, 4, 8),
                       repeats=repeats, cache=cache, progress=note)
    print(f"[tune] run-time blocks mixed: {rec}", file=sys.stderr, flush=True)
    del run, xs, us
    torch.cuda.synchronize()
    save_cache(cache, path)
    return cache


if __name__ == "__main__":
    import sys
    if "--ship" in sys.argv:
        ship()
