"""Launch-parameter autotuner for the deposit.

Times candidate launch shapes on the device for a given workload and keeps
the fastest per size bucket in a JSON cache, so later calls with similar
shapes reuse the choice without timing again.  Two tunables (see
`radio_tuning` in include/radio.h):

  target_blocks        workgroups aimed at by one deposit: how finely the
                       runs of a chunk are split across workgroups
  items_per_workgroup  work items per resident workgroup in a batched
                       deposit: finer items balance uneven jobs, coarser
                       ones pay less per-item overhead

Timing uses HIP events on the current stream around the library's own
deposit calls on scratch detectors, so it measures exactly what a caller
gets; the caller's detectors are never touched.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Sequence

import paper_2302_14812_amd as radio

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "radio_mi355x", "tuning.json")


def cache_path() -> str:
    return os.environ.get("RADIO_TUNE_CACHE", DEFAULT_CACHE)


def _bucket(v: float) -> int:
    return int(round(math.log2(max(float(v), 1.0))))


def single_key(n_particles: int, n_steps: int, n_cells: int, precision: str) -> str:
    return f"single/{precision}/p{_bucket(n_particles)}/s{_bucket(n_steps)}/c{_bucket(n_cells)}"


def batch_key(n_pairs: int, total_interactions: float, spread: float) -> str:
    return f"batch/n{_bucket(n_pairs)}/i{_bucket(total_interactions)}/r{_bucket(spread)}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


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


def tune_single(spec, chunk: "radio.Chunk", precision: str = "mixed",
                candidates: Iterable[int] = (0, 768, 1536, 3072, 6144, 12288), repeats: int = 2,
                cache: Optional[Dict[str, dict]] = None) -> dict:
    """Pick target_blocks for deposits shaped like (spec, chunk)."""
    det = radio.Detector.from_spec(spec, precision=precision)
    saved = radio.get_tuning()
    results = {}
    try:
        for tb in candidates:
            radio.set_tuning(target_blocks=int(tb))
            results[int(tb)] = _time_ms(lambda: (det.reset(), det.deposit(chunk)), repeats)
    finally:
        radio.set_tuning(**saved)
        det.close()
    best = min(results, key=results.get)
    rec = {"target_blocks": best, "ms": results[best], "timings_ms": results}
    if cache is not None:
        cache[single_key(chunk.n_particles, chunk.n_steps, spec.n_cells, precision)] = rec
    return rec


def tune_batch(specs: Sequence, chunks: Sequence["radio.Chunk"], precision: str = "mixed",
               candidates: Iterable[int] = (1, 2, 4, 8, 16), repeats: int = 2,
               cache: Optional[Dict[str, dict]] = None) -> dict:
    """Pick items_per_workgroup for batches shaped like (specs, chunks)."""
    dets = [radio.Detector.from_spec(s, precision=precision) for s in specs]
    saved = radio.get_tuning()
    results = {}

    def run():
        for d in dets:
            d.reset()
        radio.deposit_batch(dets, list(chunks))

    try:
        for k in candidates:
            radio.set_tuning(items_per_workgroup=int(k))
            results[int(k)] = _time_ms(run, repeats)
    finally:
        radio.set_tuning(**saved)
        for d in dets:
            d.close()
    best = min(results, key=results.get)
    rec = {"items_per_workgroup": best, "ms": results[best], "timings_ms": results}
    if cache is not None:
        work = [s.n_cells * c.n_particles * c.n_steps for s, c in zip(specs, chunks)]
        cache[batch_key(len(work), sum(work), max(work) / max(1, min(work)))] = rec
    return rec


def apply_single(spec, chunk, precision: str, cache: Optional[Dict[str, dict]] = None) -> bool:
    """Set target_blocks from the cache if this shape was tuned; True if it was."""
    cache = load_cache() if cache is None else cache
    rec = cache.get(single_key(chunk.n_particles, chunk.n_steps, spec.n_cells, precision))
    if rec:
        radio.set_tuning(target_blocks=rec["target_blocks"])
    return bool(rec)


def apply_batch(specs: Sequence, chunks: Sequence, cache: Optional[Dict[str, dict]] = None) -> bool:
    cache = load_cache() if cache is None else cache
    work = [s.n_cells * c.n_particles * c.n_steps for s, c in zip(specs, chunks)]
    rec = cache.get(batch_key(len(work), sum(work), max(work) / max(1, min(work))))
    if rec:
        radio.set_tuning(items_per_workgroup=rec["items_per_workgroup"])
    return bool(rec)
