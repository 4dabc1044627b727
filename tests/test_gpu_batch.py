"""Batched deposits: many (detector, chunk) pairs of uneven size in one persistent launch.

Each detector's result must equal its separate deposit (up to the order of
floating-point additions) and the CPU oracle on sampled cells.
"""
import numpy as np
import pytest

import oracle
from paper_2302_14812_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import check_parity  # noqa: E402


@pytest.fixture(scope="module")
def radio():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_14812_amd as radio
    radio._lib()
    return radio


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def sets():
    # the batched workload's recipe at reduced sizes: 12 uneven sets
    return W.batched_sets(n_sets=12, max_particles=2000, max_steps=700, sides=(4, 8, 16, 24),
                          n_t_choices=(64, 128, 256))


def _read(det):
    import torch
    E, B = det.read()
    torch.cuda.synchronize()
    return E.cpu().numpy(), B.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_separate_and_oracle(radio, sets, precision):
    tol_sep = 1e-13 if precision == "fp64" else 1e-6
    tol_or = 1e-12 if precision == "fp64" else 1e-5
    chunks = [radio.Chunk.from_numpy(wl.chunk) for wl in sets]
    dets_b = [radio.Detector.from_spec(wl.detector, precision=precision) for wl in sets]
    radio.deposit_batch(dets_b, chunks)
    sizes = [wl.interactions for wl in sets]
    assert max(sizes) / max(1, min(sizes)) > 50  # uneven on purpose
    rng = np.random.Generator(np.random.PCG64(4))
    for wl, ch, db in zip(sets, chunks, dets_b):
        ds = radio.Detector.from_spec(wl.detector, precision=precision)
        ds.deposit(ch)
        Eb, Bb = _read(db)
        Es, Bs = _read(ds)
        e = max(rel_l2(Eb, Es), rel_l2(Bb, Bs))
        print(f"[batch] {wl.name} {precision}: batch vs alone relL2 {e:.3e}", flush=True)
        assert e <= tol_sep, (wl.name, e)
        assert db.stats()["interactions"] == wl.interactions
        idx = sorted(rng.choice(wl.detector.n_cells, size=min(6, wl.detector.n_cells),
                                replace=False).tolist())
        D = oracle.deposit_workload(wl.detector, wl.chunk, cell_index=idx)
        Eo, Bo = oracle.read(D)
        check_parity(Eb[idx], Bb[idx], Eo, Bo, tol_or, f"batch {wl.name} {precision} vs oracle")
        ds.close()
        db.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_batch_as_benchmarked(radio, precision):
    """The batched-launch benchmark's 64 uneven sets as it runs them (the recipe's
    sides of 32^2 to 256^2 cells and 256 to 4096 slots, particle counts x 0.02, one
    launch with the shipped tuning), each set against the oracle on its grid
    corners and two seeded cells."""
    import torch

    from paper_2302_14812_amd import autotune
    sets = W.batched_sets(n_sets=64, scale=0.02)
    chunks = [radio.Chunk.from_numpy(wl.chunk) for wl in sets]
    dets = [radio.Detector.from_spec(wl.detector, precision=precision) for wl in sets]
    cur = radio.get_tuning()
    try:
        tuned = autotune.apply_batch([wl.detector for wl in sets], chunks)
        radio.deposit_batch(dets, chunks)
        torch.cuda.synchronize()
    finally:
        radio.set_tuning(**cur)
    print(f"[batch] 64 benchmark sets {precision}: tuned {tuned}, "
          f"{sum(wl.interactions for wl in sets):.3e} interactions", flush=True)
    rng = np.random.Generator(np.random.PCG64(64))
    tol = 1e-12 if precision == "fp64" else 1e-5
    worst = 0.0
    for wl, d in zip(sets, dets):
        n1, n2 = wl.detector.grid
        idx = sorted(set(W.grid_corner_cells(n1, n2)) |
                     set(rng.choice(n1 * n2, 2, replace=False).tolist()))
        E, B = d.read()
        torch.cuda.synchronize()
        Eg, Bg = E[idx].cpu().numpy(), B[idx].cpu().numpy()
        assert d.stats()["interactions"] == wl.interactions
        d.close()
        Eo, Bo = oracle.read(oracle.deposit_workload(wl.detector, wl.chunk, cell_index=idx))
        check_parity(Eg, Bg, Eo, Bo, tol, f"benchmark set {wl.name} {precision}")
        worst = max(worst, rel_l2(Eg, Eo), rel_l2(Bg, Bo))
    print(f"[batch] 64 benchmark sets {precision}: worst relL2 against the oracle {worst:.3e}",
          flush=True)


def test_batch_mixed_modes_duplicates_and_empty(radio, sets):
    import torch
    wl = sets[0]
    halves = W.split_steps(wl.chunk, [wl.chunk.n_steps // 2])
    c_full = radio.Chunk.from_numpy(wl.chunk)
    c_h = [radio.Chunk.from_numpy(h) for h in halves]
    det64 = radio.Detector.from_spec(wl.detector, precision="fp64")
    detmx = radio.Detector.from_spec(wl.detector, precision="mixed")
    det2s = radio.Detector.from_spec(wl.detector, precision="mixed_twosum")
    empty = radio.Chunk(c_full.x[:, :, :0].contiguous(), c_full.u[:, :, :0].contiguous(), None,
                        0.0, 0.1)
    # one call: every precision, the fp64 detector twice (two halves), an empty chunk
    radio.deposit_batch([det64, detmx, det64, det2s, detmx],
                        [c_h[0], c_full, c_h[1], c_full, empty])
    ref = radio.Detector.from_spec(wl.detector, precision="fp64")
    ref.deposit(c_full)
    Er, Br = _read(ref)
    E64, B64 = _read(det64)
    # the halves keep the state times of the whole; only the order of additions differs
    assert max(rel_l2(E64, Er), rel_l2(B64, Br)) <= 1e-13
    for d in (detmx, det2s):
        Em, Bm = _read(d)
        assert max(rel_l2(Em, Er), rel_l2(Bm, Br)) <= 1e-5
    assert det64.stats()["chunks"] == 2 and detmx.stats()["chunks"] == 2
    for d in (det64, detmx, det2s, ref):
        d.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed_twosum"])
def test_batch_time_slices_long_chunks(radio, sets, precision):
    """A batched pair whose particle orders exceed the order budget is deposited in
    the time slices of a single deposit, after the persistent launch; the other
    pairs stay in the launch.  Here the long chunk (2000 particles x 150 steps on
    32 x 32 cells) goes twice to one detector, in three slices each under a 1 MiB
    budget.  Every detector equals its whole-chunk deposits, counts the slices a
    single deposit would make, and the long chunk's detector matches the oracle
    on sampled cells."""
    import torch
    tol_whole = 1e-13 if precision == "fp64" else 1e-6
    tol_or = 1e-12 if precision == "fp64" else 1e-5
    long = W.random_chunk(2000, 150, seed=41, dt=0.05, gamma_max=10.0)
    cells = W.plane_cells([0, 0, 30.0], [1, 0, 0], [0, 1, 0], 32, 32, 6.0, 6.0)
    t0, dtd = W.arrival_window(cells, long, 400, pad_frac=0.05,
                               cell_index=W.grid_corner_cells(32, 32), seed=41)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=400)
    c_long = radio.Chunk.from_numpy(long)
    short = sets[:3]
    c_short = [radio.Chunk.from_numpy(wl.chunk) for wl in short]
    # whole-chunk references at the default budget
    ref_long = radio.Detector.from_spec(spec, precision=precision)
    ref_long.deposit(c_long)
    ref_long.deposit(c_long)
    refs = []
    for wl, c in zip(short, c_short):
        r = radio.Detector.from_spec(wl.detector, precision=precision)
        r.deposit(c)
        refs.append(r)
    torch.cuda.synchronize()
    cur = radio.get_tuning()
    try:
        radio.set_tuning(order_budget_mib=1)
        d_long = radio.Detector.from_spec(spec, precision=precision)
        d_short = [radio.Detector.from_spec(wl.detector, precision=precision) for wl in short]
        radio.deposit_batch([d_short[0], d_long, d_short[1], d_long, d_short[2]],
                            [c_short[0], c_long, c_short[1], c_long, c_short[2]])
        # slices of single deposits under the same budget
        single = []
        for wl, c in zip(short, c_short):
            d = radio.Detector.from_spec(wl.detector, precision=precision)
            d.deposit(c)
            torch.cuda.synchronize()
            single.append(d.stats()["slices"])
            d.close()
    finally:
        radio.set_tuning(**cur)
    st = d_long.stats()
    assert (st["chunks"], st["slices"]) == (2, 6)
    assert st["interactions"] == 2 * 2000 * 150 * 1024
    E, B = _read(d_long)
    Er, Br = _read(ref_long)
    e = max(rel_l2(E, Er), rel_l2(B, Br))
    print(f"[batch] long chunk twice in time slices vs whole {precision} relL2 {e:.3e}",
          flush=True)
    assert e <= tol_whole
    idx = [0, 31, 500, 992, 1023]
    D = oracle.deposit_workload(spec, long, cell_index=idx)
    Eo, Bo = oracle.read(D)
    check_parity(E[idx], B[idx], 2.0 * Eo, 2.0 * Bo, tol_or,
                 f"batch long chunk twice in time slices vs oracle {precision}")
    for wl, d, r, n_single in zip(short, d_short, refs, single):
        E, B = _read(d)
        Er, Br = _read(r)
        e = max(rel_l2(E, Er), rel_l2(B, Br))
        print(f"[batch] {wl.name} beside the sliced pairs {precision}: relL2 {e:.3e}, slices "
              f"{d.stats()['slices']} (single deposit {n_single})", flush=True)
        assert e <= tol_whole
        assert d.stats()["slices"] == n_single
    for d in [d_long, ref_long] + d_short + refs:
        d.close()


def test_batch_rejects_invalid_pairs_without_work(radio, sets):
    wl = sets[1]
    det = radio.Detector.from_spec(wl.detector)
    good = radio.Chunk.from_numpy(wl.chunk)
    bad = radio.Chunk(good.x, good.u, good.q, 0.0, -1.0)
    with pytest.raises(radio.RadioError):
        radio.deposit_batch([det, det], [good, bad])
    E, B = _read(det)
    assert np.abs(E).max() == 0.0 and det.stats()["chunks"] == 0
    det.close()


def test_tuning_roundtrip(radio):
    cur = radio.get_tuning()
    radio.set_tuning(target_blocks=1024, items_per_workgroup=2, shape=2)
    assert radio.get_tuning() == {"target_blocks": 1024, "items_per_workgroup": 2,
                                  "max_grid": cur["max_grid"],
                                  "order_budget_mib": cur["order_budget_mib"], "shape": 2}
    with pytest.raises(radio.RadioError):
        radio.set_tuning(shape=len(radio.SHAPES))
    with pytest.raises(radio.RadioError):
        radio.set_tuning(order_budget_mib=-1)
    with pytest.raises(radio.RadioError):
        radio.set_tuning(max_grid=0)
    with pytest.raises(radio.RadioError):
        radio.set_tuning(max_grid=(1 << 22) + 1)
    with pytest.raises(radio.RadioError):
        radio.set_tuning(target_blocks=-1)
    radio.set_tuning(target_blocks=0)  # automatic splits
    assert radio.get_tuning()["target_blocks"] == 0
    radio.set_tuning(**cur)
    assert radio.get_tuning() == cur


def test_autotuner_picks_a_candidate_and_caches(radio, sets, tmp_path):
    from paper_2302_14812_amd import autotune
    specs = [wl.detector for wl in sets[:6]]
    chunks = [radio.Chunk.from_numpy(wl.chunk) for wl in sets[:6]]
    cache = {}
    before = radio.get_tuning()
    rb = autotune.tune_batch(specs, chunks, precision="fp64", candidates=(1, 4), repeats=1,
                             cache=cache)
    # every shape timed at the current items per workgroup, then both candidates
    assert rb["items_per_workgroup"] in (1, 4, before["items_per_workgroup"])
    assert rb["shape"] in radio.SHAPES and len(rb["timings_ms"]) >= len(radio.SHAPES) + 1
    rs = autotune.tune_single(specs[0], chunks[0], precision="fp64", candidates=(256, 1024),
                              repeats=1, cache=cache)
    assert rs["target_blocks"] in (256, 1024) and rs["shape"] in radio.SHAPES
    assert radio.get_tuning() == before  # tuning restores the caller's settings
    path = str(tmp_path / "tune.json")
    autotune.save_cache(cache, path)
    loaded = autotune.load_cache(path, shipped=False)
    assert loaded == json_roundtrip(cache)
    assert autotune.apply_batch(specs, chunks, cache=loaded)
    t = radio.get_tuning()
    assert (t["items_per_workgroup"], t["shape"]) == (rb["items_per_workgroup"], rb["shape"])
    radio.set_tuning(**before)


def json_roundtrip(obj):
    import json
    return json.loads(json.dumps(obj))
