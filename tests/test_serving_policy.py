"""The deposit service's policy (admission by memory, batch formation), on a virtual clock."""
import numpy as np
import pytest

from paper_2302_14812_amd.serving import (Request, Scheduler, detector_bytes, poisson_arrivals,
                                          simulate, summarize)
from paper_2302_14812_amd import workloads as W


def make_sched(n_det=4, bytes_each=100, budget=1000, cells=10, max_work=1e9):
    return Scheduler({d: bytes_each for d in range(n_det)}, {d: cells for d in range(n_det)},
                     budget, max_work)


def test_admission_respects_budget_and_does_not_block_residents():
    s = make_sched(n_det=5, bytes_each=100, budget=300)
    for k, d in enumerate([0, 1, 2, 3, 0, 4, 1]):
        s.add(Request(d, 10, 2, float(k)))
    assert s.admit() == [0, 1, 2]
    assert s.used() == 300 and s.peak_resident == 3
    b = s.next_batch()
    # every request of a resident detector, in arrival order; 3 and 4 wait
    assert [r.det_id for r in b] == [0, 1, 2, 0, 1]
    assert [r.det_id for r in s.pending] == [3, 4]
    assert not s.runnable()
    assert s.next_batch() == []
    s.release(1)
    assert s.runnable() and s.admit() == [3]
    assert [r.det_id for r in s.next_batch()] == [3]
    assert s.admission_order == [0, 1, 2, 3]
    with pytest.raises(ValueError):
        s.add(Request(1, 1, 1, 9.0))  # finished detectors take no more chunks
    with pytest.raises(KeyError):
        s.add(Request(7, 1, 1, 9.0))


def test_oversized_detector_is_rejected():
    s = Scheduler({0: 50, 1: 500}, {0: 1, 1: 1}, 100, 1e9)
    s.add(Request(0, 1, 1, 0.0))
    with pytest.raises(ValueError):
        s.add(Request(1, 1, 1, 0.0))


def test_batches_are_fifo_and_bounded_in_work():
    s = make_sched(n_det=2, cells=1, max_work=100)
    works = [30, 30, 30, 30, 500, 10]
    for k, w in enumerate(works):
        s.add(Request(k % 2, w, 1, float(k)))
    s.admit()
    sizes = []
    while s.pending:
        sizes.append([r.work for r in s.next_batch()])
    # the bound cuts a batch before the request that would cross it; a request
    # larger than the bound runs alone; order is arrival order throughout
    assert sizes == [[30, 30, 30], [30], [500], [10]]
    assert s.n_batches == 4


def test_work_counts_interactions():
    s = Scheduler({0: 1}, {0: 64}, 10, 1e9)
    r = s.add(Request(0, 1000, 7, 0.0))
    assert r.work == 1000 * 7 * 64


def test_detector_bytes_counts_accumulator_and_cells():
    spec = W.DetectorSpec(cells=np.zeros((12, 3)), t0=0.0, dt_det=1.0, n_t=100)
    assert detector_bytes(spec) == 12 * 100 * 48 + 12 * 32


def _stream(n, rate, seed, n_det=4, cells=256):
    offs = poisson_arrivals(rate, n, seed)
    sched_rows = list(W.stream_schedule(n, n_det, seed, max_log_particles=4.0))
    return [Request(d, npart, st, float(t)) for (d, _, st, npart), t in zip(sched_rows, offs)]


def test_light_load_latency_is_the_service_time():
    # one chunk at a time: each waits for nothing and takes its own service time
    s = make_sched(n_det=4, cells=256)
    reqs = [Request(k % 4, 100, 4, 10.0 * k) for k in range(20)]
    simulate(s, reqs, lambda b: 1e-3 + sum(r.work for r in b) / 1e9)
    for r in reqs:
        assert r.launched == r.arrival
        assert r.latency == pytest.approx(1e-3 + 100 * 4 * 256 / 1e9)
    assert s.n_batches == 20


def test_heavy_load_forms_larger_batches_and_keeps_up():
    rate_cap = 1e11  # interactions per second of the modelled device
    reqs = _stream(400, rate=2000.0, seed=5)
    work = sum(r.n_particles * r.n_steps * 256 for r in reqs)
    span = max(r.arrival for r in reqs)
    overhead = 2e-3
    s = make_sched(n_det=4, cells=256)
    simulate(s, reqs, lambda b: overhead + sum(r.work for r in b) / rate_cap)
    st = summarize(reqs, sched=s)
    assert st["chunks"] == 400
    # offered load above what one-chunk batches could carry, yet the service
    # keeps up because batches grow and share the fixed overhead
    assert 400 * overhead + work / rate_cap > span > work / rate_cap
    assert st["batches"] < 400 / 2
    # a stable queue: the tail stays at a few batch times, far below the
    # stream's length (an overloaded one would grow towards it)
    assert st["p99_ms"] < 0.15 * 1e3 * span
    # every launch happens no earlier than the arrival and completion after launch
    for r in reqs:
        assert r.arrival <= r.launched <= r.completion


def test_inflight_bound_holds():
    s = make_sched(n_det=2, cells=1)
    reqs = [Request(k % 2, 1, 1, 0.001 * k) for k in range(50)]
    simulate(s, reqs, lambda b: 0.01, max_inflight=2)
    # at any launch time, at most two batches are unfinished
    launches = sorted({(r.batch, r.launched, r.completion) for r in reqs})
    for b, t, _ in launches:
        running = sum(1 for b2, t2, c2 in launches if t2 <= t < c2)
        assert running <= 2
    # batches run back to back on the device
    ends = sorted({r.completion for r in reqs})
    assert all(np.isclose(b - a, 0.01) for a, b in zip(ends, ends[1:]))


def test_summary_percentiles():
    reqs = [Request(0, 1, 1, 0.0) for _ in range(100)]
    for k, r in enumerate(reqs):
        r.completion = (k + 1) * 1e-3
        r.work = 1
        r.batch = k
    st = summarize(reqs)
    assert st["p50_ms"] == pytest.approx(50.5)
    assert st["p99_ms"] == pytest.approx(99.01)
    assert st["interactions_per_s"] == pytest.approx(100 / 0.1)


def test_plasma_mirror_chunk_shape_and_speed():
    a = W.plasma_mirror_chunk(50, 40, 20, seed=3)
    again = W.plasma_mirror_chunk(50, 40, 20, seed=3)
    assert np.array_equal(a.x, again.x) and np.array_equal(a.u, again.u)
    assert a.x.shape == (3, 21, 50) and a.q.shape == (50,)
    assert a.t_first == pytest.approx(40 * a.dt)
    # every step is slower than light, and the sheet oscillates about x = 0
    step = np.linalg.norm(np.diff(a.x, axis=1), axis=0)
    assert step.max() < a.dt
    assert np.abs(a.x[0]).max() < 3.0
