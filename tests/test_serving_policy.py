"""The deposit service's policy (admission by memory, batch formation), on a virtual clock."""
import numpy as np
import pytest

from paper_2302_14812_amd.serving import (Request, Scheduler, detector_bytes, plan_pieces,
                                          poisson_arrivals, simulate, summarize)
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
    assert [r.det_id for r, _ in b] == [0, 1, 2, 0, 1]
    assert [r.det_id for r in s.pending] == [3, 4]
    assert not s.runnable()
    assert s.next_batch() == []
    s.release(1)
    assert s.runnable() and s.admit() == [3]
    assert [r.det_id for r, _ in s.next_batch()] == [3]
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
        sizes.append([r.work for r, _ in s.next_batch()])
    # a batch takes what fits in arrival order, skipping a request that would
    # cross the bound (it goes first in a later batch); a request larger than
    # the bound runs alone
    assert sizes == [[30, 30, 30, 10], [30], [500]]
    assert s.n_batches == 3


def test_round_robin_over_parts():
    s = make_sched(n_det=2, cells=1, max_work=40)
    big = s.add(Request(0, 10, 1, 0.0, pieces=[(None, 10)] * 8))   # 80 in parts of 10
    small = s.add(Request(1, 10, 1, 1.0, pieces=[(None, 10)]))
    s.admit()
    b1 = s.next_batch()
    # the big request's first part, the small request, then more parts of the big one
    assert [(r is big, k) for r, k in b1] == [(True, 0), (False, 0), (True, 1), (True, 2)]
    assert s.piece_done(small)          # the small request completes with the first batch
    assert not s.piece_done(big)
    rest = []
    while s.pending:
        rest.append([k for r, k in s.next_batch()])
    assert rest == [[3, 4, 5, 6], [7]]
    for _ in range(2 + 5):
        done = s.piece_done(big)
    assert done


@pytest.mark.parametrize("n_p,n_s,n_c,limit", [(1000, 64, 4096, 1e8), (100000, 64, 65536, 2e10),
                                               (5, 3, 7, 1.0), (1000, 10, 100, 1e12)])
def test_plan_pieces_cover_the_chunk(n_p, n_s, n_c, limit):
    parts = plan_pieces(n_p, n_s, n_c, limit)
    # every (particle, segment) pair exactly once
    seen = np.zeros((n_p, n_s), dtype=int)
    for a, b, p0, p1 in parts:
        assert 0 <= a < b <= n_s and 0 <= p0 < p1 <= n_p
        seen[p0:p1, a:b] += 1
    assert (seen == 1).all()
    works = [(p1 - p0) * (b - a) * n_c for a, b, p0, p1 in parts]
    if n_p * n_s * n_c <= limit:
        assert len(parts) == 1
    else:
        # steps are cut no finer than 16 (or the chunk's own length); parts stay
        # within the limit unless one particle-run alone exceeds it
        assert min(b - a for a, b, _, _ in parts) >= min(16, n_s)
        assert max(works) <= max(limit, n_c * 2 * 16) * 1.01


def test_work_counts_interactions():
    s = Scheduler({0: 1}, {0: 64}, 10, 1e9)
    r = s.add(Request(0, 1000, 7, 0.0))
    assert r.work == 1000 * 7 * 64


def test_detector_bytes_counts_accumulator_and_cells():
    spec = W.DetectorSpec(cells=np.zeros((12, 3)), t0=0.0, dt_det=1.0, n_t=100)
    assert detector_bytes(spec) == 12 * 100 * 48 + 12 * 32


def test_admission_counts_workspaces():
    """Admission counts each detector's own deposit workspaces beside its state,
    and the service reserves the two batch workspaces, bounded for every
    workgroup shape: for the plasma-mirror detector (65536 cells) and batches
    of 4e10 interactions, about 2e10 bytes of particle orders per batch
    workspace with the 8-cell tiles of shape 1."""
    import paper_2302_14812_amd as radio
    from paper_2302_14812_amd.serving import arena_bytes, resident_bytes, workspace_bytes
    spec = W.DetectorSpec(cells=np.zeros((65536, 3)), t0=0.0, dt_det=1.0, n_t=4096)
    ws = workspace_bytes(spec, 2e10)
    assert resident_bytes(spec, 2e10) == detector_bytes(spec) + ws
    a = arena_bytes(4e10, 4e10 / 4096)
    assert 2.4e10 <= a <= 3.5e10
    for cells, groups, run in radio.SHAPES.values():
        # a detector's time slices: two runs of the shape, particles as many as
        # make piece_work with more than two runs
        n_p = -(-int(2e10) // ((2 * run + 1) * 65536))
        assert ws >= (65536 // cells) * n_p * 4 + n_p * (2 * run + 1) * 80
        # a batch of one-step chunks of 10^5 particles on that detector: 4e10 / 6.5e9
        # of them, each with one order of 65536 / cells tiles x 10^5 particles and
        # 2 x 10^5 records
        n = 4e10 / (100_000 * 65536)
        assert a >= n * ((65536 // cells) * 100_000 * 4 + 2 * 100_000 * 80)
    # on a one-tile detector the segment bound holds the records: 4e10 / 4096 segments
    # of one-step chunks need 2 x 80 bytes each
    assert a >= 4e10 / 4096 * 160


def test_batches_respect_the_segment_bound():
    """On a detector of 16 cells a batch of 1e9 interactions would hold 6e7 particle
    segments; with a bound of 1e6 segments batches stop there."""
    s = Scheduler({0: 1}, {0: 16}, 10, 1e9, max_batch_segments=1e6)
    for k in range(8):
        s.add(Request(0, 100_000, 4, float(k)))  # 4e5 segments, 6.4e6 interactions each
    sizes = []
    while s.pending:
        s.admit()
        sizes.append(len(s.next_batch()))
    assert sizes == [2, 2, 2, 2]


def _stream(n, rate, seed, n_det=4, cells=256):
    offs = poisson_arrivals(rate, n, seed)
    sched_rows = list(W.stream_schedule(n, n_det, seed, max_log_particles=4.0))
    return [Request(d, npart, st, float(t)) for (d, _, st, npart), t in zip(sched_rows, offs)]


def test_light_load_latency_is_the_service_time():
    # one chunk at a time: each waits for nothing and takes its own service time
    s = make_sched(n_det=4, cells=256)
    reqs = [Request(k % 4, 100, 4, 10.0 * k) for k in range(20)]
    simulate(s, reqs, lambda ws: 1e-3 + sum(ws) / 1e9)
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
    simulate(s, reqs, lambda ws: overhead + sum(ws) / rate_cap)
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


def test_parts_bound_the_wait_behind_a_giant_chunk():
    """A giant chunk followed by small ones: cut into parts, it no longer delays them."""
    def stream():
        reqs = [Request(0, 100000, 64, 0.0)]  # 4.2e11 interactions at 65536 cells
        reqs += [Request(1 + k % 3, 1000, 8, 0.01 + 0.05 * k) for k in range(20)]
        return reqs

    def run(piece_work):
        s = make_sched(n_det=4, cells=65536, max_work=4e10)
        reqs = stream()
        simulate(s, reqs, lambda ws: 1e-3 + sum(ws) / 1e11, piece_work=piece_work)
        return reqs

    whole = run(None)
    cut = run(2e10)
    small_whole = max(r.latency for r in whole[1:])
    small_cut = max(r.latency for r in cut[1:])
    assert small_whole > 3.0           # stuck behind 4.2 s of work
    # at most the batches already on the device (two) and its own: 3 x 0.4 s
    assert small_cut < 3 * (1e-3 + 4e10 / 1e11) + 1e-6
    # the giant one finishes about when it would have
    assert cut[0].completion < 1.2 * whole[0].completion


def test_inflight_bound_holds():
    s = make_sched(n_det=2, cells=1)
    reqs = [Request(k % 2, 1, 1, 0.001 * k) for k in range(50)]
    simulate(s, reqs, lambda ws: 0.01, max_inflight=2)
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
    assert a.first_step == 40 and a.t_first == 0.0
    assert a.state_times()[0] == 40 * a.dt
    # every step is slower than light, and the sheet oscillates about x = 0
    step = np.linalg.norm(np.diff(a.x, axis=1), axis=0)
    assert step.max() < a.dt
    assert np.abs(a.x[0]).max() < 3.0
