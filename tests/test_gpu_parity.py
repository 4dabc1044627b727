"""GPU parity: the HIP deposit against the CPU oracle on identical seeded inputs.

Bar for the double-precision path: relative L2 <= 1e-12, reported separately
for E and for B (the larger counts).  Arrival times, which the slot
coordinate amplifies, must match the oracle bit for bit.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2302_14812_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import TOL_FP64, TOLS, check_parity, rel_l2  # noqa: E402

PRECISIONS = pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_twosum"])


@pytest.fixture(scope="module")
def radio():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_14812_amd as radio
    radio._lib()  # a missing library raises here: no fallback
    return radio


def gpu_deposit(radio, spec, chunks, precision="fp64"):
    import torch
    det = radio.Detector.from_spec(spec, precision=precision)
    if not isinstance(chunks, (list, tuple)):
        chunks = [chunks]
    for ch in chunks:
        det.deposit(radio.Chunk.from_numpy(ch))
    E, B = det.read()
    torch.cuda.synchronize()
    st = det.stats()
    det.close()
    return E.cpu().numpy(), B.cpu().numpy(), st


def oracle_deposit(spec, chunk, cell_index=None):
    cnt = np.zeros(2, dtype=np.int64)
    D = oracle.deposit_workload(spec, chunk, cell_index=cell_index, counters=cnt)
    E, B = oracle.read(D)
    return E, B, cnt


def _window(cells, chunk, n_t, pad=0.05):
    t = chunk.state_times()
    lo, hi = np.inf, -np.inf
    for xc in cells:
        d = xc[:, None, None] - chunk.x
        tt = t[:, None] + np.sqrt((d * d).sum(axis=0))
        lo, hi = min(lo, tt.min()), max(hi, tt.max())
    w = hi - lo
    t0 = lo - pad * w
    return t0, (hi + pad * w - t0) / n_t


def test_arrival_times_bit_exact(radio, oracle_mod):
    import torch
    rng = np.random.Generator(np.random.PCG64(1))
    n = 3000
    scale = 10.0 ** rng.uniform(-1, 5, size=n)
    cells = rng.normal(size=(n, 3)) * scale[:, None]
    pts = rng.normal(size=(n, 3)) * rng.uniform(0, 100, size=(n, 1))
    t = rng.uniform(-50, 500, size=n)
    for c in (1.0, 0.7):
        out = radio.arrival_times(torch.from_numpy(cells).cuda(), torch.from_numpy(pts).cuda(),
                                  torch.from_numpy(t).cuda(), c=c).cpu().numpy()
        ref = np.array([oracle_mod.arrival(cells[i], pts[i], t[i], c) for i in range(n)])
        bad = np.flatnonzero(out != ref)
        assert bad.size == 0, (c, bad[:5], out[bad[:5]] - ref[bad[:5]])


def test_arrival_times_bit_exact_hard_cases(radio, oracle_mod):
    """Arrival times where the square root's rounding is hardest: distances along
    an axis (|d|^2 the rounded square of one coordinate, whose root lies next to
    a representable value), integer Pythagorean-like offsets, and magnitudes from
    1e-3 to 1e7; every one must equal the oracle's bit for bit."""
    import torch
    rng = np.random.Generator(np.random.PCG64(7))
    n = 30000
    pts = rng.normal(size=(3 * n, 3)) * rng.uniform(0, 10, size=(3 * n, 1))
    d = np.zeros((3 * n, 3))
    d[:n, 0] = 10.0 ** rng.uniform(-3, 7, size=n) * rng.choice([-1.0, 1.0], size=n)
    d[n:2 * n, :2] = rng.integers(-10 ** 6, 10 ** 6, size=(n, 2)).astype(np.float64)
    d[2 * n:] = rng.normal(size=(n, 3)) * (10.0 ** rng.uniform(-3, 7, size=(n, 1)))
    cells = pts + d
    t = rng.uniform(-50, 500, size=3 * n)
    out = radio.arrival_times(torch.from_numpy(cells).cuda(), torch.from_numpy(pts).cuda(),
                              torch.from_numpy(t).cuda(), c=1.0).cpu().numpy()
    ref = np.array([oracle_mod.arrival(cells[i], pts[i], t[i], 1.0) for i in range(3 * n)])
    bad = np.flatnonzero(out != ref)
    assert bad.size == 0, (bad[:5], out[bad[:5]] - ref[bad[:5]])


@pytest.mark.parametrize("dt_det", [1.2e-4, 0.0438, 0.04, 2.0 ** -10,
                                    # a significand of all ones (the host check sends
                                    # it to a division) and one unit below it (not)
                                    float(np.nextafter(2.0, 0.0)) * 2.0 ** -12,
                                    float(np.nextafter(np.nextafter(2.0, 0.0), 0.0)) * 2.0 ** -4])
def test_slot_coordinates_bit_exact(radio, oracle_mod, dt_det):
    """The slot coordinate (t_det - t0) / dt_det of the double deposit equals the
    oracle's correctly rounded division bit for bit: arrival times at the
    workloads' distances, and numerators that put the quotient within an ulp of
    a rounding midpoint (cell and point coincide, so t_det = t exactly)."""
    import torch
    from fractions import Fraction
    rng = np.random.Generator(np.random.PCG64(17))
    n = 4000
    cells = rng.normal(size=(n, 3)) * (10.0 ** rng.uniform(2, 5, size=(n, 1)))
    pts = rng.normal(size=(n, 3)) * rng.uniform(0, 30, size=(n, 1))
    t = rng.uniform(-50, 500, size=n)
    t0 = float(np.linalg.norm(cells, axis=1).min()) - 100.0
    out = radio.slot_coordinates(torch.from_numpy(cells).cuda(), torch.from_numpy(pts).cuda(),
                                 torch.from_numpy(t).cuda(), t0, dt_det).cpu().numpy()
    ref = np.array([oracle_mod.slot_of(oracle_mod.arrival(cells[i], pts[i], t[i]), t0, dt_det)
                    for i in range(n)])
    bad = np.flatnonzero(out != ref)
    assert bad.size == 0, (dt_det, bad[:5], out[bad[:5]] - ref[bad[:5]])
    # quotients next to rounding midpoints: x = RN(dt_det (q + ulp(q)/2)), +- an ulp
    m = 3000
    q = np.ldexp(1.0 + rng.uniform(size=m), rng.integers(-3, 20, size=m))
    half = 0.5 * (np.nextafter(q, np.inf) - q)
    x = np.array([float(Fraction(dt_det) * (Fraction(float(a)) + Fraction(float(h))))
                  for a, h in zip(q, half)])
    k = rng.integers(-1, 2, size=m)
    x = np.where(k > 0, np.nextafter(x, np.inf), np.where(k < 0, np.nextafter(x, -np.inf), x))
    p = rng.normal(size=(m, 3)) * 10.0
    out = radio.slot_coordinates(torch.from_numpy(p).cuda(), torch.from_numpy(p).cuda(),
                                 torch.from_numpy(x).cuda(), 0.0, dt_det).cpu().numpy()
    ref = np.array([oracle_mod.slot_of(v, 0.0, dt_det) for v in x])
    bad = np.flatnonzero(out != ref)
    assert bad.size == 0, (dt_det, bad[:5], out[bad[:5]] - ref[bad[:5]])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_parity_divisor_sent_to_division(radio, precision):
    """A slot width whose significand is all ones fails the host check of the
    two-correction quotient, so the double kernels divide: parity as usual."""
    chunk = W.random_chunk(29, 70, seed=13, dt=0.07, gamma_max=20.0, t_first=0.2)
    cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], 9, 7, 12.0, 9.0)
    t0, dtd0 = _window(cells, chunk, 180)
    dtd = float(np.ldexp(np.nextafter(2.0, 0.0), int(np.floor(np.log2(dtd0))) - 1))
    n_t = int(np.ceil(180 * dtd0 / dtd))
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t)
    Eg, Bg, _ = gpu_deposit(radio, spec, chunk, precision)
    Eo, Bo, _ = oracle_deposit(spec, chunk)
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"divided slot coordinate {precision}")


@PRECISIONS
def test_parity_circular_orbit(radio, precision):
    wl = W.circular_workload()
    Eg, Bg, st = gpu_deposit(radio, wl.detector, wl.chunk, precision)
    Eo, Bo, cnt = oracle_deposit(wl.detector, wl.chunk)
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"{wl.name} {precision}")
    assert st["interactions"] == wl.interactions
    assert st["clipped"] == cnt[0] and st["nonmonotone"] == cnt[1]


@pytest.mark.parametrize("seed,n_p,n_s,n_side,n_t,clip", [
    (1, 37, 77, (20, 15), 333, False),
    (2, 1, 1, (3, 1), 5, False),
    (3, 17, 33, (16, 16), 64, True),
    (4, 50, 64, (1, 1), 1, True),
    (5, 33, 95, (17, 31), 200, True),
])
@PRECISIONS
def test_parity_random_ragged(radio, precision, seed, n_p, n_s, n_side, n_t, clip):
    chunk = W.random_chunk(n_p, n_s, seed=seed, dt=0.07, gamma_max=30.0, t_first=0.3 * seed)
    cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], n_side[0], n_side[1],
                          12.0, 9.0)
    t0, dtd = _window(cells, chunk, n_t)
    if clip:  # cut both ends of the arrival interval
        t0 += 0.2 * n_t * dtd
        dtd *= 0.6
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t)
    Eg, Bg, st = gpu_deposit(radio, spec, chunk, precision)
    Eo, Bo, cnt = oracle_deposit(spec, chunk)
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"random seed={seed} {precision}")
    assert st["clipped"] == cnt[0] and st["nonmonotone"] == cnt[1]
    if clip:
        assert cnt[0] > 0


@pytest.mark.parametrize("shape", [1, 2])
@PRECISIONS
def test_workgroup_shapes_match_oracle(radio, precision, shape):
    """The other workgroup shapes (8 cells x 32 particles x runs of 16; 16 cells x 16
    particles x runs of 8) on ragged random, clipped, undulator and plasma-mirror
    cases, single deposits and a batch, against the oracle; a detector with
    options keeps the default shape."""
    cur = radio.get_tuning()
    cases = []
    for seed, n_p, n_s, side, n_t, clip in ((1, 37, 77, (20, 15), 333, False),
                                            (5, 33, 95, (17, 31), 200, True)):
        chunk = W.random_chunk(n_p, n_s, seed=seed, dt=0.07, gamma_max=30.0, t_first=0.3 * seed)
        cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], side[0], side[1],
                              12.0, 9.0)
        t0, dtd = _window(cells, chunk, n_t)
        if clip:
            t0 += 0.2 * n_t * dtd
            dtd *= 0.6
        cases.append((f"random seed={seed}", W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t),
                      chunk))
    und = W.undulator_workload(n_particles=300, n_steps=200, n_side=24, n_t=512)
    pm = W.plasma_mirror_workload(n_particles=400, n_steps=150, n_side=16, n_t=1024)
    cases += [(und.name, und.detector, und.chunk), (pm.name, pm.detector, pm.chunk)]
    try:
        radio.set_tuning(shape=shape)
        for name, spec, chunk in cases:
            Eg, Bg, st = gpu_deposit(radio, spec, chunk, precision)
            Eo, Bo, cnt = oracle_deposit(spec, chunk)
            check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"shape {shape} {name} {precision}")
            assert st["clipped"] == cnt[0] and st["nonmonotone"] == cnt[1]
        # the same cases in one batch
        import torch
        dets = [radio.Detector.from_spec(spec, precision=precision) for _, spec, _ in cases]
        radio.deposit_batch(dets, [radio.Chunk.from_numpy(c) for _, _, c in cases])
        for d, (name, spec, chunk) in zip(dets, cases):
            E, B = d.read()
            torch.cuda.synchronize()
            Eo, Bo, _ = oracle_deposit(spec, chunk)
            check_parity(E.cpu().numpy(), B.cpu().numpy(), Eo, Bo, TOLS[precision],
                         f"shape {shape} batch {name} {precision}")
            d.close()
        # a detector with options takes the default shape and stays correct
        name, spec, chunk = cases[1]
        det = radio.Detector.from_spec(spec, precision=precision, options=radio.HOLD_LINEAR)
        det.deposit(radio.Chunk.from_numpy(chunk))
        E, B = det.read()
        torch.cuda.synchronize()
        det.close()
        Do = oracle.deposit_workload(spec, chunk, options=oracle.HOLD_LINEAR)
        Eo, Bo = oracle.read(Do)
        check_parity(E.cpu().numpy(), B.cpu().numpy(), Eo, Bo, TOLS[precision],
                     f"shape {shape} with options (default shape) {precision}")
    finally:
        radio.set_tuning(**cur)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deposit_in_several_launches(radio, precision):
    """Work items beyond one launch's grid (max_grid) run as further launches with
    an item offset: the result equals the single launch and the oracle."""
    chunk = W.random_chunk(33, 95, seed=5, dt=0.07, gamma_max=30.0, t_first=1.5)
    cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], 17, 31, 12.0, 9.0)
    t0, dtd = _window(cells, chunk, 200)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=200)
    E1, B1, _ = gpu_deposit(radio, spec, chunk, precision)
    cur = radio.get_tuning()
    try:
        radio.set_tuning(max_grid=24)  # 33 tiles x 6 runs = 198 items: 9 launches of 24
        E2, B2, st = gpu_deposit(radio, spec, chunk, precision)
    finally:
        radio.set_tuning(**cur)
    assert st["interactions"] == 33 * 95 * 17 * 31
    e = max(rel_l2(E2, E1), rel_l2(B2, B1))
    print(f"[launches] {precision}: several launches vs one relL2 {e:.3e}", flush=True)
    assert e <= (1e-13 if precision == "fp64" else 1e-6)
    Eo, Bo, _ = oracle_deposit(spec, chunk)
    check_parity(E2, B2, Eo, Bo, TOLS[precision], f"several launches {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deposit_in_particle_parts(radio, precision):
    """A short chunk (two runs) of many particles on few tiles: the automatic
    plan cuts each tile's sorted particles into parts (here seven of 125 batches);
    the result equals a deposit with one item per tile and the oracle."""
    chunk = W.random_chunk(2000, 20, seed=11, dt=0.07, gamma_max=30.0, t_first=0.4)
    cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], 8, 8, 12.0, 9.0)
    t0, dtd = _window(cells, chunk, 300)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=300)
    E1, B1, st = gpu_deposit(radio, spec, chunk, precision)
    cur = radio.get_tuning()
    try:
        radio.set_tuning(target_blocks=1)  # one item per tile: no parts
        E2, B2, _ = gpu_deposit(radio, spec, chunk, precision)
    finally:
        radio.set_tuning(**cur)
    assert st["interactions"] == 2000 * 20 * 64
    e = max(rel_l2(E1, E2), rel_l2(B1, B2))
    print(f"[parts] {precision}: particle parts vs one item per tile relL2 {e:.3e}", flush=True)
    assert e <= (1e-13 if precision == "fp64" else 1e-6)
    Eo, Bo, _ = oracle_deposit(spec, chunk)
    check_parity(E1, B1, Eo, Bo, TOLS[precision], f"particle parts {precision}")


@PRECISIONS
def test_parity_undulator_small(radio, precision):
    wl = W.undulator_workload(n_particles=64, n_steps=600, n_side=24, n_t=512)
    Eg, Bg, _ = gpu_deposit(radio, wl.detector, wl.chunk, precision)
    Eo, Bo, _ = oracle_deposit(wl.detector, wl.chunk)
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"{wl.name} {precision}")


@PRECISIONS
def test_parity_plasma_mirror_small(radio, precision):
    wl = W.plasma_mirror_workload(n_particles=300, n_steps=250, n_side=16, n_t=1024)
    Eg, Bg, _ = gpu_deposit(radio, wl.detector, wl.chunk, precision)
    Eo, Bo, _ = oracle_deposit(wl.detector, wl.chunk)
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"{wl.name} {precision}")


def test_edge_cases(radio):
    import torch
    chunk = W.random_chunk(4, 20, seed=8, dt=0.05, gamma_max=5.0)
    cells = W.plane_cells([0, 0, 20.0], [1, 0, 0], [0, 1, 0], 5, 4, 3.0, 3.0)
    t0, dtd = _window(cells, chunk, 50)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=50)
    # every arrival before the window: nothing lands, everything counted clipped
    late = W.DetectorSpec(cells=cells, t0=t0 + 1e3, dt_det=dtd, n_t=50)
    Eg, Bg, st = gpu_deposit(radio, late, chunk)
    assert np.abs(Eg).max() == 0.0 and np.abs(Bg).max() == 0.0
    assert st["clipped"] == chunk.n_particles * chunk.n_steps * cells.shape[0]
    # every arrival after the window
    early = W.DetectorSpec(cells=cells, t0=t0 - 1e3, dt_det=dtd, n_t=50)
    Eg, Bg, _ = gpu_deposit(radio, early, chunk)
    Eo, Bo, _ = oracle_deposit(early, chunk)
    check_parity(Eg, Bg, Eo, Bo, TOL_FP64, "window before arrivals")
    # NULL charges mean electrons
    det = radio.Detector.from_spec(spec)
    det2 = radio.Detector.from_spec(spec)
    c1 = radio.Chunk.from_numpy(chunk)
    c_none = radio.Chunk(c1.x, c1.u, None, chunk.t_first, chunk.dt)
    c_neg = radio.Chunk(c1.x, c1.u, torch.full((chunk.n_particles,), -1.0, dtype=torch.float64,
                                               device="cuda"), chunk.t_first, chunk.dt)
    det.deposit(c_none)
    det2.deposit(c_neg)
    E1, B1 = det.read()
    E2, B2 = det2.read()
    assert torch.equal(E1, E2) and torch.equal(B1, B2)
    # empty chunks are valid no-ops
    before = det.read()[0].clone()
    empty = radio.Chunk(c1.x[:, :1, :].contiguous(), c1.u[:, :1, :].contiguous(), c1.q, 0.0,
                        0.1)  # zero segments
    det.deposit(empty)
    nop = radio.Chunk(c1.x[:, :, :0].contiguous(), c1.u[:, :, :0].contiguous(), None, 0.0, 0.1)
    det.deposit(nop)
    assert torch.equal(det.read()[0], before)
    # invalid chunks are rejected and change nothing
    bad = radio.Chunk(c1.x, c1.u, c1.q, chunk.t_first, 0.0)
    with pytest.raises(radio.RadioError) as ei:
        det.deposit(bad)
    assert ei.value.status == radio.EINVAL
    bad = radio.Chunk(c1.x, c1.u, c1.q, float("nan"), 0.1)
    with pytest.raises(radio.RadioError):
        det.deposit(bad)
    assert torch.equal(det.read()[0], before)
    # reset
    det.reset()
    E0, B0 = det.read()
    assert float(E0.abs().max()) == 0.0 and float(B0.abs().max()) == 0.0
    assert det.stats()["interactions"] == 0
    det.close()
    det2.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_state_at_a_cell(radio, precision):
    """A degenerate case of Eq. 1: a particle passing exactly through a cell
    (R = 0 at one state).  The field of the segment that ends there is not
    finite in the definition, so the slots it covers at that cell are not
    finite in the oracle; the device must leave exactly those slots non-finite
    and match the oracle everywhere else (the segment that starts at that
    state has a finite field and a finite arrival interval)."""
    chunk = W.random_chunk(3, 40, seed=31, dt=0.05, gamma_max=8.0)
    cells = W.plane_cells([0, 0, 20.0], [1, 0, 0], [0, 1, 0], 5, 4, 3.0, 3.0)
    # particle 0 in uniform motion along x at beta = 1/2, at cell 7 at state 12
    beta = 0.5
    chunk.u[:, :, 0] = 0.0
    chunk.u[0, :, 0] = beta / math.sqrt(1.0 - beta * beta)
    s = np.arange(chunk.n_steps + 1)
    chunk.x[0, :, 0] = cells[7, 0] + beta * (s - 12) * chunk.dt
    chunk.x[1, :, 0] = cells[7, 1]
    chunk.x[2, :, 0] = cells[7, 2]
    assert np.array_equal(chunk.x[:, 12, 0], cells[7])
    t0, dtd = _window(cells, chunk, 120)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=120)
    with np.errstate(all="ignore"):
        Eo, Bo, _ = oracle_deposit(spec, chunk)
    Eg, Bg, _ = gpu_deposit(radio, spec, chunk, precision=precision)
    for g, o, what in ((Eg, Eo, "E"), (Bg, Bo, "B")):
        bad_o = ~np.isfinite(o).all(axis=2)
        bad_g = ~np.isfinite(g).all(axis=2)
        assert bad_o.any() and set(np.nonzero(bad_o)[0]) == {7}
        assert np.array_equal(bad_g, bad_o), (what, np.nonzero(bad_g), np.nonzero(bad_o))
    ok = np.isfinite(Eo).all(axis=2) & np.isfinite(Bo).all(axis=2)
    check_parity(Eg[ok], Bg[ok], Eo[ok], Bo[ok], TOLS[precision],
                 f"state at a cell {precision} (finite slots)")


@pytest.mark.parametrize("precision,options", [("fp64", 0), ("fp64", 4), ("fp64", 8), ("mixed", 0)])
def test_time_slices_equal_whole_chunk(radio, precision, options):
    """A chunk whose per-tile particle orders (at most two runs each) exceed the
    order budget is deposited in time slices, each reading its neighbour states
    for betadot: the result is the whole chunk's up to summation order, for every
    hold rule (options 4, 8: previous, linear), and the oracle's."""
    import torch
    chunk = W.random_chunk(2000, 150, seed=41, dt=0.05, gamma_max=10.0)
    cells = W.plane_cells([0, 0, 30.0], [1, 0, 0], [0, 1, 0], 32, 32, 6.0, 6.0)
    t0, dtd = W.arrival_window(cells, chunk, 400, pad_frac=0.05,
                               cell_index=W.grid_corner_cells(32, 32), seed=41)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=400)

    def run():
        det = radio.Detector.from_spec(spec, precision=precision, options=options)
        det.deposit(radio.Chunk.from_numpy(chunk))
        E, B = det.read()
        torch.cuda.synchronize()
        slices = det.stats()["slices"]
        det.close()
        return E.cpu().numpy(), B.cpu().numpy(), slices

    cur = radio.get_tuning()
    try:
        Ew, Bw, n_whole = run()
        # 64 tiles x 2000 particles x 4 bytes: one MiB holds two orders, so the
        # ten runs go in three slices of four, four and two
        radio.set_tuning(order_budget_mib=1)
        Es, Bs, n_sliced = run()
    finally:
        radio.set_tuning(**cur)
    assert (n_whole, n_sliced) == (1, 3)
    check_parity(Es, Bs, Ew, Bw, 1e-13, f"time slices vs whole chunk {precision} options={options}")
    if options == 0:
        Eo, Bo, _ = oracle_deposit(spec, chunk)
        check_parity(Es, Bs, Eo, Bo, TOLS[precision], f"time slices vs oracle {precision}")


def test_time_slices_with_particle_parts(radio):
    """Time slices of a chunk on few tiles, where each slice's work items also cut
    the sorted particles into parts: 5 x 10^4 particles on 8 x 8 cells (4 tiles,
    800 kB per order), so a 1 MiB budget holds one order and the ten runs go in
    five slices of two.  Same result as the whole chunk, and the oracle's."""
    import torch
    chunk = W.random_chunk(50000, 150, seed=43, dt=0.05, gamma_max=10.0)
    cells = W.plane_cells([0, 0, 30.0], [1, 0, 0], [0, 1, 0], 8, 8, 6.0, 6.0)
    t0, dtd = W.arrival_window(cells, chunk, 400, pad_frac=0.05,
                               cell_index=W.grid_corner_cells(8, 8), seed=43)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=400)

    def run():
        det = radio.Detector.from_spec(spec, precision="fp64")
        det.deposit(radio.Chunk.from_numpy(chunk))
        E, B = det.read()
        torch.cuda.synchronize()
        slices = det.stats()["slices"]
        det.close()
        return E.cpu().numpy(), B.cpu().numpy(), slices

    cur = radio.get_tuning()
    try:
        Ew, Bw, n_whole = run()
        radio.set_tuning(order_budget_mib=1)
        Es, Bs, n_sliced = run()
    finally:
        radio.set_tuning(**cur)
    assert (n_whole, n_sliced) == (1, 5)
    check_parity(Es, Bs, Ew, Bw, 1e-13, "time slices with particle parts vs whole chunk")
    Eo, Bo, _ = oracle_deposit(spec, chunk)
    check_parity(Es, Bs, Eo, Bo, TOL_FP64, "time slices with particle parts vs oracle")


def test_chunk_split_and_superposition(radio):
    chunk = W.random_chunk(23, 150, seed=12, dt=0.04, gamma_max=20.0)
    cells = W.plane_cells([0, 3.0, 40.0], [1, 0, 0], [0, 1, 0], 13, 11, 8.0, 8.0)
    t0, dtd = _window(cells, chunk, 300)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=300)
    parts = W.split_steps(chunk, [1, 40, 41, 99])
    parts += [parts.pop(0)]  # out of order
    Eg, Bg, st = gpu_deposit(radio, spec, parts)
    assert st["chunks"] == len(parts)
    D = np.zeros((cells.shape[0], 300, 6))
    for part in parts:
        oracle.deposit_workload(spec, part, D=D)
    Eo, Bo = oracle.read(D)
    check_parity(Eg, Bg, Eo, Bo, TOL_FP64, "chunk split vs oracle of the same parts")
    # against the unsplit chunk: the parts keep the state times of the whole
    # (first_step), so only the order of the additions differs
    Eu, Bu, _ = oracle_deposit(spec, chunk)
    check_parity(Eg, Bg, Eu, Bu, TOL_FP64, "chunk split vs unsplit")
    # device-side slicing of a device chunk gives the same parts
    dev = radio.Chunk.from_numpy(chunk)
    dparts = [dev.slice_steps(0, 40), dev.slice_steps(40, 99), dev.slice_steps(99, 150)]
    assert [p.first_step for p in dparts] == [0, 40, 99]
    det = radio.Detector.from_spec(spec, precision="fp64")
    for p in dparts[::-1]:
        det.deposit(p)
    E2, B2 = det.read()
    check_parity(E2.cpu().numpy(), B2.cpu().numpy(), Eu, Bu, TOL_FP64, "device step slices")
    det.close()
    halves = [chunk.slice_particles(0, 10), chunk.slice_particles(10, 23)]
    Eg, Bg, _ = gpu_deposit(radio, spec, halves)
    check_parity(Eg, Bg, Eu, Bu, TOL_FP64, "particle split")


def test_generated_geometries_match_generators(radio):
    p = radio.Detector.plane([1.0, 2.0, 300.0], [1, 0, 0], [0, 2, 0], 7, 5, 40.0, 30.0,
                             t0=0.0, dt_det=1.0, n_t=4)
    np.testing.assert_allclose(p.cells(), W.plane_cells([1.0, 2.0, 300.0], [1, 0, 0], [0, 2, 0],
                                                         7, 5, 40.0, 30.0), rtol=1e-14, atol=1e-12)
    s = radio.Detector.sphere(1e5, [-1, 1, 0], [1, 1, 0.3], 6, 9, 0.1, 0.05,
                              t0=0.0, dt_det=1.0, n_t=4)
    np.testing.assert_allclose(s.cells(), W.sphere_cap_cells(1e5, [-1, 1, 0], [1, 1, 0.3], 6, 9,
                                                             0.1, 0.05), rtol=1e-13, atol=1e-8)
    p.close()
    s.close()


@PRECISIONS
def test_full_size_undulator_sampled_cells(radio, precision):
    """The benchmark workload at full size, in the launch configuration the benchmark
    times, compared on sampled cells (corners, centre, and a seeded random set)."""
    import torch
    wl = _undulator_full()
    det = radio.Detector.from_spec(wl.detector, precision=precision)
    ch = radio.Chunk.from_numpy(wl.chunk)
    det.deposit(ch)
    E, B = det.read()
    torch.cuda.synchronize()
    n1, n2 = wl.detector.grid
    rng = np.random.Generator(np.random.PCG64(99))
    idx = sorted(set(W.grid_corner_cells(n1, n2)) | set(rng.choice(n1 * n2, 11, replace=False).tolist()))
    Eg = E[idx].cpu().numpy()
    Bg = B[idx].cpu().numpy()
    del E, B, ch
    det.close()
    Eo, Bo, _ = _undulator_oracle(tuple(idx))
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"{wl.name} sampled {precision}")


@pytest.mark.parametrize("names", ["FAR_FIELD", "FAR_FIELD ACCEL_ONLY", "HOLD_PREVIOUS",
                                   "HOLD_LINEAR"])
def test_full_size_undulator_options_sampled_cells(radio, names):
    """The detector options as the benchmark's options leg runs them: the full
    undulator workload in mixed precision with the far field (Eq. 3), the far field
    with the acceleration term alone, the previous state's field held and the
    linear interpolation, each compared with the oracle under the same option on
    sampled cells."""
    import dataclasses
    import torch
    wl = _undulator_full()
    options = 0
    for n in names.split():
        options |= getattr(radio, n)
    det = radio.Detector.from_spec(wl.detector, precision="mixed", options=options)
    ch = radio.Chunk.from_numpy(wl.chunk)
    det.deposit(ch)
    E, B = det.read()
    torch.cuda.synchronize()
    idx = list(_OPT_CELLS)
    Eg = E[idx].cpu().numpy()
    Bg = B[idx].cpu().numpy()
    del E, B, ch
    det.close()
    spec = dataclasses.replace(wl.detector, options=options)
    Eo, Bo, _ = oracle_deposit(spec, wl.chunk, cell_index=idx)
    check_parity(Eg, Bg, Eo, Bo, TOLS["mixed"], f"{wl.name} options={options} sampled mixed")


# sampled cells of the 128 x 128 undulator detector for the options: centre and corners,
# and a seeded set
_OPT_CELLS = tuple(sorted(set(W.grid_corner_cells(128, 128)) | set(
    np.random.Generator(np.random.PCG64(97)).choice(128 * 128, 5, replace=False).tolist())))


@PRECISIONS
def test_plasma_mirror_full_detector_sampled_cells(radio, precision):
    """The plasma-mirror configuration at its full detector (256 x 256 cells, 4096
    slots) and length (1000 steps over 10 laser periods), with 2 x 10^4 of its
    2 x 10^5 electrons, in every precision, compared on sampled cells.  Its
    particle orders at two runs each exceed the default budget, so the chunk runs
    as time slices (here eleven)."""
    import time
    import torch
    wl = _plasma_full()
    det = radio.Detector.from_spec(wl.detector, precision=precision)
    ch = radio.Chunk.from_numpy(wl.chunk)
    torch.cuda.synchronize()
    t = time.perf_counter()
    det.deposit(ch)
    E, B = det.read()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    st = det.stats()
    print(f"[parity] {wl.name}: {st['slices']} slices, {wl.interactions / dt:.3e} interactions/s "
          f"(first call), bypassed/int {st['bypassed'] / st['interactions']:.2e}", flush=True)
    assert st["slices"] > 1
    n1, n2 = wl.detector.grid
    Eg = E[list(_PM_CELLS)].cpu().numpy()
    Bg = B[list(_PM_CELLS)].cpu().numpy()
    del E, B, ch
    det.close()
    Eo, Bo, _ = _plasma_oracle()
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"{wl.name} sampled {precision}")


@pytest.mark.parametrize("precision,n_steps", [("mixed", 1000), ("fp64", 500)])
def test_plasma_mirror_full_size_as_benchmarked(radio, precision, n_steps):
    """The plasma-mirror configuration at its stated size -- 2 x 10^5 electrons, 256 x
    256 cells, 4096 slots; all 1000 steps in mixed precision and the first 500 in
    double, as the benchmark runs them -- in the launch configuration the benchmark
    times (the shipped tuning: the 8 x 32 x 16 workgroup shape; time slices of its
    particle orders, 1.6e9 entries per order of two runs over the 8192 tiles),
    compared with the oracle on sampled cells."""
    import torch

    from paper_2302_14812_amd import autotune
    wl = W.plasma_mirror_workload(n_particles=200_000, n_steps=1000)
    if n_steps < wl.chunk.n_steps:
        wl.chunk = wl.chunk.slice_steps(0, n_steps)
    cur = radio.get_tuning()
    try:
        ch = radio.Chunk.from_numpy(wl.chunk)
        tuned = autotune.apply_single(wl.detector, ch, precision)
        det = radio.Detector.from_spec(wl.detector, precision=precision)
        det.deposit(ch)
        E, B = det.read()
        torch.cuda.synchronize()
        st = det.stats()
        print(f"[parity] plasma mirror 2e5 e- x {n_steps} steps {precision}: shape "
              f"{radio.SHAPES[radio.get_tuning()['shape']]}{' (tuned)' if tuned else ''}, "
              f"{st['slices']} slices, large ring {st['large_ring'] / st['interactions']:.3f}",
              flush=True)
        Eg = E[list(_PM_CELLS)].cpu().numpy()
        Bg = B[list(_PM_CELLS)].cpu().numpy()
        del E, B, ch
        det.close()
    finally:
        radio.set_tuning(**cur)
    assert st["interactions"] == 200_000 * n_steps * 65536
    assert st["slices"] > 1
    Eo, Bo, _ = oracle_deposit(wl.detector, wl.chunk, cell_index=list(_PM_CELLS))
    del wl
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"plasma mirror full size sampled {precision}")


_CACHE = {}
# sampled cells of the 256 x 256 plasma-mirror detector: corners, centre, and a seeded set
_PM_CELLS = tuple(sorted(set(W.grid_corner_cells(256, 256)) | set(
    np.random.Generator(np.random.PCG64(98)).choice(256 * 256, 11, replace=False).tolist())))


def _plasma_full():
    if "pm" not in _CACHE:
        _CACHE["pm"] = W.plasma_mirror_workload(n_particles=20_000, n_steps=1000)
    return _CACHE["pm"]


def _plasma_oracle():
    if "pm_oracle" not in _CACHE:
        wl = _plasma_full()
        _CACHE["pm_oracle"] = oracle_deposit(wl.detector, wl.chunk, cell_index=list(_PM_CELLS))
    return _CACHE["pm_oracle"]


def _undulator_full():
    if "wl" not in _CACHE:
        _CACHE["wl"] = W.undulator_workload()
    return _CACHE["wl"]


def _undulator_oracle(idx):
    key = ("oracle", idx)
    if key not in _CACHE:
        wl = _undulator_full()
        _CACHE[key] = oracle_deposit(wl.detector, wl.chunk, cell_index=list(idx))
    return _CACHE[key]
