"""The streaming deposit service on the device.

Chunks of a Poisson stream, served in continuous batches that mix
detectors, must leave every detector with the fields it gets when its
chunks are deposited alone, one by one (up to the order of floating-point
additions), and with the oracle's fields on sampled cells.  A memory budget
that holds three detectors admits the rest only as earlier ones finish.
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
def stream():
    """Five uneven plasma-mirror detectors and a 40-chunk stream over them."""
    specs = {d: W.plasma_mirror_detector(n_side=side, n_t=nt, sample_particles=16)
             for d, (side, nt) in enumerate([(6, 128), (10, 256), (16, 192), (4, 512), (12, 64)])}
    rows = list(W.stream_schedule(40, len(specs), seed=W.BASE_SEED + 50, max_steps=48,
                                  min_log_particles=1.5, max_log_particles=3.0))
    host = [(d, W.plasma_mirror_chunk(n, s0, st, seed=W.BASE_SEED + 100 + k))
            for k, (d, s0, st, n) in enumerate(rows)]
    return specs, host


def _alone(radio, spec, chunks, precision):
    import torch
    det = radio.Detector.from_spec(spec, precision=precision)
    for c in chunks:
        det.deposit(c)
    E, B = det.read()
    torch.cuda.synchronize()
    out = E.cpu().numpy(), B.cpu().numpy()
    det.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_mix_equals_alone_and_oracle(radio, stream, precision):
    from paper_2302_14812_amd.serving import DepositServer, poisson_arrivals, replay
    specs, host = stream
    dev = [(d, radio.Chunk.from_numpy(c)) for d, c in host]
    offsets = poisson_arrivals(400.0, len(dev), seed=7)
    # parts of at most 1e6 interactions: the larger chunks are cut by steps and
    # particles and their parts interleave with other chunks across batches
    with DepositServer(specs, precision=precision, max_batch_work=4e6, piece_work=1e6) as srv:
        reqs = replay(srv, dev, offsets)
        srv.drain(timeout=60)
        got = {d: srv.finish(d, timeout=60) for d in specs}
        st = srv.summary()
    print(f"[serve] {precision}: {st}", flush=True)
    assert st["chunks"] == len(dev)
    assert max(len(r.pieces) for r in reqs) > 3 and st["batches"] > 5
    rng = np.random.Generator(np.random.PCG64(11))
    tol_alone = 1e-13 if precision == "fp64" else 1e-6
    for d, spec in specs.items():
        mine = [c for dd, c in dev if dd == d]
        Ea, Ba = _alone(radio, spec, mine, precision)
        Es, Bs = got[d]
        e = max(rel_l2(Es, Ea), rel_l2(Bs, Ba))
        print(f"[serve] {precision} det {d}: {len(mine)} chunks, served vs alone {e:.3e}",
              flush=True)
        assert e <= tol_alone, (d, e)
        idx = sorted(rng.choice(spec.n_cells, size=min(4, spec.n_cells), replace=False).tolist())
        D = None
        for dd, c in host:
            if dd == d:
                D = oracle.deposit_workload(spec, c, cell_index=idx, D=D)
        if D is None:
            assert np.abs(Es).max() == 0.0
            continue
        Eo, Bo = oracle.read(D)
        check_parity(Es[idx], Bs[idx], Eo, Bo, 1e-12 if precision == "fp64" else 1e-5,
                     f"served {precision} det {d} vs oracle")


def test_memory_budget_admits_three_at_a_time(radio, stream):
    from paper_2302_14812_amd.serving import DepositServer, arena_bytes, resident_bytes
    specs, host = stream
    # five detectors of equal size; room for three beside the batch workspaces
    spec = W.plasma_mirror_detector(n_side=8, n_t=128, sample_particles=16)
    specs5 = {d: spec for d in range(5)}
    work = 4e10  # the server's default batch size; parts of half of it
    arenas = 2 * arena_bytes(work, work / 4096)
    budget = 3 * resident_bytes(spec, work / 2) + arenas + 100
    chunks = [radio.Chunk.from_numpy(c) for _, c in host[:10]]
    order = [0, 1, 2, 0, 1, 2, 3, 4, 3, 4]
    with DepositServer(specs5, precision="fp64", memory_budget=budget) as srv:
        for d, c in zip(order, chunks):
            srv.submit(d, c)
        srv.finish(0, timeout=60)
        srv.finish(1, timeout=60)
        res = {d: srv.finish(d, timeout=60) for d in (2, 3, 4)}
        st = srv.summary()
    print(f"[serve] budget: {st}", flush=True)
    assert st["peak_resident"] == 3 and st["peak_bytes"] <= budget - arenas
    assert st["chunks"] == 10
    for d in range(2, 5):
        mine = [c for dd, c in zip(order, chunks) if dd == d]
        Ea, Ba = _alone(radio, spec, mine, "fp64")
        assert max(rel_l2(res[d][0], Ea), rel_l2(res[d][1], Ba)) <= 1e-13


def test_finish_of_idle_detector_reads_zero_and_late_submit_fails(radio, stream):
    from paper_2302_14812_amd.serving import DepositServer
    specs, host = stream
    with DepositServer({0: specs[0], 1: specs[1]}, precision="fp64") as srv:
        E, B = srv.finish(1, timeout=10)
        assert E.shape == (specs[1].n_cells, specs[1].n_t, 3) and not E.any() and not B.any()
        with pytest.raises(ValueError):
            srv.submit(1, radio.Chunk.from_numpy(host[0][1]))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_as_benchmarked(radio, precision):
    """The service at the shape the benchmark's serving leg runs: eight resident
    plasma-mirror detectors of 256 x 256 cells x 4096 slots (12.9 GB each), a
    Poisson stream of chunks of 1-64 steps x 10^3-10^5 fresh electrons of the
    sheet, the server's default batch and part sizes.  Every detector's fields,
    read on the device, match the oracle's deposit of the chunks it received on
    sampled cells."""
    import torch

    from paper_2302_14812_amd.serving import DepositServer, poisson_arrivals, replay
    from parity import TOLS
    n_det = 8
    specs = {d: W.plasma_mirror_detector(n_side=256, n_t=4096, seed=W.BASE_SEED + 3 + d)
             for d in range(n_det)}
    rows = list(W.stream_schedule(24, n_det, seed=W.BASE_SEED + 500, min_steps=1, max_steps=64,
                                  min_log_particles=3.0, max_log_particles=5.0))
    host = [(d, W.plasma_mirror_chunk(n, s0, st, seed=W.BASE_SEED + 1000 + k))
            for k, (d, s0, st, n) in enumerate(rows)]
    dev = [(d, radio.Chunk.from_numpy(c)) for d, c in host]
    offsets = poisson_arrivals(20.0, len(dev), seed=W.BASE_SEED + 501)
    rng = np.random.Generator(np.random.PCG64(13))
    idx = sorted(set(W.grid_corner_cells(256, 256)) |
                 set(rng.choice(256 * 256, 3, replace=False).tolist()))
    fed = {d for d, _ in host}
    got = {}
    with DepositServer(specs, precision=precision) as srv:
        replay(srv, dev, offsets)
        srv.drain(timeout=300)
        for d in specs:
            if d not in fed:
                srv.finish(d, timeout=300, read="none")
                continue
            Et, Bt = srv.finish(d, timeout=300, read="device")
            got[d] = (Et[idx].cpu().numpy(), Bt[idx].cpu().numpy())
            del Et, Bt
            torch.cuda.empty_cache()
        st = srv.summary()
    del dev
    print(f"[serve] as benchmarked {precision}: {st['chunks']} chunks, {st['batches']} batches, "
          f"peak {st['peak_resident']} detectors, {st['peak_bytes'] / 1e9:.1f} GB", flush=True)
    assert st["chunks"] == len(host) and st["peak_resident"] == len(fed)
    for d, spec in specs.items():
        if d not in fed:
            continue
        D = None
        for dd, c in host:
            if dd == d:
                D = oracle.deposit_workload(spec, c, cell_index=idx, D=D)
        Eo, Bo = oracle.read(D)
        check_parity(*got[d], Eo, Bo, TOLS[precision], f"served as benchmarked {precision} det {d}")
