"""The run-time mode on the device: the Boris push (radio_push) against the
oracle's pusher, and push-deposit blocks against one push and one deposit of
the whole run, and against the oracle's deposit of the same trajectory."""

import numpy as np
import pytest

import oracle
from paper_2302_14812_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import TOLS, check_parity  # noqa: E402

WAVE = {"wave_amplitude": 1.5, "wave_dir": [1.0, 0.0, 0.0], "wave_pol": [0.0, 1.0, 0.0],
        "wave_omega": 1.0, "wave_phase": 0.3}


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


def _initial(n_p, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = rng.normal(0.0, 0.5, size=(3, n_p))
    u0 = rng.normal(0.0, 0.2, size=(3, n_p))
    return x0, u0


@pytest.mark.parametrize("fields", [
    dict(WAVE),
    {"E": [0.02, -0.01, 0.05], "B": [0.0, 0.3, 0.1]},
    dict(WAVE, E=[0.0, 0.0, 0.01], B=[0.05, 0.0, 0.0]),
])
def test_push_matches_oracle(radio, fields):
    import torch
    x0, u0 = _initial(200, 7)
    n_s, dt = 400, 0.05
    x = torch.zeros((3, n_s + 1, 200), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(x)
    x[:, 0] = torch.from_numpy(x0).cuda()
    u[:, 0] = torch.from_numpy(u0).cuda()
    ch = radio.Chunk(x, u, None, 0.1, dt, 3)
    radio.push(ch, qm=-1.0, **fields)
    xo, uo = oracle.boris_push(x0, u0, -1.0, dt, n_s, fields, t_first=0.1, first_step=3)
    ex, eu = rel_l2(x.cpu().numpy(), xo), rel_l2(u.cpu().numpy(), uo)
    print(f"[push] {sorted(fields)}: relL2 x {ex:.2e} u {eu:.2e}", flush=True)
    assert max(ex, eu) <= 1e-12


def test_runtime_blocks_equal_one_shot_and_oracle(radio):
    import torch
    from paper_2302_14812_amd.runtime import RunTimeDiagnostic
    n_p, block, n_blocks, dt = 64, 16, 12, 0.05
    x0, u0 = _initial(n_p, 11)
    # the forward (Thomson) direction of the wave, at 200
    cells = W.sphere_cap_cells(200.0, [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], 6, 5, 0.3, 0.2)
    n_s = block * n_blocks
    xo, uo = oracle.boris_push(x0, u0, -1.0, dt, n_s, WAVE)
    ref_chunk = W.Chunk(x=xo, u=uo, q=np.full(n_p, -1.0), t_first=0.0, dt=dt)
    t0, dtd = W.arrival_window(cells, ref_chunk, 400, pad_frac=0.05)
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=400)
    dets = [radio.Detector.from_spec(spec, precision=p) for p in ("fp64", "mixed")]
    rt = RunTimeDiagnostic(dets, x0, u0, None, dt=dt, block_steps=block, fields=dict(WAVE, qm=-1.0))
    rt.advance(n_blocks)
    assert rt.step == n_s
    # one push of the whole run, one deposit
    x = torch.zeros((3, n_s + 1, n_p), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(x)
    x[:, 0] = torch.from_numpy(x0).cuda()
    u[:, 0] = torch.from_numpy(u0).cuda()
    whole = radio.push(radio.Chunk(x, u, None, 0.0, dt), qm=-1.0, **WAVE)
    xe, ue = rt.state()
    np.testing.assert_array_equal(xe.cpu().numpy(), x[:, -1].cpu().numpy())
    np.testing.assert_array_equal(ue.cpu().numpy(), u[:, -1].cpu().numpy())
    one = radio.Detector.from_spec(spec, precision="fp64")
    one.deposit(whole)
    E1, B1 = one.read()
    Eb, Bb = dets[0].read()
    torch.cuda.synchronize()
    e = max(rel_l2(Eb.cpu().numpy(), E1.cpu().numpy()), rel_l2(Bb.cpu().numpy(), B1.cpu().numpy()))
    print(f"[runtime] blocks vs one shot relL2 {e:.2e}", flush=True)
    assert e <= 1e-13
    # the oracle's deposit of the device's own trajectory
    dev_chunk = W.Chunk(x=x.cpu().numpy(), u=u.cpu().numpy(), q=np.full(n_p, -1.0), t_first=0.0,
                        dt=dt)
    Eo, Bo = oracle.read(oracle.deposit_workload(spec, dev_chunk))
    for d, tol in zip(dets, (1e-12, 1e-5)):
        Ed, Bd = d.read()
        torch.cuda.synchronize()
        assert np.abs(Eo).max() > 0
        check_parity(Ed.cpu().numpy(), Bd.cpu().numpy(), Eo, Bo, tol,
                     f"runtime {d.precision} vs oracle")
    for d in dets + [one]:
        d.close()


# sampled cells of the 128 x 128 cap: centre, corners and a seeded set
_RT_CELLS = tuple(sorted(set(W.grid_corner_cells(128, 128)) | set(
    np.random.Generator(np.random.PCG64(71)).choice(128 * 128, 11, replace=False).tolist())))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_runtime_as_benchmarked(radio, precision):
    """The run-time mode at the size and in the launch configuration the benchmark
    times: 10^4 electrons in the plane wave pushed 16 steps at a time for 64 blocks,
    each block deposited into the 128 x 128 cap (2048 slots) with the shipped
    run-time tuning, compared on sampled cells with the oracle's deposit of the
    same trajectory (one push of the whole run, equal to the blocks' pushes)."""
    import torch

    from paper_2302_14812_amd import autotune
    from paper_2302_14812_amd.runtime import RunTimeDiagnostic, plane_wave_electrons
    n_p, block, n_blocks, dt = 10000, 16, 64, 0.05
    cells, t0, dtd, n_t, x0, u0, wave = plane_wave_electrons(n_p, block, n_blocks, dt)
    cur = radio.get_tuning()
    try:
        det = radio.Detector(cells, t0=t0, dt_det=dtd, n_t=n_t, precision=precision)
        tuned = autotune.apply_runtime(det, n_p, block, precision)
        rt = RunTimeDiagnostic([det], x0, u0, None, dt=dt, block_steps=block, fields=wave)
        rt.advance(n_blocks)
        E, B = det.read()
        torch.cuda.synchronize()
        st = det.stats()
        print(f"[runtime] as benchmarked {precision}: shape "
              f"{radio.SHAPES[radio.get_tuning()['shape']]}{' (tuned)' if tuned else ''}, "
              f"large ring {st['large_ring'] / st['interactions']:.3f}, "
              f"clipped {st['clipped']}", flush=True)
        Eg = E[list(_RT_CELLS)].cpu().numpy()
        Bg = B[list(_RT_CELLS)].cpu().numpy()
        xe, ue = rt.state()
        xe, ue = xe.cpu().numpy(), ue.cpu().numpy()
        del E, B
        det.close()
    finally:
        radio.set_tuning(**cur)
    assert st["interactions"] == n_p * block * n_blocks * 128 * 128
    n_s = block * n_blocks
    x = torch.zeros((3, n_s + 1, n_p), dtype=torch.float64, device="cuda")
    u = torch.zeros_like(x)
    x[:, 0] = torch.from_numpy(x0).cuda()
    u[:, 0] = torch.from_numpy(u0).cuda()
    whole = radio.push(radio.Chunk(x, u, None, 0.0, dt), **wave)
    host = W.Chunk(x=whole.x.cpu().numpy(), u=whole.u.cpu().numpy(), q=np.full(n_p, -1.0),
                   t_first=0.0, dt=dt)
    del x, u, whole
    # the blocks pushed exactly what one push of the whole run gives
    np.testing.assert_array_equal(xe, host.x[:, -1])
    np.testing.assert_array_equal(ue, host.u[:, -1])
    spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t)
    Eo, Bo = oracle.read(oracle.deposit_workload(spec, host, cell_index=list(_RT_CELLS)))
    assert np.abs(Eo).max() > 0
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"runtime as benchmarked {precision} sampled")
