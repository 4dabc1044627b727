"""Detector options on the device: far-field geometry (Eq. 3), the
acceleration-only field, the hold rules (previous state's field, linear
interpolation) and the potentials, each against the oracle with the same
options."""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2302_14812_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import TOLS, check_parity  # noqa: E402

# far field, accel only, both; hold previous (alone, with far field); hold linear (alone,
# with far field, with accel only); potentials (alone, far field, hold previous, hold linear)
OPTIONS = [1, 2, 3, 4, 5, 8, 9, 10, 16, 17, 20, 24]


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


def gpu_deposit(radio, spec, chunks, precision):
    import torch
    det = radio.Detector.from_spec(spec, precision=precision)
    for ch in chunks:
        det.deposit(radio.Chunk.from_numpy(ch))
    E, B = det.read()
    torch.cuda.synchronize()
    out = E.cpu().numpy(), B.cpu().numpy(), det.stats()
    det.close()
    return out


def oracle_deposit(spec, chunks, cell_index=None):
    D = None
    for ch in chunks:
        D = oracle.deposit_workload(spec, ch, cell_index=cell_index, D=D)
    return oracle.read(D)


@pytest.fixture(scope="module")
def cases():
    und = W.undulator_workload(n_particles=40, n_steps=300, n_side=16, n_t=256)
    pm = W.plasma_mirror_workload(n_particles=60, n_steps=200, n_side=12, n_t=256)
    rnd = W.random_chunk(37, 90, seed=5, dt=0.07, gamma_max=30.0, t_first=0.4)
    cells = W.plane_cells([2.0, -1.0, 60.0], [1, 0, 0], [0, 1, 0], 9, 7, 30.0, 20.0)
    t = rnd.state_times()
    tt = [t[:, None] + np.linalg.norm(xc[:, None, None] - rnd.x, axis=0) for xc in cells]
    lo, hi = min(a.min() for a in tt), max(a.max() for a in tt)
    # a window a little narrower than the arrivals, so both ends clip
    spec = W.DetectorSpec(cells=cells, t0=lo + 0.05 * (hi - lo), dt_det=0.9 * (hi - lo) / 300,
                          n_t=300)
    return {"undulator": (und.detector, [und.chunk]), "plasma_mirror": (pm.detector, [pm.chunk]),
            "random_clipped": (spec, W.split_steps(rnd, [31, 60]))}


_ORACLE = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_twosum"])
@pytest.mark.parametrize("options", OPTIONS)
@pytest.mark.parametrize("case", ["undulator", "plasma_mirror", "random_clipped"])
def test_options_match_oracle(radio, cases, case, options, precision):
    spec, chunks = cases[case]
    spec = dataclasses.replace(spec, options=options)
    Eg, Bg, st = gpu_deposit(radio, spec, chunks, precision)
    if (case, options) not in _ORACLE:
        _ORACLE[(case, options)] = oracle_deposit(spec, chunks)
    Eo, Bo = _ORACLE[(case, options)]
    assert np.abs(Eo).max() > 0.0
    check_parity(Eg, Bg, Eo, Bo, TOLS[precision], f"options {case} options={options} {precision}")


def test_options_in_one_batch_equal_separate(radio, cases):
    import torch
    spec, chunks = cases["undulator"]
    specs = [dataclasses.replace(spec, options=o) for o in (0, 1, 2, 3)]
    dch = radio.Chunk.from_numpy(chunks[0])
    dets = [radio.Detector.from_spec(s, precision=p) for s in specs for p in ("fp64", "mixed")]
    radio.deposit_batch(dets, [dch] * len(dets))
    for d in dets:
        alone = radio.Detector(d.cells(), t0=spec.t0, dt_det=spec.dt_det, n_t=spec.n_t,
                               precision=d.precision, options=d.options)
        alone.deposit(dch)
        Ea, Ba = alone.read()
        Eb, Bb = d.read()
        torch.cuda.synchronize()
        e = max(rel_l2(Eb.cpu().numpy(), Ea.cpu().numpy()), rel_l2(Bb.cpu().numpy(), Ba.cpu().numpy()))
        assert e <= (1e-13 if d.precision == "fp64" else 1e-6), (d.options, d.precision, e)
        alone.close()
        d.close()


def test_acceleration_only_of_uniform_motion_is_zero(radio):
    import torch
    chunk = W.uniform_motion([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]], [[0.3, 0.1, 2.0], [-0.2, 0.4, 1.0]],
                             n_steps=50, dt=0.1, q=-1.0)
    cells = W.plane_cells([0.0, 0.0, 300.0], [1, 0, 0], [0, 1, 0], 4, 4, 50.0, 50.0)
    for options in (2, 3):
        det = radio.Detector(cells, t0=250.0, dt_det=0.5, n_t=200, precision="fp64",
                             options=options)
        det.deposit(radio.Chunk.from_numpy(chunk))
        E, B = det.read()
        torch.cuda.synchronize()
        assert float(E.abs().max()) == 0.0 and float(B.abs().max()) == 0.0
        det.close()


def test_concentric_spherical_shells(radio):
    """A detector of three concentric caps (spherical grids of several radii about the
    origin): its cells, its deposit against the oracle, and the radiation seen by
    the outer shell -- the inner shell's, delayed by the radial distance and scaled
    by the ratio of the radii (the acceleration field falls as 1/R)."""
    import torch
    radii = [1000.0, 1250.0, 1500.0]
    det = radio.Detector.sphere(radii[0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], 8, 6, 0.08, 0.05,
                                shells=3, radius_step=250.0, t0=990.0, dt_det=0.05, n_t=11000,
                                precision="fp64", options=radio.ACCEL_ONLY)
    cells = W.sphere_shell_cells(radii, [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], 8, 6, 0.08, 0.05)
    np.testing.assert_allclose(det.cells(), cells, rtol=1e-13, atol=1e-9)
    chunk = W.circular_orbit(gamma=3.0, radius=1.0, n_steps=1500, dt=0.02, q=-1.0)
    det.deposit(radio.Chunk.from_numpy(chunk))
    E, B = det.read()
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    spec = W.DetectorSpec(cells=cells, t0=990.0, dt_det=0.05, n_t=11000, options=radio.ACCEL_ONLY)
    idx = [0, 20, 47, 48 + 20, 96 + 20, 143]
    Eo, Bo = oracle.read(oracle.deposit_workload(spec, chunk, cell_index=idx))
    e = max(rel_l2(E[idx], Eo), rel_l2(B.cpu().numpy()[idx], Bo))
    print(f"[shells] device vs oracle relL2 {e:.2e}", flush=True)
    assert e <= 1e-12
    # the same direction on the inner and outer shells: 500 / 0.05 = 10000 slots later
    inner, outer = E[20], E[96 + 20]
    shift = 10000
    lhs = outer[shift:shift + 800]
    rhs = inner[:800] * (radii[0] / radii[2])
    r = rel_l2(lhs, rhs)
    print(f"[shells] outer vs delayed, scaled inner relL2 {r:.2e}", flush=True)
    assert np.abs(inner).max() > 0 and r < 0.02
    det.close()
