"""The large slot ring against the oracle.

Tiles whose arrivals cross slots often (the plasma-mirror sheet: ~1.5 slots per
segment) take the 64-slot ring, whose kernels stage through registers and
prefetch the next batch and the next state.  The detector's `large_ring`
counter says how many interactions went that way; these tests require most
of them to, and compare the result with the oracle in every precision and
workgroup shape, with every hold rule and geometry option, and in a batch
(the persistent kernel).
"""
import numpy as np
import pytest

import oracle
from paper_2302_14812_amd import workloads as W

pytestmark = pytest.mark.gpu

from parity import TOLS, check_parity  # noqa: E402

PRECISIONS = pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_twosum"])

_CACHE = {}


@pytest.fixture(scope="module")
def radio():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_14812_amd as radio
    radio._lib()
    return radio


def _case():
    """300 electrons of the plasma-mirror sheet over 250 steps on a 16 x 16 cap with
    1024 slots: the full configuration's slots per step, so its crossing rate."""
    if "pm" not in _CACHE:
        _CACHE["pm"] = W.plasma_mirror_workload(n_particles=300, n_steps=250, n_side=16, n_t=1024)
    return _CACHE["pm"]


def _oracle(options=0):
    key = ("oracle", options)
    if key not in _CACHE:
        wl = _case()
        cnt = np.zeros(2, dtype=np.int64)
        D = oracle.deposit_workload(wl.detector, wl.chunk, options=options, counters=cnt)
        _CACHE[key] = oracle.read(D) + (cnt,)
    return _CACHE[key]


def _deposit(radio, precision, options=0):
    import torch
    wl = _case()
    det = radio.Detector.from_spec(wl.detector, precision=precision, options=options)
    det.deposit(radio.Chunk.from_numpy(wl.chunk))
    E, B = det.read()
    torch.cuda.synchronize()
    st = det.stats()
    det.close()
    return E.cpu().numpy(), B.cpu().numpy(), st


def _mostly_large(st, what):
    frac = st["large_ring"] / max(1, st["interactions"])
    print(f"[large ring] {what}: {frac:.3f} of {st['interactions']} interactions", flush=True)
    assert frac >= 0.5, (what, frac)


@pytest.mark.parametrize("shape", [0, 1, 2])
@PRECISIONS
def test_large_ring_matches_oracle(radio, precision, shape):
    cur = radio.get_tuning()
    try:
        radio.set_tuning(shape=shape)
        E, B, st = _deposit(radio, precision)
    finally:
        radio.set_tuning(**cur)
    _mostly_large(st, f"shape {shape} {precision}")
    Eo, Bo, cnt = _oracle()
    check_parity(E, B, Eo, Bo, TOLS[precision], f"large ring shape {shape} {precision}")
    assert st["clipped"] == cnt[0] and st["nonmonotone"] == cnt[1]


@pytest.mark.parametrize("opt", ["HOLD_PREVIOUS", "HOLD_LINEAR", "FAR_FIELD", "POTENTIALS"])
@PRECISIONS
def test_large_ring_options_match_oracle(radio, precision, opt):
    E, B, st = _deposit(radio, precision, getattr(radio, opt))
    _mostly_large(st, f"{opt} {precision}")
    Eo, Bo, _ = _oracle(getattr(oracle, opt))
    check_parity(E, B, Eo, Bo, TOLS[precision], f"large ring {opt} {precision}")


@PRECISIONS
def test_large_ring_in_a_batch(radio, precision):
    """The persistent kernel: the plasma-mirror case beside a slow-arrival case (the
    small ring) in one batch, each against the oracle."""
    import torch
    und = W.undulator_workload(n_particles=64, n_steps=300, n_side=16, n_t=512)
    wl = _case()
    cases = [(wl.detector, wl.chunk, _oracle()[:2]),
             (und.detector, und.chunk, oracle.read(oracle.deposit_workload(und.detector, und.chunk)))]
    dets = [radio.Detector.from_spec(spec, precision=precision) for spec, _, _ in cases]
    radio.deposit_batch(dets, [radio.Chunk.from_numpy(c) for _, c, _ in cases])
    for i, (d, (spec, chunk, (Eo, Bo))) in enumerate(zip(dets, cases)):
        E, B = d.read()
        torch.cuda.synchronize()
        st = d.stats()
        d.close()
        if i == 0:
            _mostly_large(st, f"batch {precision}")
        check_parity(E.cpu().numpy(), B.cpu().numpy(), Eo, Bo, TOLS[precision],
                     f"batch case {i} {precision}")
