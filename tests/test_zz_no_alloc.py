"""The deposit that allocates nothing (radio_deposit_trajectory_chunk_noalloc),
called through the C ABI: the same fields as the allocating entry point on two
calls in a row, the second with a smaller chunk (the scratch keeps the first
call's contents), no device memory taken by the second call, and a chunk
beyond the fixed scratch rejected with nothing deposited."""
import ctypes

import numpy as np
import pytest

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


def _fields(det):
    import torch
    E, B = det.read()
    torch.cuda.synchronize()
    return E.cpu().numpy(), B.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_allocating_deposit(radio, precision):
    import torch
    lib = radio._lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # 5000 x 901 states: 288 MB of mixed records, so the first call runs as time slices
    big = W.undulator_workload(n_particles=5000, n_steps=900, n_side=40, n_t=768)
    chunk = W.random_chunk(40, 90, seed=3, dt=0.07, gamma_max=20.0, t_first=0.4)
    cells = W.plane_cells([1.0, -2.0, 30.0], [1, 0.2, 0], [0, 1, 0.1], 11, 9, 12.0, 9.0)
    t0, dtd = W.arrival_window(cells, chunk, 200, pad_frac=0.05,
                               cell_index=W.grid_corner_cells(11, 9), seed=3)
    small_spec = W.DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=200)
    cases = [(big.detector, big.chunk), (small_spec, chunk)]  # the second call is smaller
    free = []
    for k, (spec, host) in enumerate(cases):
        dev = radio.Chunk.from_numpy(host)
        ref = radio.Detector.from_spec(spec, precision=precision)
        got = radio.Detector.from_spec(spec, precision=precision)
        assert lib.radio_deposit_trajectory_chunk(ref.handle, ctypes.byref(dev._c()), stream) == 0
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
        assert lib.radio_deposit_trajectory_chunk_noalloc(got.handle, ctypes.byref(dev._c()),
                                                          stream) == 0
        torch.cuda.synchronize()
        if k == 1:  # the scratch exists since the first call: nothing more is taken
            assert torch.cuda.mem_get_info()[0] >= free[1]
        Er, Br = _fields(ref)
        Eg, Bg = _fields(got)
        tol = 1e-13 if precision == "fp64" else 1e-6
        check_parity(Eg, Bg, Er, Br, tol, f"no-alloc vs allocating deposit, call {k + 1} {precision}")
        st_r, st_g = ref.stats(), got.stats()
        if k == 0:
            assert st_g["slices"] > 1
        assert st_g["interactions"] == st_r["interactions"] == host.n_particles * host.n_steps * spec.n_cells
        assert (st_g["clipped"], st_g["nonmonotone"]) == (st_r["clipped"], st_r["nonmonotone"])
        ref.close()
        got.close()


def test_noalloc_rejects_chunk_beyond_scratch(radio):
    import torch
    lib = radio._lib()
    cap = ctypes.c_int64()
    assert lib.radio_noalloc_scratch_bytes(ctypes.byref(cap)) == 0
    assert cap.value == 256 << 20
    # 65536 cells (4096 tiles) x 20000 particles: one particle order alone is 328 MB
    det = radio.Detector.plane([0.0, 0.0, 100.0], [1, 0, 0], [0, 1, 0], 256, 256, 10.0, 10.0,
                               t0=90.0, dt_det=0.5, n_t=16, precision="mixed")
    host = W.random_chunk(20000, 3, seed=9, dt=0.05, gamma_max=5.0)
    dev = radio.Chunk.from_numpy(host)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.radio_deposit_trajectory_chunk_noalloc(det.handle, ctypes.byref(dev._c()), stream)
    assert rc == radio.ETOOBIG
    assert lib.radio_status_string(rc).startswith(b"chunk too large")
    E, B = _fields(det)
    assert np.abs(E).max() == 0.0 and np.abs(B).max() == 0.0
    assert det.stats()["chunks"] == 0
    # the allocating entry point takes it
    det.deposit(dev)
    assert np.abs(_fields(det)[0]).max() > 0.0
    det.close()
