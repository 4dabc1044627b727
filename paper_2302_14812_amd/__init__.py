"""Python binding of libradio, the MI355X radiation-deposit library.

Argument marshalling only: every step of the deposit runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and HIP streams;
this module checks tensor shapes and types, passes raw device pointers and
the current stream through the C interface declared in include/radio.h, and
turns status codes into exceptions.  It fails loudly when the library has
not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libradio.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ETOOBIG = 0, -1, -2, -3, -4, -5
FP64, MIXED, MIXED_TWOSUM = 0, 1, 2
GEOM_EXPLICIT, GEOM_PLANE, GEOM_SPHERE = 0, 1, 2
# detector options (bit flags)
FAR_FIELD, ACCEL_ONLY, HOLD_PREVIOUS, HOLD_LINEAR, POTENTIALS = 1, 2, 4, 8, 16
_PRECISIONS = {"fp64": FP64, "mixed": MIXED, "mixed_twosum": MIXED_TWOSUM}

# every function the C header declares
EXPORTS = (
    "radio_detector_create", "radio_detector_destroy", "radio_detector_reset",
    "radio_deposit_trajectory_chunk", "radio_deposit_batch", "radio_read_detector",
    "radio_detector_load",
    "radio_detector_stats", "radio_detector_shape", "radio_detector_cells",
    "radio_arrival_times", "radio_status_string", "radio_set_tuning", "radio_get_tuning",
    "radio_spectrum", "radio_push", "radio_slot_coordinates",
    "radio_deposit_trajectory_chunk_noalloc", "radio_noalloc_scratch_bytes",
)


class RadioError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        text = _lib().radio_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{what}: {text} ({status})")


class _Desc(ctypes.Structure):
    _fields_ = [
        ("geometry", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n_cells", ctypes.c_int64), ("cells", ctypes.POINTER(ctypes.c_double)),
        ("origin", ctypes.c_double * 3), ("axis", ctypes.c_double * 3),
        ("e1", ctypes.c_double * 3), ("e2", ctypes.c_double * 3),
        ("radius", ctypes.c_double), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
        ("half1", ctypes.c_double), ("half2", ctypes.c_double),
        ("t0", ctypes.c_double), ("dt_det", ctypes.c_double), ("n_t", ctypes.c_int64),
        ("c", ctypes.c_double), ("options", ctypes.c_int32),
        ("n3", ctypes.c_int64), ("radius_step", ctypes.c_double),
    ]


class _Chunk(ctypes.Structure):
    _fields_ = [
        ("n_particles", ctypes.c_int64), ("n_steps", ctypes.c_int64),
        ("t_first", ctypes.c_double), ("dt", ctypes.c_double), ("first_step", ctypes.c_int64),
        ("x", ctypes.c_void_p), ("u", ctypes.c_void_p), ("q", ctypes.c_void_p),
    ]


class _Push(ctypes.Structure):
    _fields_ = [
        ("qm", ctypes.c_double), ("dt", ctypes.c_double),
        ("E", ctypes.c_double * 3), ("B", ctypes.c_double * 3),
        ("wave_amplitude", ctypes.c_double), ("wave_dir", ctypes.c_double * 3),
        ("wave_pol", ctypes.c_double * 3), ("wave_omega", ctypes.c_double),
        ("wave_phase", ctypes.c_double),
    ]


class _Tuning(ctypes.Structure):
    _fields_ = [("target_blocks", ctypes.c_int32), ("items_per_workgroup", ctypes.c_int32),
                ("max_grid", ctypes.c_int32), ("order_budget_mib", ctypes.c_int32),
                ("shape", ctypes.c_int32)]


# workgroup shapes of the deposit (radio_tuning.shape): cells per tile, particles
# per batch, segments per run
SHAPES = {0: (16, 16, 16), 1: (8, 32, 16), 2: (16, 16, 8)}
_TUNING_FIELDS = ("target_blocks", "items_per_workgroup", "max_grid", "order_budget_mib", "shape")


class _Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("interactions", "clipped", "nonmonotone", "chunks", "bytes", "bypassed", "slices",
                 "large_ring")]


_LIB = None


def _lib():
    """Load libradio.so (after torch, so both share torch's HIP runtime)."""
    global _LIB
    if _LIB is None:
        import torch  # noqa: F401  -- loads the HIP runtime the library must bind to
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_2302_14812_amd/build_lib.py")
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.radio_status_string.argtypes = [ctypes.c_int]
        lib.radio_status_string.restype = ctypes.c_char_p
        lib.radio_detector_create.argtypes = [ctypes.POINTER(_Desc), vp, ctypes.POINTER(vp)]
        lib.radio_detector_destroy.argtypes = [vp]
        lib.radio_detector_reset.argtypes = [vp, vp]
        lib.radio_deposit_trajectory_chunk.argtypes = [vp, ctypes.POINTER(_Chunk), vp]
        lib.radio_deposit_trajectory_chunk_noalloc.argtypes = [vp, ctypes.POINTER(_Chunk), vp]
        lib.radio_noalloc_scratch_bytes.argtypes = [ctypes.POINTER(i64)]
        lib.radio_deposit_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_Chunk),
                                            ctypes.c_int, vp]
        lib.radio_read_detector.argtypes = [vp, vp, vp, vp]
        lib.radio_detector_load.argtypes = [vp, vp, vp, vp]
        lib.radio_detector_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
        lib.radio_detector_shape.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                             ctypes.POINTER(ctypes.c_int32)]
        lib.radio_detector_cells.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        lib.radio_arrival_times.argtypes = [vp, vp, vp, i64, ctypes.c_double, vp, vp]
        lib.radio_slot_coordinates.argtypes = [vp, vp, vp, i64, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, vp, vp]
        lib.radio_spectrum.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double), vp, vp, vp, vp]
        lib.radio_push.argtypes = [ctypes.POINTER(_Push), i64, i64, ctypes.c_double, i64, vp, vp,
                                   vp]
        lib.radio_set_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        lib.radio_get_tuning.argtypes = [ctypes.POINTER(_Tuning)]
        for name in EXPORTS:
            if name != "radio_status_string":
                getattr(lib, name).restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _check(rc: int, what: str) -> None:
    if rc != OK:
        raise RadioError(rc, what)


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev_f64(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Chunk:
    """Device-resident trajectory chunk: x, u of shape (3, S+1, Np), q of shape (Np,).

    State s of the chunk is state first_step + s of its run, at time
    t_first + (first_step + s) * dt."""

    def __init__(self, x, u, q=None, t_first: float = 0.0, dt: float = 1.0, first_step: int = 0):
        import torch
        if not isinstance(x, torch.Tensor) or x.dim() != 3 or x.shape[0] != 3:
            raise ValueError("x must be a (3, S+1, Np) tensor")
        self.x = _dev_f64(x, x.shape, "x")
        self.u = _dev_f64(u, x.shape, "u")
        self.q = None if q is None else _dev_f64(q, (x.shape[2],), "q")
        self.t_first = float(t_first)
        self.dt = float(dt)
        self.first_step = int(first_step)

    @classmethod
    def from_numpy(cls, chunk, device="cuda") -> "Chunk":
        """Copy a workloads.Chunk (host arrays) to the device."""
        import torch
        return cls(torch.from_numpy(np.ascontiguousarray(chunk.x)).to(device),
                   torch.from_numpy(np.ascontiguousarray(chunk.u)).to(device),
                   torch.from_numpy(np.ascontiguousarray(chunk.q)).to(device),
                   chunk.t_first, chunk.dt, getattr(chunk, "first_step", 0))

    def slice(self, s_begin: int, s_end: int, p_begin: int = 0,
              p_end: Optional[int] = None) -> "Chunk":
        """States s_begin..s_end inclusive of particles p_begin..p_end-1 as a new chunk
        (a device copy) with the same state times; its deposit adds those particles'
        segments s_begin+1..s_end."""
        p_end = self.n_particles if p_end is None else p_end
        if not (0 <= s_begin <= s_end <= self.n_steps and 0 <= p_begin <= p_end <= self.n_particles):
            raise ValueError("slice out of bounds")
        return Chunk(self.x[:, s_begin:s_end + 1, p_begin:p_end].contiguous(),
                     self.u[:, s_begin:s_end + 1, p_begin:p_end].contiguous(),
                     None if self.q is None else self.q[p_begin:p_end].contiguous(),
                     self.t_first, self.dt, self.first_step + s_begin)

    def slice_steps(self, s_begin: int, s_end: int) -> "Chunk":
        return self.slice(s_begin, s_end)

    def slice_particles(self, p_begin: int, p_end: int) -> "Chunk":
        return self.slice(0, self.n_steps, p_begin, p_end)

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[2])

    @property
    def n_steps(self) -> int:
        return int(self.x.shape[1]) - 1

    def _c(self) -> _Chunk:
        return _Chunk(self.n_particles, self.n_steps, self.t_first, self.dt, self.first_step,
                      self.x.data_ptr(), self.u.data_ptr(),
                      None if self.q is None else self.q.data_ptr())


class Detector:
    """A virtual detector resident in device memory (RaDiO Sec. 3.1).

    Create it from explicit cell positions (`cells`, an (Nc, 3) array) or
    with Detector.plane / Detector.sphere.  Slot j covers
    [t0 + j dt_det, t0 + (j+1) dt_det), j < n_t.  options: FAR_FIELD (Eq. 3
    arrival time, cell direction and distance in Eq. 1) and/or ACCEL_ONLY (the
    acceleration term of Eq. 1 alone).
    """

    def __init__(self, cells=None, *, t0: float, dt_det: float, n_t: int, c: float = 1.0,
                 precision: str = "fp64", options: int = 0, stream=None,
                 _desc: Optional[_Desc] = None):
        lib = _lib()
        d = _desc if _desc is not None else _Desc()
        keep = None
        if _desc is None:
            cells = np.ascontiguousarray(np.asarray(cells, dtype=np.float64).reshape(-1, 3))
            keep = cells
            d.geometry = GEOM_EXPLICIT
            d.n_cells = cells.shape[0]
            d.cells = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if precision not in _PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
        d.precision = _PRECISIONS[precision]
        d.t0, d.dt_det, d.n_t, d.c = float(t0), float(dt_det), int(n_t), float(c)
        d.options = int(options)
        h = ctypes.c_void_p()
        _check(lib.radio_detector_create(ctypes.byref(d), _stream(stream), ctypes.byref(h)),
               "radio_detector_create")
        del keep
        self._h = h
        self.precision = precision
        self.options = int(options)
        n_c, nt, prec = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib.radio_detector_shape(h, ctypes.byref(n_c), ctypes.byref(nt), ctypes.byref(prec)),
               "radio_detector_shape")
        self.n_cells, self.n_t = int(n_c.value), int(nt.value)
        self.t0, self.dt_det, self.c = float(t0), float(dt_det), float(c)

    @classmethod
    def plane(cls, origin, e1, e2, n1, n2, half1, half2, **kw) -> "Detector":
        d = _Desc()
        d.geometry = GEOM_PLANE
        d.origin[:] = [float(v) for v in origin]
        d.e1[:] = [float(v) for v in e1]
        d.e2[:] = [float(v) for v in e2]
        d.n1, d.n2, d.half1, d.half2 = int(n1), int(n2), float(half1), float(half2)
        return cls(_desc=d, **kw)

    @classmethod
    def sphere(cls, radius, axis, e1, n1, n2, half1, half2, shells: int = 1,
               radius_step: float = 0.0, **kw) -> "Detector":
        """Cells on `shells` concentric spherical caps of radii radius + k radius_step."""
        d = _Desc()
        d.geometry = GEOM_SPHERE
        d.radius = float(radius)
        d.n3, d.radius_step = int(shells), float(radius_step)
        d.axis[:] = [float(v) for v in axis]
        d.e1[:] = [float(v) for v in e1]
        d.n1, d.n2, d.half1, d.half2 = int(n1), int(n2), float(half1), float(half2)
        return cls(_desc=d, **kw)

    @classmethod
    def from_spec(cls, spec, precision: str = "fp64", stream=None,
                  options: Optional[int] = None) -> "Detector":
        """From a workloads.DetectorSpec (options default to the spec's)."""
        if options is None:
            options = getattr(spec, "options", 0)
        return cls(spec.cells, t0=spec.t0, dt_det=spec.dt_det, n_t=spec.n_t, c=spec.c,
                   precision=precision, options=options, stream=stream)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("detector has been closed")
        return self._h

    def deposit(self, chunk: Chunk, stream=None) -> None:
        c = chunk._c()
        _check(_lib().radio_deposit_trajectory_chunk(self.handle, ctypes.byref(c), _stream(stream)),
               "radio_deposit_trajectory_chunk")

    def deposit_noalloc(self, chunk: Chunk, stream=None) -> None:
        """The same deposit with every workspace in the library's fixed scratch
        (no device allocation; RadioError ETOOBIG when the chunk does not fit)."""
        c = chunk._c()
        _check(_lib().radio_deposit_trajectory_chunk_noalloc(self.handle, ctypes.byref(c),
                                                              _stream(stream)),
               "radio_deposit_trajectory_chunk_noalloc")

    def read(self, E=None, B=None, stream=None) -> Tuple[object, object]:
        """Return (E, B) device tensors of shape (n_cells, n_t, 3)."""
        import torch
        shape = (self.n_cells, self.n_t, 3)
        if E is None:
            E = torch.empty(shape, dtype=torch.float64, device="cuda")
        if B is None:
            B = torch.empty(shape, dtype=torch.float64, device="cuda")
        _dev_f64(E, shape, "E")
        _dev_f64(B, shape, "B")
        _check(_lib().radio_read_detector(self.handle, E.data_ptr(), B.data_ptr(), _stream(stream)),
               "radio_read_detector")
        return E, B

    def load(self, E, B, stream=None) -> None:
        """Replace the detector's fields with (E, B) device tensors of shape (n_cells,
        n_t, 3), as read() returns them: restores a snapshot, so that later deposits
        add to it (radio_detector_load)."""
        shape = (self.n_cells, self.n_t, 3)
        _dev_f64(E, shape, "E")
        _dev_f64(B, shape, "B")
        _check(_lib().radio_detector_load(self.handle, E.data_ptr(), B.data_ptr(), _stream(stream)),
               "radio_detector_load")

    def spectrum(self, n_fft: int = 0, weights=None, stream=None, d2I: bool = True,
                 dIdw: bool = True, dIdO: bool = True):
        """Spectral intensity of the detector's fields (radio_spectrum): returns
        (omega [n_f] host array, d2I [n_cells, n_f], dIdw [n_f], dIdO [n_cells]) with
        device tensors (None for outputs not asked for); n_f = n_fft/2 + 1."""
        import torch
        N = int(n_fft) if n_fft else 1 << max(0, int(self.n_t - 1).bit_length())
        n_f = N // 2 + 1
        a = torch.empty((self.n_cells, n_f), dtype=torch.float64, device="cuda") if d2I else None
        b = torch.empty((n_f,), dtype=torch.float64, device="cuda") if dIdw else None
        c = torch.empty((self.n_cells,), dtype=torch.float64, device="cuda") if dIdO else None
        w = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
            if w.shape[0] != self.n_cells:
                raise ValueError("one weight per cell")
        ptr = (lambda t: None if t is None else t.data_ptr())
        _check(_lib().radio_spectrum(self.handle, int(n_fft),
                                     None if w is None else w.ctypes.data_as(
                                         ctypes.POINTER(ctypes.c_double)),
                                     ptr(a), ptr(b), ptr(c), _stream(stream)), "radio_spectrum")
        omega = 2.0 * np.pi * np.arange(n_f) / (N * self.dt_det)
        return omega, a, b, c

    def reset(self, stream=None) -> None:
        _check(_lib().radio_detector_reset(self.handle, _stream(stream)), "radio_detector_reset")

    def stats(self) -> dict:
        s = _Stats()
        _check(_lib().radio_detector_stats(self.handle, ctypes.byref(s)), "radio_detector_stats")
        return {n: int(getattr(s, n)) for n, _ in _Stats._fields_}

    def cells(self) -> np.ndarray:
        out = np.empty((self.n_cells, 3))
        _check(_lib().radio_detector_cells(self.handle,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "radio_detector_cells")
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(_lib().radio_detector_destroy(self._h), "radio_detector_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def deposit_batch(detectors: Sequence[Detector], chunks: Sequence[Chunk], stream=None) -> None:
    """Deposit n independent (detector, chunk) pairs in one launch."""
    if len(detectors) != len(chunks):
        raise ValueError("one chunk per detector")
    n = len(detectors)
    hs = (ctypes.c_void_p * max(n, 1))(*[d.handle for d in detectors])
    cs = (_Chunk * max(n, 1))(*[c._c() for c in chunks])
    _check(_lib().radio_deposit_batch(hs, cs, n, _stream(stream)), "radio_deposit_batch")


def get_tuning() -> dict:
    t = _Tuning()
    _check(_lib().radio_get_tuning(ctypes.byref(t)), "radio_get_tuning")
    return {k: int(getattr(t, k)) for k in _TUNING_FIELDS}


def set_tuning(target_blocks: Optional[int] = None, items_per_workgroup: Optional[int] = None,
               max_grid: Optional[int] = None, order_budget_mib: Optional[int] = None,
               shape: Optional[int] = None) -> None:
    """Set the launch tunables (radio_tuning); unnamed ones keep their values."""
    cur = get_tuning()
    new = {"target_blocks": target_blocks, "items_per_workgroup": items_per_workgroup,
           "max_grid": max_grid, "order_budget_mib": order_budget_mib, "shape": shape}
    t = _Tuning(*[int(new[k] if new[k] is not None else cur[k]) for k in _TUNING_FIELDS])
    _check(_lib().radio_set_tuning(ctypes.byref(t)), "radio_set_tuning")


def push(chunk: "Chunk", qm: float = -1.0, E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0),
         wave_amplitude: float = 0.0, wave_dir=(1.0, 0.0, 0.0), wave_pol=(0.0, 1.0, 0.0),
         wave_omega: float = 1.0, wave_phase: float = 0.0, stream=None) -> "Chunk":
    """Fill states 1..S of a device chunk from its state 0 with the run-time push
    (radio_push), at the chunk's own dt, t_first and first_step; returns the chunk."""
    d = _Push()
    d.qm, d.dt = float(qm), float(chunk.dt)
    d.E[:] = [float(v) for v in E]
    d.B[:] = [float(v) for v in B]
    d.wave_amplitude = float(wave_amplitude)
    d.wave_dir[:] = [float(v) for v in wave_dir]
    d.wave_pol[:] = [float(v) for v in wave_pol]
    d.wave_omega, d.wave_phase = float(wave_omega), float(wave_phase)
    _check(_lib().radio_push(ctypes.byref(d), chunk.n_particles, chunk.n_steps, chunk.t_first,
                             chunk.first_step, chunk.x.data_ptr(), chunk.u.data_ptr(),
                             _stream(stream)), "radio_push")
    return chunk


def arrival_times(cells, points, t, c: float = 1.0, stream=None):
    """t + |cells - points|/c on the device for (n, 3), (n, 3), (n,) float64 tensors."""
    import torch
    n = int(t.shape[0])
    _dev_f64(cells, (n, 3), "cells")
    _dev_f64(points, (n, 3), "points")
    _dev_f64(t, (n,), "t")
    out = torch.empty(n, dtype=torch.float64, device=t.device)
    _check(_lib().radio_arrival_times(cells.data_ptr(), points.data_ptr(), t.data_ptr(), n, float(c),
                                      out.data_ptr(), _stream(stream)), "radio_arrival_times")
    return out


def slot_coordinates(cells, points, t, t0: float, dt_det: float, c: float = 1.0, stream=None):
    """(t + |cells - points|/c - t0) / dt_det on the device, rounded as the double
    deposit rounds it, for (n, 3), (n, 3), (n,) float64 tensors."""
    import torch
    n = int(t.shape[0])
    _dev_f64(cells, (n, 3), "cells")
    _dev_f64(points, (n, 3), "points")
    _dev_f64(t, (n,), "t")
    out = torch.empty(n, dtype=torch.float64, device=t.device)
    _check(_lib().radio_slot_coordinates(cells.data_ptr(), points.data_ptr(), t.data_ptr(), n,
                                         float(c), float(t0), float(dt_det), out.data_ptr(),
                                         _stream(stream)), "radio_slot_coordinates")
    return out
