"""CPU oracle for the RaDiO radiation deposit -- TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library never calls it and shares no
code with it.  The arithmetic lives in radio_oracle.c (plain IEEE double,
no FMA contraction, no fast-math); this module builds it with gcc and
marshals numpy arrays into it.

Functions and the passages they follow:
  kinematics(u)            Alg. 1: beta = p / sqrt(|p|^2 + 1), 1/gamma^2
  arrival(x_cell, x, t, c) Eq. 2: t_det = t + |x_part - x_cell| / c
                           (far=True: Eq. 3, t + R_cell/c - x_part . n_cell / c)
  slot_of(tau, t0, dt_det) Alg. 2's slot function before the floor:
                           (tau - t0) / dt_det
  field(...)               Eq. 1: Lienard-Wiechert E and B = n x E (options:
                           FAR_FIELD geometry, ACCEL_ONLY second term)
  deposit(...)             Alg. 1 + Alg. 2 with the integrator-detector
                           definition of Sec. 3.2 (slot value = integral of
                           the piecewise-constant field over the slot / dt_det)
  spectrum(...)            Sec. 4: detector fields Fourier transformed in time,
                           d2I/domega dOmega, dI/domega, dI/dOmega
  boris_push(...)          the particle push that precedes the run-time deposit
                           (Sec. 3.1): Boris method in external fields
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "radio_oracle.c")
_LIB = os.path.join(_HERE, "libradio_oracle.so")

_lib = None

FAR_FIELD = 1      # Eq. 3 arrival time and the cell's direction and distance in Eq. 1
ACCEL_ONLY = 2     # only the acceleration term of Eq. 1
HOLD_PREVIOUS = 4  # segment s holds the field of state s-1 (Fig. 5 walk-through)
HOLD_LINEAR = 8    # the field varies linearly in arrival time between the two states
POTENTIALS = 16    # Lienard-Wiechert potentials (A, phi) instead of (E, B)


def build(force: bool = True) -> str:
    """Compile radio_oracle.c with gcc into libradio_oracle.so."""
    global _lib
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           "-fvisibility=hidden", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.radio_oracle_kinematics.argtypes = [dp, dp, dp]
        lib.radio_oracle_kinematics.restype = None
        lib.radio_oracle_arrival.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double]
        lib.radio_oracle_arrival.restype = ctypes.c_double
        lib.radio_oracle_arrival_far.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double]
        lib.radio_oracle_arrival_far.restype = ctypes.c_double
        lib.radio_oracle_slot_of.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.radio_oracle_slot_of.restype = ctypes.c_double
        lib.radio_oracle_field_opts.argtypes = [dp, dp, dp, ctypes.c_double, dp, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int, dp, dp]
        lib.radio_oracle_field_opts.restype = None
        lib.radio_oracle_deposit.argtypes = [dp, i64, ctypes.c_double, ctypes.c_double, i64,
                                             ctypes.c_double, i64, i64, ctypes.c_double, i64,
                                             ctypes.c_double, dp, dp, dp, ctypes.c_int, dp,
                                             ctypes.POINTER(i64), ctypes.c_int]
        lib.radio_oracle_deposit.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def kinematics(u) -> Tuple[np.ndarray, float]:
    u = _f64(u)
    beta = np.empty(3)
    g2 = ctypes.c_double()
    _load().radio_oracle_kinematics(_dptr(u), _dptr(beta), ctypes.byref(g2))
    return beta, g2.value


def arrival(x_cell, x_part, t: float, c: float = 1.0, far: bool = False) -> float:
    f = _load().radio_oracle_arrival_far if far else _load().radio_oracle_arrival
    return f(_dptr(_f64(x_cell)), _dptr(_f64(x_part)), float(t), float(c))


def slot_of(tau: float, t0: float, dt_det: float) -> float:
    """Slot coordinate (tau - t0) / dt_det of an arrival time (Alg. 2's slot
    function before the floor), one correctly rounded division."""
    return _load().radio_oracle_slot_of(float(tau), float(t0), float(dt_det))


def field(x_cell, x_part, beta, inv_gamma2: float, betadot, q: float = -1.0,
          c: float = 1.0, options: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    E = np.empty(3)
    B = np.empty(3)
    _load().radio_oracle_field_opts(_dptr(_f64(x_cell)), _dptr(_f64(x_part)), _dptr(_f64(beta)),
                                    float(inv_gamma2), _dptr(_f64(betadot)), float(q), float(c),
                                    int(options), _dptr(E), _dptr(B))
    return E, B


def deposit(cells, t0: float, dt_det: float, n_t: int, x, u, q, t_first: float, dt: float,
            c: float = 1.0, D: Optional[np.ndarray] = None, n_threads: Optional[int] = None,
            counters: Optional[np.ndarray] = None, first_step: int = 0,
            options: int = 0) -> np.ndarray:
    """Accumulate one chunk into D[n_cells, n_t, 6] (created zeroed if None).

    State s of the chunk is state first_step + s of the run, at time
    t_first + (first_step + s) * dt."""
    cells = _f64(cells).reshape(-1, 3)
    x = _f64(x)
    u = _f64(u)
    n_c = cells.shape[0]
    if x.ndim != 3 or x.shape[0] != 3 or u.shape != x.shape:
        raise ValueError("x and u must both have shape (3, S+1, Np)")
    n_states, n_p = x.shape[1], x.shape[2]
    qa = None if q is None else _f64(q)
    if qa is not None and qa.shape != (n_p,):
        raise ValueError("q must have shape (Np,)")
    if D is None:
        D = np.zeros((n_c, n_t, 6))
    if D.dtype != np.float64 or not D.flags.c_contiguous or D.shape != (n_c, n_t, 6):
        raise ValueError("D must be a C-contiguous float64 array of shape (n_cells, n_t, 6)")
    if counters is None:
        counters = np.zeros(2, dtype=np.int64)
    if n_threads is None:
        n_threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rc = _load().radio_oracle_deposit(
        _dptr(cells), n_c, float(t0), float(dt_det), int(n_t), float(c), n_p, n_states - 1,
        float(t_first), int(first_step), float(dt), _dptr(x), _dptr(u), _dptr(qa), int(options),
        _dptr(D),
        counters.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(n_threads))
    if rc != 0:
        raise ValueError(f"oracle deposit rejected its arguments (rc={rc})")
    return D


def deposit_workload(detector, chunk, cell_index=None, D=None, n_threads=None, counters=None,
                     options=None):
    """Convenience: deposit a workloads.Chunk on (a subset of) a DetectorSpec's cells
    (options default to the spec's own, if it has any)."""
    if options is None:
        options = getattr(detector, "options", 0)
    cells = detector.cells if cell_index is None else detector.cells[np.asarray(cell_index)]
    return deposit(cells, detector.t0, detector.dt_det, detector.n_t, chunk.x, chunk.u, chunk.q,
                   chunk.t_first, chunk.dt, c=detector.c, D=D, n_threads=n_threads,
                   counters=counters, first_step=getattr(chunk, "first_step", 0), options=options)


def read(D: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Split an oracle detector array into E[n_cells, n_t, 3] and B[n_cells, n_t, 3]."""
    return np.ascontiguousarray(D[..., :3]), np.ascontiguousarray(D[..., 3:])


def spectrum(E, dt_det: float, cells, n_fft: Optional[int] = None, weights=None, c: float = 1.0
             ) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Spectral intensity of detector fields E[n_cells, n_t, 3] (the detector data
    Fourier transformed with respect to time, Sec. 4).

    The slot value is the field held over its slot, so the transform of the
    piecewise-constant signal at omega is
        F(omega) = sum_j E_j exp(i omega j dt) * (exp(i omega dt) - 1) / (i omega),
    and, with R the cell's distance from the origin,
        d2I/domega dOmega = c R^2 / (4 pi^2) |F(omega)|^2            (per cell)
        dI/domega         = sum_cells weight_c d2I/domega dOmega
        dI/dOmega         = c R^2 / (4 pi) sum_j |E_j|^2 dt          (Parseval, per cell)
    at omega_m = 2 pi m / (n_fft dt), m = 0 .. n_fft/2, with the signal zero
    beyond its n_t slots (n_fft >= n_t; default the next power of two).
    Returns (omega, d2I [n_cells, n_fft/2 + 1], dIdomega, dIdOmega).
    """
    E = np.asarray(E, dtype=np.float64)
    n_c, n_t = E.shape[0], E.shape[1]
    N = int(n_fft) if n_fft else 1 << max(0, int(n_t - 1).bit_length())
    if N < n_t:
        raise ValueError("n_fft must be at least n_t")
    m = np.arange(N // 2 + 1)
    omega = 2.0 * np.pi * m / (N * dt_det)
    # |(exp(i w dt) - 1) / (i w)|^2 = (2 sin(w dt / 2) / w)^2, -> dt^2 as w -> 0
    W2 = np.empty_like(omega)
    W2[0] = dt_det * dt_det
    W2[1:] = (2.0 * np.sin(0.5 * omega[1:] * dt_det) / omega[1:]) ** 2
    Z = np.fft.fft(E, n=N, axis=1)[:, :N // 2 + 1, :]           # library DFT, sum_j E_j e^{-i w t_j}
    R2 = (np.asarray(cells, dtype=np.float64) ** 2).sum(axis=1)
    d2I = (c * R2 / (4.0 * np.pi ** 2))[:, None] * W2[None, :] * (np.abs(Z) ** 2).sum(axis=2)
    w = np.ones(n_c) if weights is None else np.asarray(weights, dtype=np.float64)
    dIdw = w @ d2I
    dIdO = c * R2 / (4.0 * np.pi) * (E * E).sum(axis=(1, 2)) * dt_det
    return omega, d2I, dIdw, dIdO


def push_fields(x, t, fields):
    """External fields at positions x (3, Np) and time t: uniform E and B plus a
    plane wave E = a pol cos(omega (t - k.x) + phase), B = k x E."""
    E = np.repeat(np.asarray(fields.get("E", (0, 0, 0)), dtype=np.float64)[:, None], x.shape[1], 1)
    B = np.repeat(np.asarray(fields.get("B", (0, 0, 0)), dtype=np.float64)[:, None], x.shape[1], 1)
    a = float(fields.get("wave_amplitude", 0.0))
    if a != 0.0:
        k = np.asarray(fields["wave_dir"], dtype=np.float64)
        pol = np.asarray(fields["wave_pol"], dtype=np.float64)
        ph = fields.get("wave_omega", 1.0) * (t - k @ x) + fields.get("wave_phase", 0.0)
        Ew = a * pol[:, None] * np.cos(ph)[None, :]
        E = E + Ew
        B = B + np.cross(k[:, None], Ew, axis=0)
    return E, B


def boris_push(x0, u0, qm: float, dt: float, n_steps: int, fields: dict, t_first: float = 0.0,
               first_step: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """States 0..n_steps of particles pushed by the Boris method (Boris 1970) in
    the external fields of push_fields, c = 1, u = gamma beta.  One step: half
    drift, the Boris kick with the fields at the half step (half electric kick,
    magnetic rotation, half electric kick), half drift, so that x and u are
    samples at the same times t_first + (first_step + s) dt (the run-time mode's
    push, Sec. 3.1).  Returns x, u of shape (3, n_steps + 1, Np)."""
    x = np.empty((3, n_steps + 1, np.shape(x0)[1]))
    u = np.empty_like(x)
    x[:, 0] = x0
    u[:, 0] = u0
    h = 0.5 * qm * dt
    for s in range(n_steps):
        xs, us = x[:, s], u[:, s]
        g = np.sqrt(1.0 + (us * us).sum(axis=0))
        xh = xs + 0.5 * dt * us / g
        th = t_first + (first_step + s + 0.5) * dt
        E, B = push_fields(xh, th, fields)
        um = us + h * E
        gm = np.sqrt(1.0 + (um * um).sum(axis=0))
        tv = h * B / gm
        up = um + np.cross(um, tv, axis=0)
        sv = 2.0 * tv / (1.0 + (tv * tv).sum(axis=0))
        un = um + np.cross(up, sv, axis=0) + h * E
        gn = np.sqrt(1.0 + (un * un).sum(axis=0))
        u[:, s + 1] = un
        x[:, s + 1] = xh + 0.5 * dt * un / gn
    return x, u
