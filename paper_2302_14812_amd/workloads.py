"""Seeded synthetic inputs shaped like the paper's radiation workloads.

This module only builds inputs: particle trajectories (positions and momenta
sampled at the trajectory steps), per-particle charges, detector cell
positions and a detector time window.  It holds none of the radiation
arithmetic (no field evaluation, no deposit), so the CPU oracle and the GPU
library can both be fed from it without sharing any of the method.

Conventions (Sec. 2 and the helical example of Sec. 3 of the paper):
Gaussian units with c = 1, lengths in c/omega_n, times in 1/omega_n, charge
in units of e (electrons carry q = -1), momentum u = p/(m c) = gamma*beta.

Array layout handed to both sides (structure of arrays, float64):
    x[k, s, p]  position component k of particle p at trajectory state s
    u[k, s, p]  momentum component k (units of m c)
    q[p]        signed charge
State s of a chunk sits at time t_first + (first_step + s)*dt; S segments join
S+1 states.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 230214812


@dataclasses.dataclass
class Chunk:
    """A block of trajectory states: S+1 states of n_particles particles.

    State s of the block is state first_step + s of its run, at time
    t_first + (first_step + s) * dt."""

    x: np.ndarray  # (3, S+1, Np) float64
    u: np.ndarray  # (3, S+1, Np) float64
    q: np.ndarray  # (Np,) float64
    t_first: float
    dt: float
    first_step: int = 0

    @property
    def n_particles(self) -> int:
        return int(self.x.shape[2])

    @property
    def n_steps(self) -> int:
        return int(self.x.shape[1]) - 1

    def state_times(self) -> np.ndarray:
        steps = self.first_step + np.arange(self.n_steps + 1, dtype=np.int64)
        return self.t_first + steps.astype(np.float64) * self.dt

    def slice_steps(self, s_begin: int, s_end: int) -> "Chunk":
        """States s_begin..s_end inclusive (segments s_begin+1..s_end), at the same times."""
        return Chunk(
            x=np.ascontiguousarray(self.x[:, s_begin:s_end + 1, :]),
            u=np.ascontiguousarray(self.u[:, s_begin:s_end + 1, :]),
            q=self.q,
            t_first=self.t_first,
            dt=self.dt,
            first_step=self.first_step + s_begin,
        )

    def slice_particles(self, p_begin: int, p_end: int) -> "Chunk":
        return Chunk(
            x=np.ascontiguousarray(self.x[:, :, p_begin:p_end]),
            u=np.ascontiguousarray(self.u[:, :, p_begin:p_end]),
            q=np.ascontiguousarray(self.q[p_begin:p_end]),
            t_first=self.t_first,
            dt=self.dt,
            first_step=self.first_step,
        )


@dataclasses.dataclass
class DetectorSpec:
    """Detector cells plus one uniform time array (t0, dt_det, n_t)."""

    cells: np.ndarray  # (Nc, 3) float64
    t0: float
    dt_det: float
    n_t: int
    c: float = 1.0
    grid: Tuple[int, int] = (0, 0)  # (n1, n2) when the cells come from a 2-D grid
    options: int = 0                # detector options: 1 far field (Eq. 3), 2 acceleration only

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    detector: DetectorSpec
    chunk: Chunk

    @property
    def interactions(self) -> int:
        return self.chunk.n_particles * self.chunk.n_steps * self.detector.n_cells


# --------------------------------------------------------------------------
# detector geometries (Sec. 3.1: spherical grids centred at the origin and
# cartesian planes); cell index c = i2*n1 + i1
# --------------------------------------------------------------------------

def _unit(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


def plane_cells(center, e1, e2, n1: int, n2: int, half1: float, half2: float) -> np.ndarray:
    """Cell centres of an n1 x n2 cartesian grid spanning +-half1, +-half2."""
    center = np.asarray(center, dtype=np.float64)
    e1 = _unit(e1)
    e2 = _unit(e2)
    a1 = -half1 + (np.arange(n1) + 0.5) * (2.0 * half1 / n1)
    a2 = -half2 + (np.arange(n2) + 0.5) * (2.0 * half2 / n2)
    A2, A1 = np.meshgrid(a2, a1, indexing="ij")  # (n2, n1)
    pos = center[None, None, :] + A1[..., None] * e1 + A2[..., None] * e2
    return np.ascontiguousarray(pos.reshape(n1 * n2, 3))


def sphere_cap_cells(radius: float, axis, e1, n1: int, n2: int,
                     half1: float, half2: float) -> np.ndarray:
    """Cells on a sphere of the given radius centred at the origin.

    Longitude (about e2 = axis x e1) spans +-half1 and latitude spans
    +-half2, both measured from `axis`; cell centres sit at the middle of
    each angular bin.
    """
    axis = _unit(axis)
    e1 = np.asarray(e1, dtype=np.float64)
    e1 = _unit(e1 - np.dot(e1, axis) * axis)
    e2 = np.cross(axis, e1)
    lon = -half1 + (np.arange(n1) + 0.5) * (2.0 * half1 / n1)
    lat = -half2 + (np.arange(n2) + 0.5) * (2.0 * half2 / n2)
    LAT, LON = np.meshgrid(lat, lon, indexing="ij")  # (n2, n1)
    d = (np.cos(LAT)[..., None] * (np.cos(LON)[..., None] * axis + np.sin(LON)[..., None] * e1)
         + np.sin(LAT)[..., None] * e2)
    return np.ascontiguousarray((radius * d).reshape(n1 * n2, 3))


def sphere_shell_cells(radii: Sequence[float], axis, e1, n1: int, n2: int, half1: float,
                       half2: float) -> np.ndarray:
    """Concentric caps, one per radius, in the order of the radii."""
    return np.ascontiguousarray(np.concatenate(
        [sphere_cap_cells(r, axis, e1, n1, n2, half1, half2) for r in radii]))


def arrival_window(cells: np.ndarray, chunk: Chunk, n_t: int, pad_frac: float = 0.02,
                   max_particles: int = 64, cell_index: Optional[Sequence[int]] = None,
                   seed: int = 0, c: float = 1.0) -> Tuple[float, float]:
    """Pick a detector time window (t0, dt_det) for a workload.

    Light-travel bounds over a sample: min/max of t_s + |x_cell - x_s|/c over
    every state of a seeded subsample of particles and a subset of cells,
    padded by pad_frac of the width on both sides.  Only the window choice
    depends on this; both implementations receive the same (t0, dt_det).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_p = chunk.n_particles
    if n_p <= max_particles:
        pidx = np.arange(n_p)
    else:
        pidx = np.sort(rng.choice(n_p, size=max_particles, replace=False))
    if cell_index is None:
        cell_index = np.arange(cells.shape[0])
    cidx = np.asarray(cell_index)
    t = chunk.state_times()
    xs = chunk.x[:, :, pidx]  # (3, S+1, P)
    lo, hi = np.inf, -np.inf
    for ci in cidx:
        d = cells[ci][:, None, None] - xs
        tt = t[:, None] + np.sqrt((d * d).sum(axis=0)) / c
        lo = min(lo, float(tt.min()))
        hi = max(hi, float(tt.max()))
    w = hi - lo
    t0 = lo - pad_frac * w
    t1 = hi + pad_frac * w
    return t0, (t1 - t0) / n_t


def grid_corner_cells(n1: int, n2: int) -> List[int]:
    """Centre and four corners of an n1 x n2 grid (indices c = i2*n1 + i1)."""
    pts = [(n1 // 2, n2 // 2), (0, 0), (n1 - 1, 0), (0, n2 - 1), (n1 - 1, n2 - 1)]
    return [i2 * n1 + i1 for (i1, i2) in pts]


# --------------------------------------------------------------------------
# trajectories
# --------------------------------------------------------------------------

def circular_orbit(gamma: float = 5.0, radius: float = 1.0, n_steps: int = 2000,
                   dt: float = 0.01, q: float = -1.0, phase: float = 0.0) -> Chunk:
    """One charge in uniform circular motion in the x-y plane about the origin."""
    beta = math.sqrt(1.0 - 1.0 / (gamma * gamma))
    omega = beta / radius
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    ph = omega * t + phase
    x = np.zeros((3, n_steps + 1, 1))
    u = np.zeros((3, n_steps + 1, 1))
    x[0, :, 0] = radius * np.cos(ph)
    x[1, :, 0] = radius * np.sin(ph)
    gb = gamma * beta
    u[0, :, 0] = -gb * np.sin(ph)
    u[1, :, 0] = gb * np.cos(ph)
    return Chunk(x=x, u=u, q=np.full(1, q), t_first=0.0, dt=dt)


def planar_undulator(n_particles: int, n_steps: int, periods: float, gamma_mean: float,
                     gamma_sigma: float, K: float, offset_sigma: float, seed: int,
                     omega_u: float = 1.0, q: float = -1.0, substeps: int = 8) -> Chunk:
    """Electrons wiggling in x with u_x = K sin(omega_u t), |u| constant.

    x(t) = x0 + K/(gamma omega_u) (1 - cos omega_u t); z(t) integrates
    beta_z with a substepped Simpson rule; transverse offsets x0, y0 are
    normal with the given sigma, z0 = 0.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gam = rng.normal(gamma_mean, gamma_sigma, size=n_particles)
    x0 = rng.normal(0.0, offset_sigma, size=n_particles)
    y0 = rng.normal(0.0, offset_sigma, size=n_particles)
    T = periods * 2.0 * math.pi / omega_u
    dt = T / n_steps
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    x = np.empty((3, n_steps + 1, n_particles))
    u = np.empty((3, n_steps + 1, n_particles))
    s_om = np.sin(omega_u * t)
    ux = K * s_om[:, None] * np.ones((1, n_particles))
    u[0] = ux
    u[1] = 0.0
    u[2] = np.sqrt(gam[None, :] ** 2 - 1.0 - ux * ux)
    x[0] = x0[None, :] + (K / (gam[None, :] * omega_u)) * (1.0 - np.cos(omega_u * t))[:, None]
    x[1] = y0[None, :]
    # z: Simpson over each step with 2*substeps sub-intervals
    m = 2 * substeps
    wts = np.ones(m + 1)
    wts[1:m:2] = 4.0
    wts[2:m:2] = 2.0
    wts *= (dt / m) / 3.0
    frac = np.arange(m + 1, dtype=np.float64) / m
    g2 = gam * gam
    z = np.zeros(n_particles)
    x[2, 0] = 0.0
    for s in range(n_steps):
        ts = t[s] + frac * dt
        uxs = K * np.sin(omega_u * ts)  # (m+1,)
        bz = np.sqrt(g2[None, :] - 1.0 - (uxs * uxs)[:, None]) / gam[None, :]
        z = z + wts @ bz
        x[2, s + 1] = z
    return Chunk(x=x, u=u, q=np.full(n_particles, q), t_first=0.0, dt=dt)


def sinusoidal_orbit(n_steps: int, gamma: float = 50.0, r_beta: float = 2.0,
                     k_beta: float = 0.1, dt: float = 0.01, q: float = -1.0,
                     substeps: int = 8) -> Chunk:
    """One electron moving along x with a sinusoidal excursion in y (the paper's
    spectral benchmark: gamma 50, r_beta = 2, k_beta = 0.1, so K = gamma k_beta
    r_beta = 10, dt = 0.01, in units where c = 1).

    u_y = K cos(k_beta t), |u| constant; y = r_beta sin(k_beta t) exactly and x
    integrates beta_x with a substepped Simpson rule.
    """
    K = gamma * k_beta * r_beta
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    x = np.zeros((3, n_steps + 1, 1))
    u = np.zeros((3, n_steps + 1, 1))
    uy = K * np.cos(k_beta * t)
    u[1, :, 0] = uy
    u[0, :, 0] = np.sqrt(gamma * gamma - 1.0 - uy * uy)
    x[1, :, 0] = (K / (gamma * k_beta)) * np.sin(k_beta * t)
    m = 2 * substeps
    wts = np.ones(m + 1)
    wts[1:m:2] = 4.0
    wts[2:m:2] = 2.0
    wts *= (dt / m) / 3.0
    frac = np.arange(m + 1, dtype=np.float64) / m
    xs = 0.0
    for s in range(n_steps):
        uys = K * np.cos(k_beta * (t[s] + frac * dt))
        xs += wts @ (np.sqrt(gamma * gamma - 1.0 - uys * uys) / gamma)
        x[0, s + 1, 0] = xs
    return Chunk(x=x, u=u, q=np.full(1, q), t_first=0.0, dt=dt)


def line_cells(radius: float, n: int, half: float) -> np.ndarray:
    """A line of cells on a sphere about the origin in the z-x plane, at angles
    -half..half from the x axis (bin middles), as the spectral benchmark's detector."""
    return sphere_cap_cells(radius, [1.0, 0.0, 0.0], [0.0, 0.0, 1.0], n, 1, half, 0.0)


def helical_undulator(n_particles: int, n_steps: int, periods: float, gamma_mean: float,
                      gamma_sigma: float, K: float, offset_sigma: float, seed: int,
                      omega_u: float = 1.0, q: float = -1.0) -> Chunk:
    """Electrons on a helix about z: u_perp = K(cos, sin)(omega_u t), u_z constant."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gam = rng.normal(gamma_mean, gamma_sigma, size=n_particles)
    x0 = rng.normal(0.0, offset_sigma, size=n_particles)
    y0 = rng.normal(0.0, offset_sigma, size=n_particles)
    T = periods * 2.0 * math.pi / omega_u
    dt = T / n_steps
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    uz = np.sqrt(gam * gam - 1.0 - K * K)
    x = np.empty((3, n_steps + 1, n_particles))
    u = np.empty((3, n_steps + 1, n_particles))
    c_om = np.cos(omega_u * t)[:, None]
    s_om = np.sin(omega_u * t)[:, None]
    u[0] = K * c_om * np.ones((1, n_particles))
    u[1] = K * s_om * np.ones((1, n_particles))
    u[2] = uz[None, :] * np.ones((n_steps + 1, 1))
    r = (K / (gam * omega_u))[None, :]
    x[0] = x0[None, :] + r * s_om
    x[1] = y0[None, :] + r * (1.0 - c_om)
    x[2] = (uz / gam)[None, :] * t[:, None]
    return Chunk(x=x, u=u, q=np.full(n_particles, q), t_first=0.0, dt=dt)


def plasma_mirror_sheet(n_particles: int, n_steps: int, periods: float, seed: int,
                        gamma_peak: float = 10.0, half_width_wavelengths: float = 10.0,
                        incidence: float = math.pi / 4, jitter: float = 0.01,
                        q: float = -1.0) -> Chunk:
    """Electrons on the sheet x = 0 driven normal to it by an oblique wave.

    Laser units (omega = 1, lambda = 2 pi).  beta_x0 = A cos(t - k_y y0)
    with k_y = sin(incidence) and A set so that the peak gamma is
    gamma_peak; every particle carries a fixed momentum jitter of
    `jitter` times the peak momentum per component.  Positions integrate
    beta with the trapezoid rule.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = 2.0 * math.pi
    hw = half_width_wavelengths * lam
    y0 = rng.uniform(-hw, hw, size=n_particles)
    z0 = rng.uniform(-hw, hw, size=n_particles)
    A = math.sqrt(1.0 - 1.0 / (gamma_peak * gamma_peak))
    u_peak = gamma_peak * A
    du = rng.normal(0.0, jitter * u_peak, size=(3, n_particles))
    ky = math.sin(incidence)
    T = periods * lam
    dt = T / n_steps
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    x = np.empty((3, n_steps + 1, n_particles))
    u = np.empty((3, n_steps + 1, n_particles))
    phase0 = ky * y0
    beta_prev = None
    pos = np.stack([np.zeros(n_particles), y0, z0])
    for s in range(n_steps + 1):
        bx = A * np.cos(t[s] - phase0)
        ux0 = bx / np.sqrt(1.0 - bx * bx)
        us = du.copy()
        us[0] += ux0
        u[:, s, :] = us
        beta = us / np.sqrt(1.0 + (us * us).sum(axis=0))[None, :]
        if beta_prev is not None:
            pos = pos + 0.5 * dt * (beta_prev + beta)
        x[:, s, :] = pos
        beta_prev = beta
    return Chunk(x=x, u=u, q=np.full(n_particles, q), t_first=0.0, dt=dt)


def static_charges(positions: np.ndarray, n_steps: int, dt: float, q) -> Chunk:
    """Charges at rest at the given (Np, 3) positions."""
    positions = np.asarray(positions, dtype=np.float64)
    n_p = positions.shape[0]
    x = np.repeat(positions.T[:, None, :], n_steps + 1, axis=1)
    u = np.zeros_like(x)
    return Chunk(x=np.ascontiguousarray(x), u=u, q=np.broadcast_to(np.asarray(q, dtype=np.float64),
                                                                    (n_p,)).copy(),
                 t_first=0.0, dt=dt)


def uniform_motion(x0: np.ndarray, u: np.ndarray, n_steps: int, dt: float, q,
                   t_first: float = 0.0) -> Chunk:
    """Charges moving with constant momenta u (Np, 3) from positions x0 (Np, 3)."""
    x0 = np.asarray(x0, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    beta = u / np.sqrt(1.0 + (u * u).sum(axis=1))[:, None]
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    x = x0.T[:, None, :] + beta.T[:, None, :] * t[None, :, None]
    uu = np.repeat(u.T[:, None, :], n_steps + 1, axis=1)
    n_p = x0.shape[0]
    return Chunk(x=np.ascontiguousarray(x), u=np.ascontiguousarray(uu),
                 q=np.broadcast_to(np.asarray(q, dtype=np.float64), (n_p,)).copy(),
                 t_first=t_first, dt=dt)


def random_chunk(n_particles: int, n_steps: int, seed: int, dt: float = 0.05,
                 gamma_max: float = 20.0, spread: float = 1.0, t_first: float = 0.0) -> Chunk:
    """Generic smooth random trajectories for parity tests.

    Each particle follows a sum of two random rotations of its momentum
    plus a random drift; positions integrate beta with the trapezoid rule,
    so every step moves less than c*dt.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    S = n_steps
    t = t_first + np.arange(S + 1, dtype=np.float64) * dt
    g0 = np.exp(rng.uniform(0.0, math.log(gamma_max), size=n_particles))
    ub = np.sqrt(g0 * g0 - 1.0)
    d0 = rng.normal(size=(3, n_particles))
    d0 /= np.linalg.norm(d0, axis=0)
    a1 = rng.normal(size=(3, n_particles)) * 0.5 * ub
    a2 = rng.normal(size=(3, n_particles)) * 0.2 * ub
    w1 = rng.uniform(0.2, 3.0, size=n_particles)
    w2 = rng.uniform(0.5, 7.0, size=n_particles)
    ph = rng.uniform(0, 2 * math.pi, size=(2, n_particles))
    u = (ub * d0)[:, None, :] + a1[:, None, :] * np.sin(w1[None, :] * t[:, None] + ph[0])[None] \
        + a2[:, None, :] * np.cos(w2[None, :] * t[:, None] + ph[1])[None]
    beta = u / np.sqrt(1.0 + (u * u).sum(axis=0))[None]
    x = np.empty_like(u)
    x[:, 0, :] = rng.normal(size=(3, n_particles)) * spread
    for s in range(1, S + 1):
        x[:, s, :] = x[:, s - 1, :] + 0.5 * dt * (beta[:, s - 1, :] + beta[:, s, :])
    q = rng.choice(np.array([-1.0, 1.0, -2.0, 0.5]), size=n_particles)
    return Chunk(x=np.ascontiguousarray(x), u=np.ascontiguousarray(u), q=q, t_first=t_first, dt=dt)


def split_steps(chunk: Chunk, bounds: Sequence[int]) -> List[Chunk]:
    """Cut a chunk at the given state indices, sharing one state at each cut."""
    edges = [0] + [int(b) for b in bounds] + [chunk.n_steps]
    return [chunk.slice_steps(a, b) for a, b in zip(edges[:-1], edges[1:]) if b > a]


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def circular_workload(n_side: int = 32, n_t: int = 512, n_steps: int = 2000) -> Workload:
    """One electron, gamma 5, radius 1, dt 0.01; 32x32 plane at z = 1000 spanning +-50."""
    chunk = circular_orbit(gamma=5.0, radius=1.0, n_steps=n_steps, dt=0.01, q=-1.0)
    cells = plane_cells([0, 0, 1000.0], [1, 0, 0], [0, 1, 0], n_side, n_side, 50.0, 50.0)
    t0, dtd = arrival_window(cells, chunk, n_t, pad_frac=0.002)
    det = DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t, grid=(n_side, n_side))
    return Workload("circular_gamma5_1e_32x32_512bins", det, chunk)


def undulator_workload(n_particles: int = 10_000, n_steps: int = 4096, n_side: int = 128,
                       n_t: int = 2048, seed_offset: int = 2) -> Workload:
    """Planar undulator ensemble: gamma ~ N(50, 0.5), K = 1, 20 periods; 1e5 sphere cap."""
    seed = BASE_SEED + seed_offset
    chunk = planar_undulator(n_particles, n_steps, periods=20.0, gamma_mean=50.0, gamma_sigma=0.5,
                             K=1.0, offset_sigma=0.1, seed=seed)
    cells = sphere_cap_cells(1.0e5, [0, 0, 1], [1, 0, 0], n_side, n_side, 0.04, 0.04)
    t0, dtd = arrival_window(cells, chunk, n_t, cell_index=grid_corner_cells(n_side, n_side),
                             seed=seed)
    det = DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t, grid=(n_side, n_side))
    return Workload(f"undulator_{n_particles}e_{n_steps}steps_{n_side}x{n_side}_{n_t}bins", det, chunk)


def plasma_mirror_workload(n_particles: int = 200_000, n_steps: int = 1000, n_side: int = 256,
                           n_t: int = 4096, seed_offset: int = 3) -> Workload:
    """Sheet of electrons driven at 45 degrees, peak gamma 10; cap on the specular direction."""
    seed = BASE_SEED + seed_offset
    chunk = plasma_mirror_sheet(n_particles, n_steps, periods=10.0, seed=seed)
    inc = math.pi / 4
    axis = [-math.cos(inc), math.sin(inc), 0.0]
    cells = sphere_cap_cells(1.0e5, axis, [math.sin(inc), math.cos(inc), 0.0], n_side, n_side,
                             0.1, 0.1)
    t0, dtd = arrival_window(cells, chunk, n_t, cell_index=grid_corner_cells(n_side, n_side),
                             seed=seed)
    det = DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t, grid=(n_side, n_side))
    return Workload(f"plasma_mirror_{n_particles}e_{n_steps}steps_{n_side}x{n_side}_{n_t}bins",
                    det, chunk)


def batched_sets(n_sets: int = 64, seed_offset: int = 4, scale: float = 1.0,
                 max_particles: int = 100_000, max_steps: int = 4000,
                 sides: Sequence[int] = (32, 64, 128, 256),
                 n_t_choices: Sequence[int] = (256, 512, 1024, 2048, 4096)) -> List[Workload]:
    """Independent trajectory sets of uneven size, each with its own detector.

    Particle counts are log-uniform in [1e2, max_particles] (times `scale`),
    steps uniform in [500, max_steps], gamma0 uniform in [2, 100], helical
    or sinusoidal motion with equal probability, K uniform in [0.5, 3].
    """
    out = []
    for i in range(n_sets):
        seed = BASE_SEED + seed_offset + 1000 * i
        rng = np.random.Generator(np.random.PCG64(seed))
        n_p = max(1, int(round(10 ** rng.uniform(2.0, math.log10(max_particles)) * scale)))
        n_s = int(rng.integers(min(500, max_steps), max_steps + 1))
        helical = bool(rng.integers(0, 2))
        g0 = float(rng.uniform(2.0, 100.0))
        K = float(rng.uniform(0.5, 3.0))
        side = int(rng.choice(np.asarray(sides)))
        n_t = int(rng.choice(np.asarray(n_t_choices)))
        periods = 4.0
        if helical:
            K = min(K, math.sqrt(max(g0 * g0 * 0.98 * 0.98 - 1.0, 0.0)) * 0.5)
            chunk = helical_undulator(n_p, n_s, periods, g0, 0.01 * g0, K, 0.1, seed + 1)
        else:
            chunk = planar_undulator(n_p, n_s, periods, g0, 0.01 * g0, K, 0.1, seed + 1, substeps=2)
        half = (1.0 + K) / g0
        cells = sphere_cap_cells(1.0e4, [0, 0, 1], [1, 0, 0], side, side, half, half)
        t0, dtd = arrival_window(cells, chunk, n_t, cell_index=grid_corner_cells(side, side),
                                 seed=seed)
        det = DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t, grid=(side, side))
        out.append(Workload(f"set{i}_{'helix' if helical else 'planar'}_{n_p}e_{n_s}s_{side}_{n_t}",
                            det, chunk))
    return out


def stream_schedule(n_chunks: int, n_detectors: int, seed: int, min_steps: int = 1,
                    max_steps: int = 64, min_log_particles: float = 3.0,
                    max_log_particles: float = 5.0, total_steps: int = 1000
                    ) -> Iterator[Tuple[int, int, int, int]]:
    """Yield (detector, first_state, n_steps, n_particles) for a chunk stream.

    Each detector keeps a step cursor that advances by the chunk length and
    wraps at total_steps; the target detector is uniform.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cursor = [0] * n_detectors
    for _ in range(n_chunks):
        d = int(rng.integers(0, n_detectors))
        s = int(rng.integers(min_steps, max_steps + 1))
        n = int(round(10 ** rng.uniform(min_log_particles, max_log_particles)))
        if cursor[d] + s > total_steps:
            cursor[d] = 0
        yield d, cursor[d], s, n
        cursor[d] += s


def plasma_mirror_chunk(n_particles: int, s_begin: int, n_steps: int, seed: int,
                        steps_total: int = 1000, periods: float = 10.0, gamma_peak: float = 10.0,
                        half_width_wavelengths: float = 10.0, incidence: float = math.pi / 4,
                        jitter: float = 0.01, q: float = -1.0) -> Chunk:
    """A chunk of the plasma-mirror sheet as a running simulation would emit it.

    Fresh particles drawn like plasma_mirror_sheet, states s_begin ..
    s_begin + n_steps of a run of steps_total steps over `periods` laser
    periods.  The position at s_begin follows the unjittered motion in closed
    form (x = A (sin(t - k_y y0) + sin(k_y y0))); within the chunk positions
    integrate the jittered beta with the trapezoid rule, so every step moves
    less than c dt.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = 2.0 * math.pi
    hw = half_width_wavelengths * lam
    y0 = rng.uniform(-hw, hw, size=n_particles)
    z0 = rng.uniform(-hw, hw, size=n_particles)
    A = math.sqrt(1.0 - 1.0 / (gamma_peak * gamma_peak))
    u_peak = gamma_peak * A
    du = rng.normal(0.0, jitter * u_peak, size=(3, n_particles))
    ky = math.sin(incidence)
    dt = periods * lam / steps_total
    t = (s_begin + np.arange(n_steps + 1, dtype=np.float64)) * dt
    phase0 = ky * y0
    x = np.empty((3, n_steps + 1, n_particles))
    u = np.empty((3, n_steps + 1, n_particles))
    pos = np.stack([A * (np.sin(t[0] - phase0) + np.sin(phase0)), y0, z0])
    beta_prev = None
    for s in range(n_steps + 1):
        bx = A * np.cos(t[s] - phase0)
        us = du.copy()
        us[0] += bx / np.sqrt(1.0 - bx * bx)
        u[:, s, :] = us
        beta = us / np.sqrt(1.0 + (us * us).sum(axis=0))[None, :]
        if beta_prev is not None:
            pos = pos + 0.5 * dt * (beta_prev + beta)
        x[:, s, :] = pos
        beta_prev = beta
    return Chunk(x=x, u=u, q=np.full(n_particles, q), t_first=0.0, dt=dt, first_step=s_begin)


def plasma_mirror_detector(n_side: int = 256, n_t: int = 4096, seed: int = BASE_SEED + 3,
                           sample_particles: int = 64) -> DetectorSpec:
    """The plasma-mirror detector (cap about the specular direction at 1e5, +-0.1 rad)
    with its window chosen from a sample of the whole 1000-step run."""
    inc = math.pi / 4
    axis = [-math.cos(inc), math.sin(inc), 0.0]
    cells = sphere_cap_cells(1.0e5, axis, [math.sin(inc), math.cos(inc), 0.0], n_side, n_side,
                             0.1, 0.1)
    sample = plasma_mirror_sheet(sample_particles, 1000, periods=10.0, seed=seed)
    t0, dtd = arrival_window(cells, sample, n_t, cell_index=grid_corner_cells(n_side, n_side),
                             seed=seed)
    return DetectorSpec(cells=cells, t0=t0, dt_det=dtd, n_t=n_t, grid=(n_side, n_side))
