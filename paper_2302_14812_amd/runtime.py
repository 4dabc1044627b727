"""The run-time mode (Sec. 3.1): the deposit as a sub-step right after the push.

Particles are pushed on the device (radio_push) one block of steps at a time
into a resident chunk, and the block is deposited into every detector at once
(radio_deposit_batch) before the next push; the last state of a block becomes
state 0 of the next, so consecutive blocks share one state as the deposit
requires, and no state ever leaves device memory.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

import paper_2302_14812_amd as radio


class RunTimeDiagnostic:
    """Push-and-deposit driver.

    detectors: radio.Detector objects receiving every block.  x0, u0: (3, Np)
    initial positions and momenta (host arrays or device tensors).  q: (Np,)
    charges or None (electrons).  block_steps: steps per push-deposit cycle.
    fields: keyword arguments of radio.push (qm, E, B, wave_*).
    """

    def __init__(self, detectors: Sequence["radio.Detector"], x0, u0, q=None, *, dt: float,
                 block_steps: int = 16, t_first: float = 0.0, first_step: int = 0,
                 fields: Optional[dict] = None):
        import torch
        if block_steps < 1:
            raise ValueError("block_steps must be at least 1")
        self.detectors = list(detectors)
        self.fields = dict(fields or {})
        x0 = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
        u0 = torch.as_tensor(u0, dtype=torch.float64, device="cuda")
        if x0.dim() != 2 or x0.shape[0] != 3 or u0.shape != x0.shape:
            raise ValueError("x0 and u0 must have shape (3, Np)")
        n_p = x0.shape[1]
        x = torch.empty((3, block_steps + 1, n_p), dtype=torch.float64, device="cuda")
        u = torch.empty_like(x)
        x[:, 0] = x0
        u[:, 0] = u0
        qd = None if q is None else torch.as_tensor(q, dtype=torch.float64, device="cuda").contiguous()
        self.chunk = radio.Chunk(x, u, qd, t_first, dt, first_step)
        self.block_steps = block_steps

    @property
    def step(self) -> int:
        """Index in the run of the current state (state 0 of the resident chunk)."""
        return self.chunk.first_step

    def advance(self, n_blocks: int = 1, stream=None) -> None:
        """Push and deposit n_blocks blocks, all enqueued on `stream`."""
        for _ in range(n_blocks):
            radio.push(self.chunk, stream=stream, **self.fields)
            radio.deposit_batch(self.detectors, [self.chunk] * len(self.detectors), stream)
            # the last state starts the next block (ordered after the deposit's reads)
            import torch
            with torch.cuda.stream(stream) if stream is not None else _null():
                self.chunk.x[:, 0] = self.chunk.x[:, -1]
                self.chunk.u[:, 0] = self.chunk.u[:, -1]
            self.chunk.first_step += self.block_steps

    def state(self):
        """The current positions and momenta, (3, Np) device tensors."""
        return self.chunk.x[:, 0], self.chunk.u[:, 0]


def plane_wave_electrons(n_p: int = 10000, block_steps: int = 16, n_blocks: int = 64,
                         dt: float = 0.05, n_cells_side: int = 128, n_t: int = 2048, seed: int = 700):
    """The run-time benchmark's setting: n_p electrons at rest, uniform in a box of
    side 4, driven by a plane wave (a = 1.5, omega = 1, along +x, polarised along
    +y) for block_steps * n_blocks steps of dt, seen by an n_cells_side^2 cap of a
    sphere of radius 1e4 about +x (+-0.3 rad) with n_t slots over the arrival
    window of a 64-electron sample pushed on the device.  Returns (cells, t0,
    dt_det, n_t, x0, u0, fields) with x0, u0 host arrays (3, n_p) and fields the
    keyword arguments of radio.push."""
    import torch

    from paper_2302_14812_amd import workloads as W
    rng = np.random.Generator(np.random.PCG64(W.BASE_SEED + seed))
    x0 = rng.uniform(-2.0, 2.0, size=(3, n_p))
    u0 = np.zeros((3, n_p))
    wave = {"qm": -1.0, "wave_amplitude": 1.5, "wave_dir": [1.0, 0.0, 0.0],
            "wave_pol": [0.0, 1.0, 0.0], "wave_omega": 1.0, "wave_phase": 0.0}
    xs = torch.zeros((3, block_steps * n_blocks + 1, 64), dtype=torch.float64, device="cuda")
    us = torch.zeros_like(xs)
    xs[:, 0] = torch.from_numpy(x0[:, :64]).cuda()
    sample = radio.push(radio.Chunk(xs, us, None, 0.0, dt), **wave)
    cells = W.sphere_cap_cells(1e4, [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], n_cells_side, n_cells_side,
                               0.3, 0.3)
    host = W.Chunk(x=sample.x.cpu().numpy(), u=sample.u.cpu().numpy(), q=np.full(64, -1.0),
                   t_first=0.0, dt=dt)
    t0, dtd = W.arrival_window(cells, host, n_t, pad_frac=0.05)
    return cells, t0, dtd, n_t, x0, u0, wave


class _null:
    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False
