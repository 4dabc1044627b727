"""A streaming deposit service: trajectory chunks in, detector fields kept in HBM.

The service models the paper's run-time mode (Sec. 3.1: the deposit as a
sub-step after each particle push) for many detectors at once.  Producers
submit chunks -- a few steps of many particles, sharing one state with the
previous chunk of the same detector -- as the simulation emits them.  The
service keeps every detector's accumulated fields resident in device memory,
admits detectors while their memory fits a budget, and deposits whatever is
pending in batches: chunks that arrive while a batch is on the GPU join the
next batch, and one batch is prepared while the previous one runs (the
library alternates two batch workspaces).  Each chunk's latency is the time
from submission until the batch that carried it has finished on the device.

Two layers:
  Scheduler      pure bookkeeping (admission by memory, batch formation),
                 testable without a GPU with a fake clock;
  DepositServer  the threads that drive the library on a dedicated stream.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Request:
    det_id: int
    n_particles: int
    n_steps: int
    arrival: float
    payload: object = None            # the device chunk (DepositServer) or anything (tests)
    work: int = 0                     # interactions: n_particles * n_steps * n_cells
    ready: object = None              # event on the producer's stream after the chunk was written
    pieces: Optional[List[Tuple[object, int]]] = None  # (payload, work) parts, in order
    next_piece: int = 0               # parts handed to batches so far
    open_pieces: int = 0              # parts handed out and not yet finished
    batch: int = -1                   # index of the batch that carried its last part
    launched: Optional[float] = None  # when its first part was launched
    completion: Optional[float] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.completion is None else self.completion - self.arrival


def plan_pieces(n_particles: int, n_steps: int, n_cells: int, piece_work: float,
                min_steps: int = 16) -> List[Tuple[int, int, int, int]]:
    """Cut a chunk into parts of at most about piece_work interactions.

    Parts are (s_begin, s_end, p_begin, p_end): states s_begin..s_end (sharing
    one state with the neighbouring part, so the parts add up to the whole) of
    particles p_begin..p_end-1.  Steps are cut first, into ranges of at least
    min_steps (one pass of the deposit over the particle order covers that
    many); particles are cut after that.
    """
    work = n_particles * n_steps * n_cells
    if work <= piece_work or n_particles == 0 or n_steps == 0:
        return [(0, n_steps, 0, n_particles)]
    n_s = int(min(math.ceil(work / piece_work), max(1, n_steps // min_steps)))
    sb = np.linspace(0, n_steps, n_s + 1).round().astype(int)
    parts = []
    for a, b in zip(sb[:-1], sb[1:]):
        w = n_particles * (b - a) * n_cells
        n_p = int(min(math.ceil(w / piece_work), n_particles))
        pb = np.linspace(0, n_particles, n_p + 1).round().astype(int)
        parts.extend((int(a), int(b), int(p0), int(p1)) for p0, p1 in zip(pb[:-1], pb[1:]))
    return parts


class Scheduler:
    """Admission by memory and batch formation over the parts of the requests.

    A detector becomes resident when a pending request for it is considered
    and its bytes fit the budget next to the resident detectors; requests for
    detectors that do not fit wait (and do not block requests for resident
    detectors behind them).  A batch visits the pending requests of resident
    detectors in arrival order and takes the next part of each, round after
    round, until max_batch_work interactions or max_batch_segments particle
    segments (a batch takes at least one part; the segments bound the state
    records and particle orders of the batch's workspace on small detectors):
    a request cut into many parts advances by a part per round and never
    holds back the requests that arrived after it for longer than a batch.
    """

    def __init__(self, detector_bytes: Dict[int, int], cells: Dict[int, int], budget: int,
                 max_batch_work: float, max_batch_segments: Optional[float] = None):
        self.detector_bytes = dict(detector_bytes)
        self.cells = dict(cells)
        self.budget = int(budget)
        self.max_batch_work = float(max_batch_work)
        self.max_batch_segments = float("inf") if max_batch_segments is None else float(
            max_batch_segments)
        self.resident: Dict[int, int] = {}
        self.finished: set = set()
        self.pending: Deque[Request] = collections.deque()
        self.admission_order: List[int] = []
        self.peak_used = 0
        self.peak_resident = 0
        self.n_batches = 0

    def add(self, req: Request) -> Request:
        if req.det_id not in self.detector_bytes:
            raise KeyError(f"unknown detector {req.det_id}")
        if req.det_id in self.finished:
            raise ValueError(f"detector {req.det_id} has been finished")
        if self.detector_bytes[req.det_id] > self.budget:
            raise ValueError(f"detector {req.det_id} needs {self.detector_bytes[req.det_id]} bytes,"
                             f" more than the budget of {self.budget}")
        req.work = req.n_particles * req.n_steps * self.cells[req.det_id]
        if req.pieces is None:
            req.pieces = [(req.payload, req.work)]
        self.pending.append(req)
        return req

    def used(self) -> int:
        return sum(self.resident.values())

    def admit(self) -> List[int]:
        """Make detectors resident for pending requests while they fit; return the new ones."""
        new = []
        for req in self.pending:
            d = req.det_id
            if d in self.resident or d in new:
                continue
            need = self.detector_bytes[d]
            if self.used() + sum(self.detector_bytes[n] for n in new) + need <= self.budget:
                new.append(d)
        for d in new:
            self.resident[d] = self.detector_bytes[d]
            self.admission_order.append(d)
        self.peak_used = max(self.peak_used, self.used())
        self.peak_resident = max(self.peak_resident, len(self.resident))
        return new

    def runnable(self) -> bool:
        """True if a batch could be formed now, possibly after admitting detectors."""
        free = self.budget - self.used()
        return any(r.det_id in self.resident or self.detector_bytes[r.det_id] <= free
                   for r in self.pending)

    def next_batch(self) -> List[Tuple[Request, int]]:
        """The next batch as (request, part index) pairs."""
        batch: List[Tuple[Request, int]] = []
        work = 0.0
        segs = 0.0
        progress = True
        while progress:
            progress = False
            for req in list(self.pending):
                if req.det_id not in self.resident:
                    continue
                k = req.next_piece
                w = req.pieces[k][1]
                g = w / max(1, self.cells[req.det_id])  # particle segments of the part
                if batch and (work + w > self.max_batch_work or
                              segs + g > self.max_batch_segments):
                    continue
                batch.append((req, k))
                work += w
                segs += g
                req.next_piece += 1
                req.open_pieces += 1
                req.batch = self.n_batches
                progress = True
                if req.next_piece == len(req.pieces):
                    self.pending.remove(req)
        if batch:
            self.n_batches += 1
        return batch

    def piece_done(self, req: Request) -> bool:
        """Record that one handed-out part of req finished; True when req is complete."""
        req.open_pieces -= 1
        return req.open_pieces == 0 and req.next_piece == len(req.pieces)

    def release(self, det_id: int) -> None:
        self.resident.pop(det_id, None)
        self.finished.add(det_id)


class DepositServer:
    """Threads around the library: a scheduler loop and a completion watcher.

    specs: detector id -> workloads.DetectorSpec.  memory_budget: bytes of
    device memory the service may hold (default: 90% of the free memory at
    start): the two batch workspaces of the library (reserved up front for
    batches of max_batch_work interactions and max_batch_segments particle
    segments, arena_bytes) and the resident detectors, each with its
    accumulator and the workspaces its own deposits may grow (resident_bytes).
    max_batch_work: interactions per batch; max_batch_segments: particle
    segments per batch (default max_batch_work / 4096: binding only for
    detectors of fewer than 4096 cells).  Chunks are cut into parts of at most
    piece_work interactions (default half a batch) and half a batch's segments.
    max_inflight: batches enqueued on the device at once; while that many run,
    arriving chunks wait and join the next batch (continuous batching).
    """

    def __init__(self, specs: Dict[int, object], precision: str = "mixed",
                 memory_budget: Optional[int] = None, max_batch_work: float = 4e10,
                 piece_work: Optional[float] = None, max_inflight: int = 2,
                 max_batch_segments: Optional[float] = None,
                 clock: Callable[[], float] = time.perf_counter):
        import torch

        import paper_2302_14812_amd as radio
        radio._lib()  # fail here, loudly, when the library is missing
        self._radio = radio
        self._torch = torch
        self.specs = dict(specs)
        self.precision = precision
        self.clock = clock
        if memory_budget is None:
            free, _ = torch.cuda.mem_get_info()
            memory_budget = int(0.9 * free)
        self.max_inflight = int(max_inflight)
        self.piece_work = float(max_batch_work / 2 if piece_work is None else piece_work)
        self.max_batch_segments = float(max_batch_work / 4096 if max_batch_segments is None
                                        else max_batch_segments)
        self.piece_segments = self.max_batch_segments / 2
        self.memory_budget = int(memory_budget)
        self.arena_reserve = 2 * arena_bytes(max_batch_work, self.max_batch_segments)
        if self.arena_reserve >= self.memory_budget:
            raise ValueError(f"the batch workspaces ({self.arena_reserve} bytes) leave no room for "
                             f"detectors in a budget of {self.memory_budget} bytes")
        self.sched = Scheduler({d: resident_bytes(s, self.piece_work)
                                for d, s in self.specs.items()},
                               {d: s.n_cells for d, s in self.specs.items()},
                               self.memory_budget - self.arena_reserve, max_batch_work,
                               self.max_batch_segments)
        self.detectors: Dict[int, object] = {}
        self.stream = torch.cuda.Stream()  # default priority
        self.requests: List[Request] = []
        self._lock = threading.Condition()
        self._inflight: Deque[Tuple[object, List[Tuple[Request, int]]]] = collections.deque()
        self._running = True
        self._error: Optional[BaseException] = None
        self._outstanding: Dict[int, int] = collections.defaultdict(int)
        self._sched_thread = threading.Thread(target=self._schedule_loop, daemon=True)
        self._done_thread = threading.Thread(target=self._completion_loop, daemon=True)
        self._sched_thread.start()
        self._done_thread.start()

    # ---------------------------------------------------------------- producer side
    def submit(self, det_id: int, chunk) -> Request:
        """Queue a device chunk (radio.Chunk) for detector det_id; returns its request.

        The chunk's arrays must stay unchanged until the request completes; the
        service orders its stream after the work the caller's current stream
        has enqueued so far (the writes of the chunk)."""
        torch = self._torch
        arrival = self.clock()
        if det_id not in self.specs:
            raise KeyError(f"unknown detector {det_id}")
        n_c = self.specs[det_id].n_cells
        plan = plan_pieces(chunk.n_particles, chunk.n_steps, n_c,
                           min(self.piece_work, self.piece_segments * n_c))
        if len(plan) == 1:
            pieces = [chunk]
        else:  # device copies, ordered on the caller's stream before the event below
            pieces = [chunk.slice(a, b, p0, p1) for a, b, p0, p1 in plan]
        n_c = self.specs[det_id].n_cells
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        req = Request(det_id, chunk.n_particles, chunk.n_steps, arrival, chunk, ready=ev,
                      pieces=[(c, c.n_particles * c.n_steps * n_c) for c in pieces])
        with self._lock:
            self._raise_if_failed()
            self.sched.add(req)
            self.requests.append(req)
            self._outstanding[det_id] += 1
            self._lock.notify_all()
        return req

    def finish(self, det_id: int, timeout: Optional[float] = None, read: str = "host"):
        """Wait for every chunk of det_id, read its fields and free its memory.

        read="host": return (E, B) as host arrays (n_cells, n_t, 3); "device":
        as device tensors; "none": return None.  A detector that never received
        a chunk reads as zeros.  No chunk may be submitted for det_id afterwards."""
        if read not in ("host", "device", "none"):
            raise ValueError("read must be 'host', 'device' or 'none'")
        t_end = None if timeout is None else time.monotonic() + timeout
        with self._lock:
            while self._outstanding[det_id] > 0:
                self._raise_if_failed()
                left = None if t_end is None else t_end - time.monotonic()
                if left is not None and left <= 0:
                    raise TimeoutError(f"detector {det_id} still has work")
                self._lock.wait(timeout=0.5 if left is None else min(left, 0.5))
            self._raise_if_failed()
            det = self.detectors.pop(det_id, None)
            self.sched.finished.add(det_id)  # reject late submissions from here on
        out = None
        if det is None:
            if read != "none":
                spec = self.specs[det_id]
                E = np.zeros((spec.n_cells, spec.n_t, 3))
                out = (E, np.zeros_like(E))
                if read == "device":
                    out = tuple(self._torch.from_numpy(a).cuda() for a in out)
        else:
            if read != "none":
                Et, Bt = det.read(stream=self.stream)
                self.stream.synchronize()
                out = (Et, Bt) if read == "device" else (Et.cpu().numpy(), Bt.cpu().numpy())
                del Et, Bt
            det.close()
        with self._lock:
            self.sched.release(det_id)
            self._lock.notify_all()
        return out

    def drain(self, timeout: Optional[float] = None) -> None:
        """Wait until every submitted chunk has been deposited."""
        t_end = None if timeout is None else time.monotonic() + timeout
        with self._lock:
            while any(v > 0 for v in self._outstanding.values()):
                self._raise_if_failed()
                left = None if t_end is None else t_end - time.monotonic()
                if left is not None and left <= 0:
                    raise TimeoutError("requests still outstanding")
                self._lock.wait(timeout=0.5 if left is None else min(left, 0.5))
            self._raise_if_failed()

    def close(self) -> None:
        with self._lock:
            self._running = False
            self._lock.notify_all()
        self._sched_thread.join()
        self._done_thread.join()
        self.stream.synchronize()
        for det in self.detectors.values():
            det.close()
        self.detectors.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ---------------------------------------------------------------- reporting
    def summary(self, skip: int = 0) -> dict:
        return summarize(self.requests, skip=skip, sched=self.sched)

    # ---------------------------------------------------------------- internals
    def _raise_if_failed(self) -> None:
        if self._error is not None:
            raise RuntimeError("deposit service failed") from self._error

    def _ready(self) -> bool:
        return len(self._inflight) < self.max_inflight and self.sched.runnable()

    def _schedule_loop(self) -> None:
        torch = self._torch
        radio = self._radio
        try:
            while True:
                with self._lock:
                    while self._running and not self._ready():
                        self._lock.wait(timeout=0.5)
                    if not self._running:
                        return
                    for d in self.sched.admit():
                        self.detectors[d] = radio.Detector.from_spec(
                            self.specs[d], precision=self.precision, stream=self.stream)
                    batch = self.sched.next_batch()
                    dets = [self.detectors[r.det_id] for r, _ in batch]
                if not batch:
                    continue
                t = self.clock()
                for r, k in batch:
                    if k == 0:
                        r.launched = t
                        self.stream.wait_event(r.ready)
                radio.deposit_batch(dets, [r.pieces[k][0] for r, k in batch], self.stream)
                ev = torch.cuda.Event()
                ev.record(self.stream)
                with self._lock:
                    self._inflight.append((ev, batch))
                    self._lock.notify_all()
        except BaseException as e:  # surfaced to callers by _raise_if_failed
            with self._lock:
                self._error = e
                self._lock.notify_all()

    def _completion_loop(self) -> None:
        try:
            while True:
                with self._lock:
                    while self._running and not self._inflight:
                        self._lock.wait(timeout=0.5)
                    if not self._inflight:
                        return
                    ev, batch = self._inflight[0]
                ev.synchronize()
                t = self.clock()
                with self._lock:
                    self._inflight.popleft()
                    for r, k in batch:
                        r.pieces[k] = (None, r.pieces[k][1])  # the part's memory may go
                        if self.sched.piece_done(r):
                            r.completion = t
                            r.payload = None
                            r.ready = None
                            self._outstanding[r.det_id] -= 1
                    self._lock.notify_all()
        except BaseException as e:
            with self._lock:
                self._error = e
                self._lock.notify_all()


def detector_bytes(spec) -> int:
    """Device bytes of a detector's state: six accumulator words per
    (cell, slot) and the cell positions with their index map."""
    return int(spec.n_cells) * int(spec.n_t) * 48 + int(spec.n_cells) * 32


# The library's deposit plan, for bounds that hold in every workgroup shape
# (radio_tuning.shape): the smallest tile (cells) and run (segments) of the
# shapes, runs per particle order, and the largest state record (double).
def _shape_minima():
    import paper_2302_14812_amd as radio
    return (min(c for c, _, _ in radio.SHAPES.values()),
            min(r for _, _, r in radio.SHAPES.values()))


(_TILE_CELLS, _RUN_L), _RUNS_PER_ORDER, _REC_BYTES = _shape_minima(), 2, 80


def workspace_bytes(spec, piece_work: float) -> int:
    """Upper bound of the workspaces a detector's own deposits grow (state records,
    one particle order, ring choices).  In a batch a part runs in the batch's
    workspaces unless its particle orders exceed the library's order budget;
    it then runs in time slices of at most two runs on the detector's own
    workspaces, which needs more than two runs (2 L + 1 states for runs of L
    segments) and so at most piece_work / ((2 L + 1) n_cells) particles.
    Taken with the smallest tile and run of any shape, this bounds each shape's
    orders (tiles x particles) and records (particles x states)."""
    n_c = int(spec.n_cells)
    tiles = -(-n_c // _TILE_CELLS)
    states = _RUNS_PER_ORDER * _RUN_L + 1
    n_p = int(math.ceil(piece_work / (float(states) * n_c)))
    return tiles * n_p * 4 + n_p * states * _REC_BYTES + tiles


def resident_bytes(spec, piece_work: float) -> int:
    """Device bytes admission counts for a resident detector: its state and the
    workspaces its deposits may grow."""
    return detector_bytes(spec) + workspace_bytes(spec, piece_work)


def arena_bytes(max_batch_work: float, max_batch_segments: float) -> int:
    """Upper bound of one batch workspace of the library for batches of up to W =
    max_batch_work interactions and S = max_batch_segments particle segments.
    A pair of n_p particles, n_s segments and n_c cells holds at most n_s
    particle orders (one per two runs) of ceil(n_c/C) n_p entries of 4 bytes
    for tiles of C cells, <= 4 W/C + 4 S over the batch; state records of at
    most 80 bytes for n_p (n_s + 1) <= 2 n_p n_s states, <= 160 S; ring choices
    of ceil(n_c/C) bytes, <= W/C + one per pair; and its job and work items.
    C is the smallest tile of any workgroup shape.  A quarter on top covers the
    last two, plus 64 MiB."""
    W, S = float(max_batch_work), float(max_batch_segments)
    orders = 4.0 * W / _TILE_CELLS + 4.0 * S
    records = 2.0 * _REC_BYTES * S
    choices = W / _TILE_CELLS
    return int(math.ceil(1.25 * (orders + records + choices))) + (64 << 20)


def summarize(requests: Sequence[Request], skip: int = 0, sched: Optional[Scheduler] = None
              ) -> dict:
    """p50/p99 chunk latency and throughput over completed requests (after the first `skip`)."""
    done = sorted((r for r in requests if r.completion is not None), key=lambda r: r.arrival)
    done = done[skip:]
    if not done:
        return {"chunks": 0}
    lat = np.array([r.latency for r in done])
    t0 = min(r.arrival for r in done)
    t1 = max(r.completion for r in done)
    work = sum(r.work for r in done)
    out = {"chunks": len(done), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
           "mean_ms": float(lat.mean() * 1e3), "interactions": int(work),
           "interactions_per_s": work / (t1 - t0) if t1 > t0 else float("nan"),
           "batches": len({r.batch for r in done})}
    if sched is not None:
        out["batches"] = sched.n_batches
        out["peak_resident"] = sched.peak_resident
        out["peak_bytes"] = sched.peak_used
    return out


def simulate(sched: Scheduler, requests: Sequence[Request],
             service_time: Callable[[List[float]], float], max_inflight: int = 2,
             piece_work: Optional[float] = None) -> List[Request]:
    """Run the service's policy against a model of the device, on a virtual clock.

    requests carry their arrival times (and sizes); service_time(part works)
    gives the device time of a batch.  The policy is the server's: requests
    are cut into parts of at most piece_work interactions; whenever fewer than
    max_inflight batches are on the device and a pending request can run,
    admit what fits and launch the next batch; batches run one after another
    in launch order.  Returns the requests with launch and completion times
    filled in.  Detectors are never finished here, so requests of detectors
    that never fit stay pending.
    """
    arrivals = sorted(requests, key=lambda r: r.arrival)
    for r in arrivals:
        if piece_work is not None and r.pieces is None:
            n_c = sched.cells[r.det_id]
            limit = min(piece_work, sched.max_batch_segments / 2 * n_c)
            r.pieces = [(None, (p1 - p0) * (b - a) * n_c)
                        for a, b, p0, p1 in plan_pieces(r.n_particles, r.n_steps, n_c, limit)]
    i = 0
    now = 0.0
    device_free = 0.0
    inflight: List[float] = []          # completion times
    while True:
        while i < len(arrivals) and arrivals[i].arrival <= now:
            sched.add(arrivals[i])
            i += 1
        inflight = [t for t in inflight if t > now]
        if len(inflight) < max_inflight and sched.runnable():
            sched.admit()
            batch = sched.next_batch()
            if batch:
                start = max(now, device_free)
                end = start + float(service_time([r.pieces[k][1] for r, k in batch]))
                device_free = end
                inflight.append(end)
                for r, k in batch:
                    if k == 0:
                        r.launched = now
                    if sched.piece_done(r):
                        r.completion = end
                continue
        nxt = [t for t in inflight if t > now]
        if i < len(arrivals):
            nxt.append(arrivals[i].arrival)
        if not nxt:
            break
        now = min(nxt)
    return list(requests)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival offsets (seconds) of a Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def replay(server: DepositServer, items: Sequence[Tuple[int, object]], offsets: Sequence[float],
           clock: Callable[[], float] = time.perf_counter,
           progress: Optional[Callable[[int], None]] = None) -> List[Request]:
    """Submit items[k] = (detector, device chunk) at offsets[k] seconds after the start;
    progress(k), if given, is called after each submission."""
    start = clock()
    reqs = []
    for k, ((det_id, chunk), off) in enumerate(zip(items, offsets)):
        wait = start + float(off) - clock()
        if wait > 0:
            time.sleep(wait)
        reqs.append(server.submit(det_id, chunk))
        if progress is not None:
            progress(k)
    return reqs
