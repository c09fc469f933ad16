"""Continuous-batching request loop for Poisson / Laplace solves.

Policy (host side) over the library's tick primitive (lap_batch_step):

* requests queue in arrival order;
* at every tick, queued requests are admitted while their multigrid
  hierarchy's HBM footprint (lap_grid_footprint), plus the headroom the
  backend asks for its per-tick tables (tick_reserve), fits the context's
  largest free arena block and the active set is below `max_active`;
  admission copies the request's boundary data and source into a
  device-resident hierarchy;
* a request whose footprint exceeds the whole arena (capacity) can never be
  admitted: it fails at once with status LAP_ENOMEM instead of blocking the
  queue;
* if a tick still runs out of arena (TickOutOfMemory), the most recently
  admitted grid that has not stepped yet (else the most recent one) is
  released and goes back to the head of the queue, and the tick is retried
  with the others; a grid that cannot tick alone fails with LAP_ENOMEM;
* one tick advances every active grid by one outer step (one FP32 V-cycle
  inside FP64 defect correction), all grids' operations of a level merged
  into single launches; grids whose stopping rule holds leave the active set,
  their solution is read back and their hierarchy returned to the arena, so
  the next queued requests can join at the following tick;
* when no request is waiting, a tick runs `burst` outer steps back to back
  before reading the grids' state (a grid that converges inside the burst
  stops on the device), trading admission delay for fewer host round trips;
* a request that finds the device idle and nobody waiting, and is small
  enough (`solo_max_nodes`), is solved alone to its tolerance in one library
  call (single-grid graph replay, no merged plan, one status read per step
  instead of one per tick); requests arriving meanwhile queue for at most
  that solve;
* latency of a request = time its result is readable - its arrival time.

The backend is any object with footprint(m, n) -> bytes, free_bytes(),
admit(request) -> handle, tick(handles, steps) -> (done flags, infos), and
retire(handle) -> result, and optionally solve_alone(handle, request) ->
info, capacity() -> bytes, tick_reserve(active grids) -> bytes and
release(handle) (give the memory back without a result).  `DeviceBackend`
drives liblap; tests drive the policy with a simulated backend on a virtual
clock.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

ENOMEM = -2                         # lap_status LAP_ENOMEM


class TickOutOfMemory(MemoryError):
    """A tick could not allocate its per-tick tables in the arena."""


@dataclass
class Job:
    rid: int
    arrival: float
    m: int
    n: int
    tol: float
    payload: object = None        # backend-specific input (device tensors, seeds, ...)
    admitted: float | None = None
    finished: float | None = None
    iterations: int | None = None
    status: int | None = None
    result: object = None
    handle: object = None
    stepped: bool = False         # has taken part in a batched tick

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


@dataclass
class ServeStats:
    jobs: list = field(default_factory=list)
    ticks: int = 0
    wall: float = 0.0
    max_active: int = 0
    busy_ticks: int = 0
    solo: int = 0                 # requests solved alone (idle device, nobody waiting)

    def summary(self, lup_of=None):
        lat = np.array([j.latency for j in self.jobs if j.latency is not None])
        done = len(lat)
        out = {
            "requests": len(self.jobs),
            "completed": done,
            "solves_per_s": done / self.wall if self.wall > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if done else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if done else None,
            "mean_ms": float(lat.mean() * 1e3) if done else None,
            "ticks": self.ticks,
            "max_active": self.max_active,
            "wall_s": self.wall,
            "failed": sum(1 for j in self.jobs if j.status not in (None, 0)),
            "solo": self.solo,
        }
        if lup_of is not None and self.wall > 0:
            out["GLUP/s"] = sum(lup_of(j) for j in self.jobs if j.finished is not None) / self.wall / 1e9
        return out


class Server:
    """Continuous batching with admission by footprint."""

    def __init__(self, backend, max_active: int = 512, clock=time.perf_counter, burst: int = 1,
                 solo_max_nodes: int = 4097 * 4097):
        self.backend = backend
        self.max_active = max_active
        self.clock = clock
        self.burst = max(1, int(burst))
        self.solo_max_nodes = solo_max_nodes if hasattr(backend, "solve_alone") else 0
        self.queue: list[Job] = []
        self.active: list[Job] = []

    def submit(self, job: Job):
        self.queue.append(job)

    def _fail(self, job, status=ENOMEM):
        job.status = status
        job.finished = self.clock()
        job.handle = None

    def _admit(self, now):
        cap = getattr(self.backend, "capacity", None)
        reserve = getattr(self.backend, "tick_reserve", None)
        while self.queue and len(self.active) < self.max_active:
            job = self.queue[0]
            if job.arrival > now:
                break
            need = self.backend.footprint(job.m, job.n)
            if cap is not None and need + (reserve(1) if reserve else 0) > cap():
                self.queue.pop(0)           # can never fit: fail now rather than block the queue
                self._fail(job)
                continue
            if reserve is not None:
                need += reserve(len(self.active) + 1)
            if need > self.backend.free_bytes():
                break                       # wait for memory to free up (FIFO: no overtaking)
            self.queue.pop(0)
            job.handle = self.backend.admit(job)
            job.admitted = self.clock()
            self.active.append(job)

    def _tick_active(self, steps):
        """backend.tick over the active set; on TickOutOfMemory release the
        most recently admitted grid (preferring one that has not stepped),
        requeue it at the head of the queue and retry with the others."""
        while True:
            try:
                return self.backend.tick([j.handle for j in self.active], steps)
            except TickOutOfMemory:
                if len(self.active) == 1:
                    job = self.active.pop()
                    if hasattr(self.backend, "release"):
                        self.backend.release(job.handle)
                    self._fail(job)
                    return [], []
                fresh = [k for k, j in enumerate(self.active) if not j.stepped]
                k = fresh[-1] if fresh else len(self.active) - 1
                job = self.active.pop(k)
                self.backend.release(job.handle)
                job.handle = None
                job.admitted = None
                job.stepped = False
                self.queue.insert(0, job)

    def tick(self, stats: ServeStats | None = None):
        """Admit what fits, advance every active grid by one outer step (or
        `burst` steps), retire the finished ones; a lone small request on an
        idle device is solved alone instead.  Returns the finished jobs."""
        self._admit(self.clock())
        if not self.active:
            return []
        if len(self.active) == 1 and not self.queue:
            job = self.active[0]
            if not job.stepped and job.m * job.n <= self.solo_max_nodes:
                info = self.backend.solve_alone(job.handle, job)
                self._retire(job, info)
                self.active = []
                if stats is not None:
                    stats.ticks += 1
                    stats.solo += 1
                    stats.max_active = max(stats.max_active, 1)
                return [job]
        steps = 1 if self.queue else self.burst
        done, infos = self._tick_active(steps)
        finished, still = [], []
        for job, d, info in zip(self.active, done, infos):
            job.stepped = True
            if d:
                self._retire(job, info)
                finished.append(job)
            else:
                still.append(job)
        self.active = still
        if stats is not None:
            stats.ticks += 1
            stats.busy_ticks += 1
            stats.max_active = max(stats.max_active, len(self.active) + len(finished))
        return finished

    def _retire(self, job, info):
        job.result = self.backend.retire(job.handle)
        job.finished = self.clock()
        job.iterations = info.get("iterations")
        job.status = info.get("status")
        job.handle = None

    def run(self, jobs: list[Job], t0: float | None = None, idle_sleep: float = 0.0) -> ServeStats:
        """Serve a whole stream: job.arrival is relative to the start."""
        stats = ServeStats(jobs=list(jobs))
        start = self.clock() if t0 is None else t0
        pending = sorted(jobs, key=lambda j: j.arrival)
        for j in pending:
            j.arrival = start + j.arrival
        k = 0
        while k < len(pending) or self.queue or self.active:
            now = self.clock()
            while k < len(pending) and pending[k].arrival <= now:
                self.submit(pending[k])
                k += 1
            if not self.active and self.queue and self.queue[0].arrival <= now:
                # nothing runs, so the arena holds no grid: a queued request
                # that still does not fit cannot be served
                self._admit(now)
                if not self.active and self.queue and self.queue[0].arrival <= self.clock():
                    self._fail(self.queue.pop(0))
                continue
            if not self.active and not self.queue and k < len(pending):
                # idle: wait for the next arrival
                wait = pending[k].arrival - self.clock()
                if wait > 0 and idle_sleep >= 0:
                    self._sleep(wait)
                continue
            self.tick(stats)
        stats.wall = self.clock() - start
        for j in jobs:
            j.arrival -= start
            if j.finished is not None:
                j.finished -= start
        return stats

    def _sleep(self, dt):
        sleeper = getattr(self.backend, "sleep", None)
        if sleeper is not None:
            sleeper(dt)
        else:
            time.sleep(dt)


def serve_sequential(backend_solve, jobs: list[Job], clock=time.perf_counter) -> ServeStats:
    """Baseline: one request at a time in arrival order (FIFO), each solved
    to its tolerance before the next starts."""
    stats = ServeStats(jobs=list(jobs))
    start = clock()
    for job in sorted(jobs, key=lambda j: j.arrival):
        now = clock() - start
        if job.arrival > now:
            time.sleep(job.arrival - now)
        job.admitted = clock() - start
        info = backend_solve(job)
        job.finished = clock() - start
        job.iterations = info.get("iterations")
        job.status = info.get("status")
    stats.wall = clock() - start
    stats.ticks = len(jobs)
    return stats


class DeviceBackend:
    """liblap backend: grids with the mixed-precision hierarchy only, ticks
    through lap_batch_step.  job.payload = (psi0, f, dx, dy) device tensors."""

    def __init__(self, ctx, precision: str = "mixed", keep_results: bool = False, omega: float = 1.0):
        from . import LAP_ALLOC_MIXED, LAP_ALLOC_FP64
        self.ctx = ctx
        self.precision = precision
        self.omega = omega          # relaxation of the multigrid smoother
        self.alloc = LAP_ALLOC_MIXED if precision == "mixed" else LAP_ALLOC_FP64
        self.keep_results = keep_results

    def footprint(self, m, n):
        from . import footprint
        return footprint(m, n, self.alloc)

    def free_bytes(self):
        return self.ctx.usage()[1]

    def capacity(self):
        return int(self.ctx.arena.numel())

    def tick_reserve(self, active):
        """Arena headroom for one tick's merged plan and control tables
        (tile tables and launch items: well under 256 KiB per grid up to
        4097^2) besides the grids' hierarchies."""
        return (8 << 20) + active * (256 << 10)

    def release(self, g):
        g.destroy()

    def admit(self, job):
        psi0, f, dx, dy = job.payload
        g = self.ctx.grid(psi0, f, dx, dy, alloc=self.alloc)
        g.set_tol(job.tol)
        g.set_omega(self.omega)
        return g

    def tick(self, grids, steps=1):
        from . import LapError
        from ._native import LAP_ENOMEM
        try:
            return self.ctx.batch_step(grids, precision=self.precision, steps=steps)
        except LapError as e:
            if e.status == LAP_ENOMEM:
                raise TickOutOfMemory(str(e)) from e
            raise

    def solve_alone(self, g, job):
        return g.solve("mg", precision=self.precision, omega=self.omega, tol=job.tol, max_iter=1000)

    def retire(self, g):
        out = g.read() if self.keep_results else None
        g.destroy()
        return out
