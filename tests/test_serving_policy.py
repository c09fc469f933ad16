"""The serving policy on a virtual clock with a simulated backend (CPU only):
admission by footprint, FIFO order, continuous batching (requests join while
others run), retirement, latency accounting, the sequential baseline."""
import numpy as np

import workloads as W
from paper_2208_02427_amd.serving import Job, Server, ServeStats, serve_sequential


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class SimBackend:
    """Each grid needs `cycles` ticks; a tick costs base + per-grid time on
    the virtual clock; memory is a fixed pool."""

    def __init__(self, clock, pool=10_000, tick_base=1e-3, per_grid=1e-4, sync=0.0):
        self.clock = clock
        self.pool = pool
        self.used = 0
        self.tick_base = tick_base
        self.per_grid = per_grid
        self.sync = sync           # host round trip per tick
        self.steps = []
        self.admitted = []
        self.max_used = 0
        self.batches = []

    def footprint(self, m, n):
        return m * n

    def free_bytes(self):
        return self.pool - self.used

    def admit(self, job):
        self.used += self.footprint(job.m, job.n)
        self.max_used = max(self.max_used, self.used)
        self.admitted.append(job.rid)
        return {"job": job, "left": job.payload}

    def tick(self, handles, steps=1):
        self.batches.append(len(handles))
        self.steps.append(steps)
        self.clock.t += self.sync + steps * (self.tick_base + self.per_grid * len(handles))
        done = []
        for h in handles:
            h["left"] -= steps        # a grid that converges inside the burst stops there
            done.append(h["left"] <= 0)
        return done, [{"iterations": h["job"].payload, "status": 0} for h in handles]

    def retire(self, h):
        self.used -= self.footprint(h["job"].m, h["job"].n)
        return "result"

    def sleep(self, dt):
        self.clock.t += dt


class SoloBackend(SimBackend):
    """SimBackend that can also solve one grid alone: its steps back to back
    with no per-tick round trip."""

    def __init__(self, *a, **kw):
        super().__init__(*a, **kw)
        self.solo = []

    def solve_alone(self, h, job):
        self.solo.append(job.rid)
        self.clock.t += job.payload * (self.tick_base + self.per_grid)
        h["left"] = 0
        return {"iterations": job.payload, "status": 0}


def jobs_from_stream(rate, count, seed=5, lo=17, hi=257):
    reqs = W.poisson_requests(rate, count, seed=seed, lo=lo, hi=hi)
    return [Job(r.rid, r.arrival, r.m, r.n, r.tol, payload=7 if r.tol < 1e-9 else 5) for r in reqs]


def test_all_requests_complete_with_fifo_admission():
    clk = Clock()
    be = SimBackend(clk, pool=200_000)
    jobs = jobs_from_stream(rate=2000.0, count=300)
    stats = Server(be, max_active=64, clock=clk).run(jobs)
    s = stats.summary()
    assert s["completed"] == 300 and s["failed"] == 0
    assert be.admitted == sorted(be.admitted)            # FIFO admission
    assert be.max_used <= be.pool                         # never over the memory pool
    assert max(be.batches) <= 64                          # never above max_active
    assert all(j.latency >= 0 for j in jobs)
    # continuous batching: grids are advanced together (batches > 1)
    assert max(be.batches) > 1
    # each job needed exactly its cycle count of ticks after admission
    assert all(j.iterations == j.payload for j in jobs)


def test_memory_pressure_defers_admission():
    clk = Clock()
    be = SimBackend(clk, pool=70_000)
    jobs = [Job(k, 0.0, 257, 257, 1e-10, payload=3) for k in range(4)]   # 66k each: one at a time
    stats = Server(be, clock=clk).run(jobs)
    assert stats.summary()["completed"] == 4
    assert max(be.batches) == 1 and be.max_used <= 70_000


def test_requests_join_while_others_run():
    clk = Clock()
    be = SimBackend(clk, pool=10**9, tick_base=1e-3, per_grid=0.0)
    jobs = [Job(0, 0.0, 33, 33, 1e-10, payload=10), Job(1, 0.0035, 33, 33, 1e-10, payload=2)]
    Server(be, clock=clk).run(jobs)
    # job 1 arrives during job 0's 4th tick, joins, and finishes first
    assert jobs[1].finished < jobs[0].finished
    assert 2 in be.batches


def test_latency_grows_past_saturation():
    res = {}
    for rate in (100.0, 100000.0):
        clk = Clock()
        be = SimBackend(clk, pool=10**9, tick_base=1e-3, per_grid=2e-4)
        jobs = jobs_from_stream(rate=rate, count=200)
        res[rate] = Server(be, max_active=16, clock=clk).run(jobs).summary()
    assert res[100000.0]["p99_ms"] > res[100.0]["p99_ms"]
    assert res[100.0]["p50_ms"] < 20


def test_sequential_baseline():
    jobs = [Job(k, 0.0, 17, 17, 1e-8) for k in range(5)]
    stats = serve_sequential(lambda j: {"iterations": 3, "status": 0}, jobs)
    assert stats.summary()["completed"] == 5
    assert [j.finished for j in jobs] == sorted(j.finished for j in jobs)


def test_summary_percentiles():
    st = ServeStats(jobs=[Job(k, 0.0, 3, 3, 1.0, finished=float(k + 1)) for k in range(100)], wall=100.0)
    s = st.summary()
    assert s["p50_ms"] == np.percentile(np.arange(1, 101), 50) * 1e3
    assert s["solves_per_s"] == 1.0


def test_burst_ticks_cut_round_trips_at_low_load():
    """With nothing waiting, a tick runs `burst` steps before the host reads
    back: at low load latency drops by the saved round trips; every job still
    needs exactly its own number of steps."""
    res = {}
    for burst in (1, 4):
        clk = Clock()
        be = SimBackend(clk, pool=10**9, tick_base=2e-4, per_grid=1e-5, sync=3e-4)
        jobs = jobs_from_stream(rate=50.0, count=100)
        stats = Server(be, clock=clk, burst=burst).run(jobs)
        res[burst] = (stats.summary(), be.steps)
        assert all(j.iterations == j.payload for j in jobs)
    assert max(res[1][1]) == 1 and max(res[4][1]) == 4
    assert res[4][0]["p50_ms"] < res[1][0]["p50_ms"]


def test_burst_falls_back_to_single_steps_when_requests_wait():
    clk = Clock()
    be = SimBackend(clk, pool=70_000, tick_base=1e-3, per_grid=0.0)
    jobs = [Job(k, 0.0, 257, 257, 1e-10, payload=5) for k in range(3)]   # one fits at a time
    Server(be, clock=clk, burst=4).run(jobs)
    # while others queue, ticks are single steps; the last job runs alone with bursts
    assert be.steps[0] == 1 and be.steps[-1] == 4


def test_lone_small_request_is_solved_alone():
    """A request that finds the device idle and nobody waiting is solved alone
    (no per-tick round trips); under load the same requests are batched, and
    requests above the size limit never go alone."""
    res = {}
    for rate in (20.0, 20000.0):
        clk = Clock()
        be = SoloBackend(clk, pool=10**9, tick_base=2e-4, per_grid=1e-5, sync=3e-4)
        jobs = jobs_from_stream(rate=rate, count=100)
        stats = Server(be, clock=clk).run(jobs)
        s = stats.summary()
        assert s["completed"] == 100 and s["solo"] == len(be.solo)
        assert all(j.iterations == j.payload for j in jobs)
        res[rate] = (s, max(be.batches) if be.batches else 0)
    assert res[20.0][0]["solo"] > 80               # nearly every request arrives to an idle device
    assert res[20000.0][0]["solo"] < 10 and res[20000.0][1] > 1
    clk = Clock()
    be = SoloBackend(clk, pool=10**9)
    jobs = [Job(0, 0.0, 129, 129, 1e-10, payload=3), Job(1, 1.0, 33, 33, 1e-10, payload=3)]
    Server(be, clock=clk, solo_max_nodes=65 * 65).run(jobs)
    assert be.solo == [1] and be.batches == [1, 1, 1]    # 129^2 above the limit: three batched ticks


def test_solo_latency_beats_ticks_at_low_load():
    res = {}
    for solo in (0, 2049 * 2049):
        clk = Clock()
        be = SoloBackend(clk, pool=10**9, tick_base=2e-4, per_grid=1e-5, sync=3e-4)
        jobs = jobs_from_stream(rate=20.0, count=100)
        res[solo] = Server(be, clock=clk, solo_max_nodes=solo).run(jobs).summary()
    assert res[0]["solo"] == 0
    assert res[2049 * 2049]["p50_ms"] < res[0]["p50_ms"]


class TightBackend(SimBackend):
    """SimBackend with an arena capacity, a per-tick table reserve and a
    tick that fails (TickOutOfMemory) while the active set exceeds
    `tick_limit` grids; release() gives a grid's memory back."""

    def __init__(self, *a, tick_limit=None, **kw):
        super().__init__(*a, **kw)
        self.tick_limit = tick_limit
        self.released = []
        self.oom_ticks = 0

    def capacity(self):
        return self.pool

    def tick_reserve(self, active):
        return 10 * active

    def tick(self, handles, steps=1):
        from paper_2208_02427_amd.serving import TickOutOfMemory
        if self.tick_limit is not None and len(handles) > self.tick_limit:
            self.oom_ticks += 1
            raise TickOutOfMemory("plan does not fit")
        return super().tick(handles, steps)

    def release(self, h):
        self.released.append(h["job"].rid)
        self.used -= self.footprint(h["job"].m, h["job"].n)


def test_request_that_never_fits_fails_without_blocking_the_queue():
    clock = Clock()
    be = TightBackend(clock, pool=5000)
    jobs = [Job(0, 0.0, 10, 10, 1e-8, payload=3),
            Job(1, 0.001, 100, 100, 1e-8, payload=3),       # 10000 > the whole pool
            Job(2, 0.002, 20, 20, 1e-8, payload=2)]
    stats = Server(be, clock=clock).run(jobs)
    s = stats.summary()
    assert s["completed"] == 3 and s["failed"] == 1
    assert jobs[1].status == -2 and jobs[1].result is None
    assert jobs[0].status == 0 and jobs[2].status == 0 and jobs[2].result == "result"
    assert 1 not in be.admitted and be.used == 0


def test_admission_keeps_headroom_for_tick_tables():
    """Two grids of 2500 fit a 5000 pool by footprint alone, but not with the
    reserve of 10 per active grid: the second waits for the first."""
    clock = Clock()
    be = TightBackend(clock, pool=5000)
    jobs = [Job(0, 0.0, 50, 50, 1e-8, payload=4), Job(1, 0.0, 50, 50, 1e-8, payload=4)]
    Server(be, clock=clock).run(jobs)
    assert max(be.batches) == 1 and be.max_used <= 5000 - 10
    assert all(j.status == 0 for j in jobs)


def test_tick_out_of_memory_requeues_the_newest_grid():
    """Ticks of more than two grids fail: the server releases the newest
    grid that has not stepped, requeues it, and every request completes."""
    clock = Clock()
    be = TightBackend(clock, pool=100_000, tick_limit=2)
    jobs = [Job(k, 0.0, 10, 10, 1e-8, payload=3 + k) for k in range(5)]
    stats = Server(be, clock=clock).run(jobs)
    s = stats.summary()
    assert s["completed"] == 5 and s["failed"] == 0
    assert be.oom_ticks > 0 and be.released
    assert max(be.batches) <= 2
    assert [j.iterations for j in jobs] == [3, 4, 5, 6, 7]


def test_grid_that_cannot_tick_alone_fails():
    clock = Clock()
    be = TightBackend(clock, pool=100_000, tick_limit=0)
    jobs = [Job(0, 0.0, 10, 10, 1e-8, payload=3)]
    stats = Server(be, clock=clock).run(jobs)
    assert stats.summary()["failed"] == 1 and jobs[0].status == -2
    assert be.used == 0
