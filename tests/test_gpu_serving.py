"""The serving loop on the device: a Poisson stream of small requests served
with continuous batching; every result meets its tolerance (residual
recomputed by the oracle) and equals the same request solved alone."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev
from oracle import grid as ogrid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("burst,solo", [(1, 0), (3, 0), (3, 2049 * 2049)])
def test_served_results_meet_tolerance_and_match_alone(burst, solo):
    """solo = 0: every request goes through batched ticks; otherwise a lone
    small request on an idle device is solved alone (single-grid path)."""
    torch, lap = need_gpu()
    from paper_2208_02427_amd.serving import Job, Server, DeviceBackend
    reqs = W.poisson_requests(rate=400.0, count=24, seed=11, lo=17, hi=129)
    probs = [W.request_problem(r) for r in reqs]
    say("serve", [(r.m, r.n, r.tol) for r in reqs])
    ctx = lap.Context(arena_bytes=512 << 20)
    jobs = [Job(r.rid, r.arrival, r.m, r.n, r.tol,
                payload=(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)) for r, p in zip(reqs, probs)]
    stats = Server(DeviceBackend(ctx, keep_results=True), max_active=8, burst=burst, solo_max_nodes=solo).run(jobs)
    s = stats.summary()
    say("served", s["solo"], "alone of", len(jobs), "max active", stats.max_active)
    assert s["completed"] == len(jobs) and s["failed"] == 0
    if solo:
        assert s["solo"] > 0
    else:
        assert s["solo"] == 0 and stats.max_active > 1
    used, _ = ctx.usage()
    assert used < (1 << 20)                    # every hierarchy went back to the arena
    ctx2 = lap.Context(arena_bytes=256 << 20)
    for job, p in zip(jobs, probs):
        u = job.result.cpu().numpy()
        r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
        assert ogrid.norm2(ogrid.residual(u, p.f, p.dx, p.dy)) / r0 < job.tol * 1.0001
        g = ctx2.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy, alloc=lap.LAP_ALLOC_MIXED)
        info = g.solve("mg", precision="mixed", tol=job.tol, max_iter=1000)
        assert info["iterations"] == job.iterations
        assert np.array_equal(g.read().cpu().numpy(), u)
        g.destroy()
