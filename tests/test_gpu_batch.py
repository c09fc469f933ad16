"""Batched and served solves: a grid solved inside a ragged batch (or
advanced by continuous-batching ticks next to other grids) gives the same
result, bit for bit, as the same grid solved alone; every grid meets its
tolerance, checked by the oracle's residual of the returned field."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, maxabs
from oracle import grid as ogrid

pytestmark = pytest.mark.gpu


def _grids(ctx, probs, torch):
    return [ctx.grid(to_dev(torch, p.psi0), None if p.f is None else to_dev(torch, p.f), p.dx, p.dy)
            for p in probs]


def _rel_res(p, u):
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    return ogrid.norm2(ogrid.residual(u, p.f, p.dx, p.dy)) / r0


@pytest.mark.parametrize("method,precision", [("mg", "fp64"), ("mg", "mixed"), ("adi", "fp64")])
def test_batch_alone_vs_mix_bitwise(method, precision):
    torch, lap = need_gpu()
    if method == "mg":
        probs = W.ragged_batch(count=12, lo=33, hi=257, seed=4)
        kw = dict(method=method, precision=precision, tol=1e-10, max_iter=60, omega=1.0)
    else:
        # line relaxation converges at 1 - O(h^2): small grids, over-relaxed
        probs = W.ragged_batch(count=12, lo=17, hi=49, seed=4)
        kw = dict(method=method, precision=precision, tol=1e-10, max_iter=20000, omega=1.5, check_every=10)
    say("batch", method, precision, [(p.m, p.n) for p in probs])
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = _grids(ctx, probs, torch)
    infos = ctx.solve_batch(gs, **kw)
    mix = [g.read().cpu().numpy() for g in gs]
    for p, g, info, u in zip(probs, gs, infos, mix):
        assert info["status"] == 0, info
        assert _rel_res(p, u) < 1e-10 * 1.0001
    # alone: the same grids one at a time on a fresh context
    ctx2 = lap.Context(arena_bytes=1 << 30)
    for p, u, info in zip(probs, mix, infos):
        g = ctx2.grid(to_dev(torch, p.psi0), None, p.dx, p.dy)
        alone = g.solve(**kw)
        assert alone["iterations"] == info["iterations"]
        assert np.array_equal(g.read().cpu().numpy(), u)
        g.destroy()


@pytest.mark.parametrize("steps", [1, 3])
def test_batch_step_ticks_match_alone(steps):
    """Continuous batching: grids join at different ticks and leave when done
    (ticks of `steps` outer steps: a grid converging inside a tick stops
    there); each result equals the grid solved alone."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=6, lo=33, hi=129, seed=7, bumps=True)
    say("ticks", [(p.m, p.n) for p in probs])
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = _grids(ctx, probs, torch)
    tols = [1e-8, 1e-10, 1e-8, 1e-10, 1e-10, 1e-8]
    for g, t in zip(gs, tols):
        g.set_tol(t)
    active = []
    finished = {}
    pending = list(range(len(gs)))
    tick = 0
    while pending or active:
        if pending and tick % 2 == 0:        # a new request joins every other tick
            active.append(pending.pop(0))
        done, infos = ctx.batch_step([gs[k] for k in active], precision="mixed", steps=steps)
        still = []
        for k, d, info in zip(active, done, infos):
            if d:
                finished[k] = (info, gs[k].read().cpu().numpy())
            else:
                still.append(k)
        active = still
        tick += 1
        assert tick < 500
    ctx2 = lap.Context(arena_bytes=1 << 30)
    for k, p in enumerate(probs):
        info, u = finished[k]
        assert info["status"] == 0
        assert _rel_res(p, u) < tols[k]
        g = ctx2.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
        alone = g.solve("mg", precision="mixed", tol=tols[k], max_iter=1000)
        assert alone["iterations"] == info["iterations"]
        assert np.array_equal(g.read().cpu().numpy(), u), k
        g.destroy()


def test_batch_timing_counts_only_full_work_launches():
    """Kernel statistics of a batched solve leave out the launches of the
    round whose stopping tests ended the last grids (they exit at once),
    apart from that round's test itself: check blocks of 3 ADI iterations,
    6 iterations -> 3 tests, 2 row and 2 column launches per iteration
    (grids of 81..129 points a side take one merged launch per line half)."""
    torch, lap = need_gpu()
    from paper_2208_02427_amd._native import KC_ADI_ROWS, KC_ADI_COLS, KC_RESIDUAL
    probs = W.ragged_batch(count=6, lo=81, hi=129, seed=5)
    say("batch timing", [(p.m, p.n) for p in probs])
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = _grids(ctx, probs, torch)
    ctx.set_timing(1)
    nit = 6
    infos = ctx.solve_batch(gs, method="adi", omega=1.0, tol=0.0, max_iter=nit, check_every=3)
    assert all(i["iterations"] == nit for i in infos)
    assert ctx.kernel_stats(KC_ADI_ROWS)["launches"] == 2 * nit
    assert ctx.kernel_stats(KC_ADI_COLS)["launches"] == 2 * nit
    assert ctx.kernel_stats(KC_RESIDUAL)["launches"] == nit // 3 + 1
    ctx.close()
