"""Ragged batches of mixed solves with several FP32 V-cycles per FP64 defect
correction (lap_opts.inner in lap_solve_batch): every grid of the merged
launches ends where it ends solved alone (bitwise, same step count, same
test quantities), the one-cycle choice of each step taken per grid on the
device.  Grids solved alone are checked against the oracle's mixed solve in
test_gpu_mixed_inner.py; here the batch is also checked against the oracle's
step count and residual directly."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, maxabs
from oracle import grid as ogrid, solve as osolve

pytestmark = pytest.mark.gpu


def _grids(torch, ctx, probs):
    return [ctx.grid(to_dev(torch, q.psi0), None if q.f is None else to_dev(torch, q.f), q.dx, q.dy) for q in probs]


def _batch_vs_alone(torch, lap, probs, fuse, **kw):
    ctx = lap.Context(arena_bytes=1 << 30)
    ctx.set_fusion(fuse)
    gs = _grids(torch, ctx, probs)
    infos = ctx.solve_batch(gs, **kw)
    mix = [g.read().cpu().numpy() for g in gs]
    for q, g, info, u in zip(probs, gs, infos, mix):
        g.write(to_dev(torch, q.psi0))
        alone = g.solve(**kw)
        assert info["status"] == 0 and info["iterations"] == alone["iterations"], (q.m, q.n, info, alone)
        assert info["rel_res_l2"] == alone["rel_res_l2"], (q.m, q.n)
        assert np.array_equal(u, g.read().cpu().numpy()), (q.m, q.n)
    ctx.close()
    return infos, mix


@pytest.mark.parametrize("inner", [2, 3, 4])
@pytest.mark.parametrize("fuse", [True, False])
def test_batch_inner_cycles_vs_alone_bitwise(inner, fuse):
    """Ten anisotropic grids of 33..257 points a side with sources (some
    whose whole FP32 cycle is one LDS-resident subtree)."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=10, lo=33, hi=257, seed=11, bumps=True)
    say("batch inner", inner, fuse, [(q.m, q.n) for q in probs])
    _batch_vs_alone(torch, lap, probs, fuse, method="mg", precision="mixed", inner=inner, tol=1e-10, max_iter=60)


def test_batch_inner_cycles_vs_oracle():
    """Each grid of a mixed batch with three FP32 cycles per correction takes
    the oracle's step count and lands within 1e-9 of its solution, with a
    recomputed relative residual below 1e-10."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=6, lo=33, hi=129, seed=12, bumps=True)
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = _grids(torch, ctx, probs)
    say("batch inner vs oracle", [(q.m, q.n) for q in probs])
    infos = ctx.solve_batch(gs, method="mg", precision="mixed", inner=3, tol=1e-10, max_iter=60)
    for q, g, info in zip(probs, gs, infos):
        f = np.zeros((q.m, q.n)) if q.f is None else q.f
        ref, k, _ = osolve.mixed_solve(q.psi0, f, q.dx, q.dy, tol=1e-10, inner=3)
        u = g.read().cpu().numpy()
        assert info["status"] == 0 and info["iterations"] == k, (q.m, q.n, info["iterations"], k)
        assert maxabs(u, ref) <= 1e-9 * max(1.0, float(np.max(np.abs(ref))))
        r0 = ogrid.norm2(ogrid.residual(q.psi0, f, q.dx, q.dy))
        assert ogrid.norm2(ogrid.residual(u, f, q.dx, q.dy)) / r0 < 1e-10 * 1.0001
    ctx.close()


def test_batch_of_one_grid_inner_cycles():
    """A batch of one grid keeps the tiling table's shapes (four columns per
    lane on the four-sweep pass where the table gives them)."""
    torch, lap = need_gpu()
    p = W.square_problem(513, seed=2, bumps=True, bump_seed=3)
    say("batch of one, inner 4")
    _batch_vs_alone(torch, lap, [p], True, method="mg", precision="mixed", inner=4, tol=1e-10, max_iter=60)


def test_batch_inner_cycles_with_relaxed_smoother():
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=8, lo=33, hi=257, seed=13, bumps=True)
    say("batch inner omega", [(q.m, q.n) for q in probs])
    _batch_vs_alone(torch, lap, probs, True, method="mg", precision="mixed", inner=3, omega=1.15, tol=1e-10,
                    max_iter=60)


@pytest.mark.parametrize("max_iter", [1, 2, 3])
def test_batch_inner_cycles_stopped_by_max_iter(max_iter):
    """Grids that reach max_iter before the tolerance stop with LAP_ENOTCONV
    (their gates set like a converged grid's, so their later launches exit),
    each exactly where it stops alone with the same limit."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=8, lo=33, hi=257, seed=14, bumps=True)
    say("batch inner max_iter", max_iter)
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = _grids(torch, ctx, probs)
    kw = dict(method="mg", precision="mixed", inner=3, tol=1e-10, max_iter=max_iter)
    infos = ctx.solve_batch(gs, **kw)
    mix = [g.read().cpu().numpy() for g in gs]
    for q, g, info, u in zip(probs, gs, infos, mix):
        g.write(to_dev(torch, q.psi0))
        alone = g.solve(**kw)
        assert info["status"] == alone["status"] and info["iterations"] == alone["iterations"], (q.m, q.n)
        assert info["rel_res_l2"] == alone["rel_res_l2"], (q.m, q.n)
        assert np.array_equal(u, g.read().cpu().numpy()), (q.m, q.n)
    if max_iter < 3:
        assert all(i["status"] != 0 for i in infos)
    ctx.close()
