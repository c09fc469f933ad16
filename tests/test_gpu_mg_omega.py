"""Multigrid with an over-relaxed red-black smoother (omega_s = 1.15, the
smoother's `omega` of LAP_MG) against the oracle: k FP64 V(2,2) cycles, mixed
steps of one and several FP32 cycles, fused and unfused, a converged solve
with the oracle's cycle count, and a ragged batch against each grid alone."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, rand_problem, maxabs
from oracle import multigrid as omg, grid as ogrid, solve as osolve

pytestmark = pytest.mark.gpu

W_S = 1.15


@pytest.mark.parametrize("m,n", [(257, 193), (129, 65), (65, 129)])
@pytest.mark.parametrize("fuse", [True, False])
def test_fp64_cycles_vs_oracle(m, n, fuse):
    torch, lap = need_gpu()
    psi, f, dx, dy = rand_problem(m, n, 5 * m + n, dx=1.0 / (m - 1), dy=1.2 / (n - 1), source=True)
    ctx = lap.Context(arena_bytes=256 << 20)
    ctx.set_fusion(fuse)
    g = ctx.grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
    lv = omg.hierarchy(m, n, dx, dy)
    ref = psi.copy()
    for k in (1, 2, 3):
        say("mg omega cycles", m, n, fuse, k)
        g.write(to_dev(torch, psi))
        info = g.solve("mg", omega=W_S, tol=0.0, max_iter=k)
        assert info["iterations"] == k
        r = ogrid.residual(ref, f, dx, dy)
        e = np.zeros_like(r)
        omg.vcycle(lv, 0, e, r, 2, 2, W_S)
        ref += e
        assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10 * max(1.0, float(np.max(np.abs(ref))))
    g.destroy()
    ctx.close()


@pytest.mark.parametrize("inner", [1, 2, 4])
@pytest.mark.parametrize("fuse", [True, False])
def test_mixed_steps_vs_oracle(inner, fuse):
    torch, lap = need_gpu()
    m, n = 257, 193
    psi, f, dx, dy = rand_problem(m, n, 77 + inner, dx=1.0 / (m - 1), dy=1.2 / (n - 1), source=True)
    ctx = lap.Context(arena_bytes=256 << 20)
    ctx.set_fusion(fuse)
    g = ctx.grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
    lv = omg.hierarchy(m, n, dx, dy)
    ref, ref64 = psi.copy(), psi.copy()
    for k in (1, 2, 3):
        say("mg omega mixed", inner, fuse, k)
        g.write(to_dev(torch, psi))
        info = g.solve("mg", precision="mixed", inner=inner, omega=W_S, tol=0.0, max_iter=k)
        assert info["iterations"] == k
        omg.mixed_step(ref, f, lv, 2, 2, W_S, inner=inner)
        r = ogrid.residual(ref64, f, dx, dy)
        e = np.zeros_like(r)
        for _ in range(inner):
            omg.vcycle(lv, 0, e, r, 2, 2, W_S)
        ref64 += e
        got = maxabs(g.read().cpu().numpy(), ref)
        assert got <= 3.0 * maxabs(ref, ref64) + 1e-12 * float(np.max(np.abs(ref))), (k, got)
    g.destroy()
    ctx.close()


@pytest.mark.parametrize("precision,inner", [("fp64", 1), ("mixed", 1), ("mixed", 4)])
def test_solve_to_tol_vs_oracle(precision, inner):
    """Solves to 1e-10 take the oracle's cycle (step) count and land within
    1e-9 of its field; with omega_s = 1 the FP64 solve takes more cycles."""
    torch, lap = need_gpu()
    p = W.square_problem(513, seed=2, bumps=True, bump_seed=3)
    ctx = lap.Context(arena_bytes=512 << 20)
    g = ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
    say("mg omega solve", precision, inner)
    info = g.solve("mg", precision=precision, inner=inner, omega=W_S, tol=1e-10, max_iter=60)
    u = g.read().cpu().numpy()
    if precision == "fp64":
        ref, k, _ = osolve.mg_solve(p.psi0, p.f, p.dx, p.dy, tol=1e-10, omega_s=W_S)
        _, k1, _ = osolve.mg_solve(p.psi0, p.f, p.dx, p.dy, tol=1e-10)
        assert k < k1
    else:
        ref, k, _ = osolve.mixed_solve(p.psi0, p.f, p.dx, p.dy, tol=1e-10, omega_s=W_S, inner=inner)
    assert info["status"] == 0 and info["iterations"] == k, (info["iterations"], k)
    assert maxabs(u, ref) <= 1e-9 * max(1.0, float(np.max(np.abs(ref))))
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    assert ogrid.norm2(ogrid.residual(u, p.f, p.dx, p.dy)) / r0 < 1e-10 * 1.0001
    g.destroy()
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_vs_alone_bitwise(precision):
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=10, lo=33, hi=257, seed=4, bumps=True)
    kw = dict(method="mg", precision=precision, omega=W_S, tol=1e-10, max_iter=60)
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = [ctx.grid(to_dev(torch, q.psi0), None if q.f is None else to_dev(torch, q.f), q.dx, q.dy) for q in probs]
    say("mg omega batch", precision)
    infos = ctx.solve_batch(gs, **kw)
    mix = [g.read().cpu().numpy() for g in gs]
    for q, g, info, u in zip(probs, gs, infos, mix):
        g.write(to_dev(torch, q.psi0))
        alone = g.solve(**kw)
        assert info["status"] == 0 and info["iterations"] == alone["iterations"]
        assert np.array_equal(u, g.read().cpu().numpy())
    ctx.close()


def test_batch_step_with_grid_omega():
    """Continuous batching with lap_grid_set_omega: ticks of a mixed batch
    whose grids carry omega_s = 1.15 (two of them 1) end each grid where it
    ends solved alone with its own omega, bitwise; omega outside (0, 2) is
    refused."""
    torch, lap = need_gpu()
    from paper_2208_02427_amd import LapError
    probs = W.ragged_batch(count=5, lo=33, hi=129, seed=8, bumps=True)
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = [ctx.grid(to_dev(torch, q.psi0), None if q.f is None else to_dev(torch, q.f), q.dx, q.dy) for q in probs]
    omegas = [W_S, 1.0, W_S, W_S, 1.0]
    for g, w in zip(gs, omegas):
        g.set_omega(w)
    for bad in (0.0, 2.0, -1.0):
        with pytest.raises(LapError):
            gs[0].set_omega(bad)
    say("batch step omega", [(q.m, q.n) for q in probs])
    active, finished, tick = list(range(len(gs))), {}, 0
    while active:
        done, infos = ctx.batch_step([gs[k] for k in active], precision="mixed", steps=2)
        still = []
        for k, d, info in zip(active, done, infos):
            if d:
                finished[k] = (info, gs[k].read().cpu().numpy())
            else:
                still.append(k)
        active = still
        tick += 1
        assert tick < 200
    for k, (q, g, w) in enumerate(zip(probs, gs, omegas)):
        g.write(to_dev(torch, q.psi0))
        alone = g.solve("mg", precision="mixed", omega=w, tol=1e-10, max_iter=200)
        assert finished[k][0]["status"] == 0 and finished[k][0]["iterations"] == alone["iterations"]
        assert np.array_equal(finished[k][1], g.read().cpu().numpy())
    ctx.close()
