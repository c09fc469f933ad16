"""Multigrid with zebra line smoothing (LAP_SMOOTH_ZEBRA) against the oracle.

One smoothing step is one zebra ADI iteration (odd rows, even rows, odd
columns, even columns; each line solved exactly, relaxation after the solve)
of the SLOR / ADI sections, used inside the V-cycle of the multigrid
section; the oracle is oracle.multigrid.vcycle(smoother='zebra').  Grids are
anisotropic (dx != dy), with and without a source, of several depths.
FP64 cycles agree with the oracle to 1e-10 max-abs; mixed steps (FP32 line
solves by the segmented solver against the oracle's float32 Thomas
recurrences) to 2e-6 of the field's scale; batched runs equal the grid
alone bit for bit."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, maxabs
from oracle import multigrid as omg, grid as ogrid, solve as osolve

pytestmark = pytest.mark.gpu

CASES = [(65, 33, 2.0, True), (49, 97, 0.5, True), (129, 129, 1.5, False), (33, 17, 1.0, True),
         (97, 161, 0.7, True), (17, 9, 1.3, False)]


def _problem(m, n, beta, src, seed):
    rng = np.random.default_rng(seed)
    dy = 1.0 / (n - 1)
    dx = beta * dy
    psi = W.random_boundary(m, n, rng)
    f = W.gaussian_bumps(m, n, dx, dy, rng) if src else None
    return psi, f, dx, dy


_CTX = {}


def _ctx(torch, lap):
    if "c" not in _CTX:
        _CTX["c"] = lap.Context(arena_bytes=1 << 30)
    return _CTX["c"]


@pytest.mark.parametrize("m,n,beta,src", CASES)
@pytest.mark.parametrize("k", [1, 3])
def test_zebra_fp64_cycles_vs_oracle(m, n, beta, src, k):
    torch, lap = need_gpu()
    say("zebra fp64 cycles", m, n, beta, src, k)
    psi, f, dx, dy = _problem(m, n, beta, src, m * n + k)
    g = _ctx(torch, lap).grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)
    info = g.solve("mg", smoother="zebra", nu1=1, nu2=1, tol=0.0, max_iter=k)
    assert info["iterations"] == k
    lv = omg.hierarchy(m, n, dx, dy)
    ref = psi.copy()
    for _ in range(k):
        omg.vcycle(lv, 0, ref, f, 1, 1, smoother="zebra")
    assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10
    g.destroy()


@pytest.mark.parametrize("m,n,beta,src", CASES[:4])
def test_zebra_mixed_steps_vs_oracle(m, n, beta, src):
    torch, lap = need_gpu()
    psi, f, dx, dy = _problem(m, n, beta, src, 7 * m + n)
    g = _ctx(torch, lap).grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)
    lv = omg.hierarchy(m, n, dx, dy)
    ref = psi.copy()
    for k in (1, 2, 3):
        say("zebra mixed steps", m, n, beta, k)
        g.write(to_dev(torch, psi))
        info = g.solve("mg", precision="mixed", smoother="zebra", nu1=1, nu2=1, tol=0.0, max_iter=k)
        assert info["iterations"] == k
        omg.mixed_step(ref, f, lv, 1, 1, smoother="zebra")
        scale = float(np.max(np.abs(ref)))
        assert maxabs(g.read().cpu().numpy(), ref) <= 2e-6 * scale
    g.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zebra_full_solve_matches_oracle(precision):
    """Solved to 1e-10: the oracle's cycle count (within one), its residual
    recomputed from the GPU result below tol, and the oracle's solution to
    1e-10 of the field's scale; the second solve replays the graph and gives
    the same bits."""
    torch, lap = need_gpu()
    m, n, beta = 129, 65, 2.0
    psi, f, dx, dy = _problem(m, n, beta, True, 11)
    g = _ctx(torch, lap).grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
    say("zebra full solve", precision)
    kw = dict(precision=precision, smoother="zebra", nu1=1, nu2=1, tol=1e-10, max_iter=40)
    info = g.solve("mg", **kw)
    u1 = g.read().cpu().numpy()
    g.write(to_dev(torch, psi))
    info2 = g.solve("mg", **kw)
    assert info2["iterations"] == info["iterations"]
    assert np.array_equal(g.read().cpu().numpy(), u1)
    if precision == "fp64":
        ref, kref, _ = osolve.mg_solve(psi, f, dx, dy, tol=1e-10, nu1=1, nu2=1, smoother="zebra")
    else:
        ref, kref, _ = osolve.mixed_solve(psi, f, dx, dy, tol=1e-10, nu1=1, nu2=1, smoother="zebra")
    assert info["status"] == 0 and abs(info["iterations"] - kref) <= 1, (info, kref)
    assert info["iterations"] <= 9
    r0 = ogrid.norm2(ogrid.residual(psi, f, dx, dy))
    assert ogrid.norm2(ogrid.residual(u1, f, dx, dy)) / r0 < 1e-10 * 1.0001
    assert maxabs(u1, ref) <= 1e-10 * max(1.0, float(np.max(np.abs(ref))))
    g.destroy()


@pytest.mark.parametrize("precision,k", [("fp64", 2), ("mixed", 2), ("mixed", 3)])
def test_zebra_batch_vs_oracle_and_alone(precision, k):
    """Ten anisotropic ragged grids (4 to 6 levels) in merged launches: k
    cycles / steps against the oracle, and bitwise equal to each grid alone."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=10, lo=33, hi=257, seed=4, bumps=True)
    say("zebra batch", precision, k, [(p.m, p.n) for p in probs])
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = [ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy) for p in probs]
    kw = dict(method="mg", precision=precision, smoother="zebra", nu1=1, nu2=1, tol=0.0, max_iter=k)
    # a first solve leaves corrections in every buffer; the second, from the
    # reset inputs, must not see them
    ctx.solve_batch(gs, **{**kw, "max_iter": k + 1})
    for g, p in zip(gs, probs):
        g.write(to_dev(torch, p.psi0))
    infos = ctx.solve_batch(gs, **kw)
    for p, g, info in zip(probs, gs, infos):
        assert info["iterations"] == k
        lv = omg.hierarchy(p.m, p.n, p.dx, p.dy)
        ref = p.psi0.copy()
        for _ in range(k):
            if precision == "fp64":
                omg.vcycle(lv, 0, ref, p.f, 1, 1, smoother="zebra")
            else:
                omg.mixed_step(ref, p.f, lv, 1, 1, smoother="zebra")
        got = g.read().cpu().numpy()
        tol = 1e-10 if precision == "fp64" else 2e-6 * float(np.max(np.abs(ref)))
        assert maxabs(got, ref) <= tol, (p.m, p.n)
        alone = ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
        alone.solve(**{**{a: b for a, b in kw.items() if a != "method"}, "max_iter": k + 1}, method="mg")
        alone.write(to_dev(torch, p.psi0))
        alone.solve(**{a: b for a, b in kw.items() if a != "method"}, method="mg")
        assert np.array_equal(alone.read().cpu().numpy(), got), (p.m, p.n)
        alone.destroy()
    ctx.close()


def test_zebra_batch_converges_in_few_cycles():
    """The anisotropic ragged batch (beta in [0.5, 2]) solved to 1e-10 with
    mixed zebra-smoothed V(1,1) cycles: every grid in at most 9 outer steps
    (point red-black V(2,2) needs up to 14 on this mix), and each grid's
    residual, recomputed by the oracle, below tol."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=24, lo=33, hi=257, seed=4)
    say("zebra batch to tol", [(p.m, p.n) for p in probs])
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = [ctx.grid(to_dev(torch, p.psi0), None, p.dx, p.dy) for p in probs]
    infos = ctx.solve_batch(gs, method="mg", precision="mixed", smoother="zebra", nu1=1, nu2=1, tol=1e-10,
                            max_iter=40)
    for p, g, info in zip(probs, gs, infos):
        assert info["status"] == 0 and info["iterations"] <= 9, (p.m, p.n, info)
        u = g.read().cpu().numpy()
        r0 = ogrid.norm2(ogrid.residual(p.psi0, None, p.dx, p.dy))
        assert ogrid.norm2(ogrid.residual(u, None, p.dx, p.dy)) / r0 < 1e-10 * 1.0001
    ctx.close()


def test_zebra_argument_errors():
    torch, lap = need_gpu()
    from paper_2208_02427_amd import LapError
    ctx = _ctx(torch, lap)
    psi = np.zeros((9, 8193))
    psi[0, :] = 1.0
    g = ctx.grid(to_dev(torch, psi), None, 1.0 / 8192, 1.0 / 8)
    with pytest.raises(LapError):                 # rows of 8191 unknowns exceed the segmented solver
        g.solve("mg", smoother="zebra", nu1=1, nu2=1, raise_on_fail=True)
    g.destroy()
    g = ctx.grid(to_dev(torch, np.zeros((17, 17))), None, 0.1, 0.1)
    with pytest.raises(LapError):
        g.solve("mg", smoother="zebra", nu1=9, nu2=1, raise_on_fail=True)
    with pytest.raises(LapError):
        g.solve("mg", smoother=7, raise_on_fail=True)
    g.destroy()
