"""Fused smoothing passes (two sweeps per pass; residual + full weighting
folded into the last pre-smoothing pass; bilinear correction into the first
post-smoothing pass).  A fused pass evaluates every node with the one-sweep
kernels' expressions on the same operands, so solutions are compared bit for
bit with fusion switched off, across tilings and halos, alone and batched."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, rand_problem
from oracle import grid as ogrid

pytestmark = pytest.mark.gpu

KC_PRE, KC_TWO, KC_RESIDUAL = 10, 11, 8


def _run(lap, torch, prob, fuse, sub=-1, tiling=None, **kw):
    psi, f, dx, dy = prob
    ctx = lap.Context(arena_bytes=256 << 20)
    ctx.set_fusion(fuse)
    ctx.set_subtree(sub)
    if tiling is not None:
        V, ty, tgt = tiling
        for sc in range(8):
            for cls in range(15):
                for dt in (0, 1):
                    ctx.set_tiling(cls, dt, sc, V, ty, tgt)
    ctx.set_timing(True)
    g = ctx.grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)
    info = g.solve("mg", **kw)
    out = g.read().cpu().numpy()
    fused = ctx.kernel_stats(KC_PRE)["launches"] + ctx.kernel_stats(KC_TWO)["launches"]
    g.destroy()
    ctx.close()
    return info, out, fused


CASES = [
    # m, n, precision, nu1, nu2, source
    (257, 257, "fp64", 2, 2, False),
    (257, 257, "fp64", 2, 2, True),
    (513, 129, "mixed", 2, 2, True),
    (129, 257, "fp64", 1, 1, True),
    (129, 129, "fp64", 3, 1, False),
    (129, 129, "mixed", 1, 3, True),
    (257, 129, "fp64", 0, 2, True),
    (129, 129, "fp64", 4, 2, True),
    (65, 33, "mixed", 2, 2, True),
    (129, 257, "mixed", 4, 2, True),     # post + defect pass after two pre passes
    (257, 129, "mixed", 2, 2, False),
    (4097, 129, "mixed", 2, 2, True),    # many windows, 16-row chunks with row-block norm partials
]


@pytest.mark.parametrize("m,n,precision,nu1,nu2,source", CASES)
def test_fused_bitwise_vs_unfused(m, n, precision, nu1, nu2, source):
    torch, lap = need_gpu()
    prob = rand_problem(m, n, seed=3 * m + n, dx=1.0 / (m - 1), dy=1.2 / (m - 1), source=source)
    kw = dict(precision=precision, tol=1e-10, max_iter=40, nu1=nu1, nu2=nu2)
    say("fused", m, n, precision, nu1, nu2, source)
    sub = 0 if m * n < 65 * 65 else -1      # small grids: the whole FP32 cycle would be one subtree
    off = _run(lap, torch, prob, False, sub=sub, **kw)
    on = _run(lap, torch, prob, True, sub=sub, **kw)
    assert off[2] == 0 and on[2] > 0
    assert on[0]["status"] == 0 and on[0]["iterations"] == off[0]["iterations"]
    assert np.array_equal(on[1], off[1])
    psi, f, dx, dy = prob
    r0 = ogrid.norm2(ogrid.residual(psi, f, dx, dy))
    assert ogrid.norm2(ogrid.residual(on[1], f, dx, dy)) / r0 < 1e-10 * 1.0001


@pytest.mark.parametrize("tiling", [(1, 16, 0), (2, 32, 0), (4, 16, 0), (2, 0, 256), (4, 0, 8192), (1, 0, 64)])
def test_fused_bitwise_across_tilings(tiling):
    """Many windows and chunks, ragged last window and chunk, no subtree
    (every level through the streaming kernels)."""
    torch, lap = need_gpu()
    prob = rand_problem(449, 321, seed=17)
    kw = dict(precision="fp64", tol=0.0, max_iter=3)
    say("fused tiling", tiling)
    ref = _run(lap, torch, prob, False, sub=0, **kw)
    got = _run(lap, torch, prob, True, sub=0, tiling=tiling, **kw)
    assert np.array_equal(got[1], ref[1])
    kw["precision"] = "mixed"
    ref = _run(lap, torch, prob, False, sub=0, **kw)
    got = _run(lap, torch, prob, True, sub=0, tiling=tiling, **kw)
    assert np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_fused_bitwise(precision):
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=10, lo=33, hi=513, seed=9, bumps=True)
    kw = dict(method="mg", precision=precision, tol=1e-10, max_iter=60)
    res = {}
    for fuse in (False, True):
        say("batch fused", precision, fuse)
        ctx = lap.Context(arena_bytes=1 << 30)
        ctx.set_fusion(fuse)
        ctx.set_timing(True)
        gs = [ctx.grid(to_dev(torch, p.psi0), None if p.f is None else to_dev(torch, p.f), p.dx, p.dy)
              for p in probs]
        infos = ctx.solve_batch(gs, **kw)
        res[fuse] = ([g.read().cpu().numpy() for g in gs], [i["iterations"] for i in infos],
                     ctx.kernel_stats(KC_PRE)["launches"])
        ctx.close()
    assert res[False][2] == 0 and res[True][2] > 0
    assert res[False][1] == res[True][1]
    for a, b in zip(res[False][0], res[True][0]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("max_iter,tol", [(1, 0.0), (2, 0.0), (3, 0.0), (40, 1e30), (40, 1e-10)])
def test_fused_stops_and_restarts(max_iter, tol):
    """FP64 V(2,2), fused passes against one launch per sweep: stopping after
    1, 2, 3 cycles, at the initial iterate, at convergence; then a warm
    restart of the same grid from its result.  Bitwise, with the same
    iteration counts."""
    torch, lap = need_gpu()
    psi, f, dx, dy = rand_problem(129, 97, seed=21, dx=1.0 / 128, dy=1.0 / 96, source=True)
    res = {}
    for fuse in (False, True):
        ctx = lap.Context(arena_bytes=256 << 20)
        ctx.set_fusion(fuse)
        g = ctx.grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
        i1 = g.solve("mg", precision="fp64", tol=tol, max_iter=max_iter)
        a = g.read().cpu().numpy()
        i2 = g.solve("mg", precision="fp64", tol=1e-10, max_iter=40)
        b = g.read().cpu().numpy()
        res[fuse] = (i1["iterations"], a, i2["iterations"], b)
        g.destroy()
        ctx.close()
    say("stops", max_iter, tol, res[False][0], res[False][2])
    assert res[False][0] == res[True][0] and res[False][2] == res[True][2]
    assert np.array_equal(res[False][1], res[True][1])
    assert np.array_equal(res[False][3], res[True][3])


@pytest.mark.parametrize("mode", [1, 2])
def test_timing_counts_only_full_work_launches(mode):
    """Kernel statistics of a solve hold exactly the launches before and
    including the deciding stopping test: one fused pre pass per cycle, one
    post pass per cycle, and the final test (speculative launches after the
    device stopped are left out).  The final test is the norms-only probe of
    the pre pass (timed with the residual-norm kernels) once the tests predict
    it ends the solve, as on this geometric convergence.  Mode 2 times the
    finest level only."""
    torch, lap = need_gpu()
    p = W.square_problem(513, seed=2)
    ctx = lap.Context(arena_bytes=256 << 20)
    ctx.set_timing(mode)
    g = ctx.grid(to_dev(torch, p.psi0), None, p.dx, p.dy)
    say("timing", mode)
    for _ in range(2):
        ctx.reset_stats()
        g.write(to_dev(torch, p.psi0))
        info = g.solve("mg", tol=1e-10, max_iter=40)
        k = info["iterations"]
        pre = ctx.kernel_stats(KC_PRE, fine_only=True)
        two = ctx.kernel_stats(KC_TWO, fine_only=True)
        probe = ctx.kernel_stats(KC_RESIDUAL, fine_only=True)
        assert probe["launches"] == 1
        assert pre["launches"] == k and two["launches"] == k
        assert pre["device_ms"] > 0 and two["device_ms"] > 0
        allp = ctx.kernel_stats(KC_PRE)
        assert allp["launches"] > pre["launches"]          # coarse levels counted too
        if mode == 2:
            assert allp["device_ms"] == pytest.approx(pre["device_ms"])   # ... but not timed
    g.destroy()
    ctx.close()


KC_DEFECT = 3


@pytest.mark.parametrize("max_iter,tol", [(1, 0.0), (2, 0.0), (3, 0.0), (4, 0.0), (40, 1e-10)])
def test_mixed_post_defect_pass(max_iter, tol):
    """Mixed V(2,2) with fusion: every outer step after the first opens with
    one pass that finishes the previous FP32 cycle (its level-0 bilinear
    correction + two sweeps) and does this step's FP64 defect correction, so
    the level-0 FP32 post-smoothing never has a launch of its own.  Bitwise
    against fusion off, eager and with graph replay (two steps per graph),
    stopping after 1-4 steps and at convergence, then a warm restart."""
    torch, lap = need_gpu()
    psi, f, dx, dy = rand_problem(257, 193, seed=23, dx=1.0 / 256, dy=1.0 / 192, source=True)
    res = {}
    for mode in ("off", "eager", "graph"):
        ctx = lap.Context(arena_bytes=256 << 20)
        ctx.set_fusion(mode != "off")
        g = ctx.grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
        kw = dict(precision="mixed", use_graph=(mode == "graph"))
        i1 = g.solve("mg", tol=tol, max_iter=max_iter, **kw)
        a = g.read().cpu().numpy()
        i2 = g.solve("mg", tol=1e-10, max_iter=40, **kw)
        b = g.read().cpu().numpy()
        res[mode] = (i1["iterations"], a, i2["iterations"], b)
        g.destroy()
        ctx.close()
    say("post+defect", max_iter, tol, res["off"][0], res["off"][2])
    for mode in ("eager", "graph"):
        assert res[mode][0] == res["off"][0] and res[mode][2] == res["off"][2]
        assert np.array_equal(res[mode][1], res["off"][1])
        assert np.array_equal(res[mode][3], res["off"][3])


def test_mixed_post_defect_launch_counts():
    """With the post + defect pass, a mixed solve of k steps records k + 1
    defect-class launches (the first step's plain defect correction, then one
    fused pass per step up to the deciding test) and no level-0 FP32
    post-smoothing launch."""
    torch, lap = need_gpu()
    psi, f, dx, dy = rand_problem(513, 257, seed=29, dx=1.0 / 512, dy=1.0 / 256, source=True)
    ctx = lap.Context(arena_bytes=256 << 20)
    ctx.set_timing(True)
    g = ctx.grid(to_dev(torch, psi), to_dev(torch, f), dx, dy)
    info = g.solve("mg", precision="mixed", tol=1e-10, max_iter=40)
    k = info["iterations"]
    say("post+defect counts", k)
    assert info["status"] == 0 and k >= 3
    assert ctx.kernel_stats(KC_DEFECT)["launches"] == k + 1
    assert ctx.kernel_stats(KC_TWO, fine_only=True)["launches"] == 0
    assert ctx.kernel_stats(KC_PRE, fine_only=True)["launches"] == k
    g.destroy()
    ctx.close()


def test_mixed_norms_alone_equal_batched():
    """Alone, the post + defect pass of a level of <= 1025 rows walks 16-row
    chunks; in a merged batch launch, 64-row chunks.  Its norm partials are
    kept per (window, row) there, so both reduce the same values in the same
    order: the reported residuals are bitwise equal, as are the iterates and
    the iteration counts (taller levels share one tiling)."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=8, lo=97, hi=513, seed=13, bumps=True)
    probs.append(W.square_problem(1281, seed=2, bumps=True, bump_seed=3))
    say("norms alone/batched", [(p.m, p.n) for p in probs])
    assert any(p.n <= 1025 for p in probs) and any(p.n > 1025 for p in probs)
    ctx = lap.Context(arena_bytes=1 << 30)
    gs = [ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy) for p in probs]
    infos = ctx.solve_batch(gs, method="mg", precision="mixed", tol=1e-10, max_iter=60)
    outs = [g.read().cpu().numpy() for g in gs]
    ctx.close()
    ctx2 = lap.Context(arena_bytes=1 << 30)
    for p, ib, ub in zip(probs, infos, outs):
        g = ctx2.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
        ia = g.solve("mg", precision="mixed", tol=1e-10, max_iter=60)
        assert ia["status"] == 0 and ia["iterations"] == ib["iterations"]
        assert ia["rel_res_l2"] == ib["rel_res_l2"] and ia["res_linf"] == ib["res_linf"], (p.m, p.n)
        assert np.array_equal(g.read().cpu().numpy(), ub)
        g.destroy()
    ctx2.close()
