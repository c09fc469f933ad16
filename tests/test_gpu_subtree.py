"""Small-level subtree: the part of a V-cycle below the first level whose
remaining hierarchy fits one workgroup's LDS runs as one launch.  Every node
value is formed by the same expression on the same operands as in the
multi-launch schedule, so solutions are compared bit for bit with the
subtree switched off; the oracle's residual of the result checks the tolerance.
"""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, rand_problem
from oracle import grid as ogrid

pytestmark = pytest.mark.gpu

KC_SUBTREE = 9


def _solve(lap, torch, ctx, prob, sub, **kw):
    psi, f, dx, dy = prob
    ctx.set_subtree(sub)
    ctx.set_timing(True)
    ctx.reset_stats()
    g = ctx.grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)
    info = g.solve("mg", **kw)
    out = g.read().cpu().numpy()
    launches = ctx.kernel_stats(KC_SUBTREE)["launches"]
    g.destroy()
    ctx.set_timing(False)
    return info, out, launches


CASES = [
    # m, n, precision, nu1, nu2, omega
    (257, 257, "fp64", 2, 2, 1.0),
    (257, 129, "mixed", 2, 2, 1.0),
    (129, 513, "fp64", 1, 1, 1.0),
    (513, 257, "mixed", 3, 1, 1.15),
    (65, 65, "fp64", 0, 2, 1.0),
    (65, 97, "mixed", 1, 3, 0.9),
    (33, 33, "mixed", 2, 2, 1.0),
]


@pytest.mark.parametrize("m,n,precision,nu1,nu2,omega", CASES)
def test_subtree_bitwise_vs_multilaunch(m, n, precision, nu1, nu2, omega):
    torch, lap = need_gpu()
    # mesh ratio dy/dx = 1.3: point smoothing keeps its multigrid rate
    prob = rand_problem(m, n, seed=m + 7 * n, dx=1.0 / (m - 1), dy=1.3 / (m - 1))
    kw = dict(precision=precision, tol=1e-10, max_iter=40, nu1=nu1, nu2=nu2, omega=omega)
    say("subtree", m, n, precision, nu1, nu2, omega)
    ctx = lap.Context(arena_bytes=256 << 20)
    _, lds = ctx.get_subtree()
    assert lds >= 32768
    off = _solve(lap, torch, ctx, prob, 0, **kw)
    on = _solve(lap, torch, ctx, prob, -1, **kw)
    assert off[2] == 0
    assert on[2] > 0, "the subtree was not used"
    assert on[0]["iterations"] == off[0]["iterations"]
    assert on[0]["status"] == 0
    assert np.array_equal(on[1], off[1])
    psi, f, dx, dy = prob
    r0 = ogrid.norm2(ogrid.residual(psi, f, dx, dy))
    assert ogrid.norm2(ogrid.residual(on[1], f, dx, dy)) / r0 < 1e-10 * 1.0001
    ctx.close()


def test_subtree_node_limit_moves_the_root():
    """A node cap picks a lower root; the field stays bitwise the same."""
    torch, lap = need_gpu()
    prob = rand_problem(257, 257, seed=11)
    kw = dict(precision="fp64", tol=0.0, max_iter=3)
    ctx = lap.Context(arena_bytes=256 << 20)
    outs = []
    for cap in (0, -1, 33 * 33, 17 * 17):
        say("subtree cap", cap)
        info, out, launches = _solve(lap, torch, ctx, prob, cap, **kw)
        assert info["iterations"] == 3
        assert (launches > 0) == (cap != 0)
        outs.append(out)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert ctx.get_subtree()[0] == 17 * 17
    with pytest.raises(lap.LapError):
        ctx.set_subtree(-2)
    ctx.close()


def test_subtree_with_separable_coarsest():
    """Long thin grid: the FP32 V-cycle's subtree ends in the separable
    coarsest solve (more than 256 coarsest unknowns)."""
    torch, lap = need_gpu()
    m, n = 9, 1025
    prob = rand_problem(m, n, seed=5, dx=1.0 / 1024, dy=1.0 / 1024)
    kw = dict(precision="mixed", tol=1e-10, max_iter=40)
    say("subtree separable", m, n)
    ctx = lap.Context(arena_bytes=256 << 20)
    off = _solve(lap, torch, ctx, prob, 0, **kw)
    on = _solve(lap, torch, ctx, prob, -1, **kw)
    assert on[2] > 0
    assert on[0]["status"] == 0 and on[0]["iterations"] == off[0]["iterations"]
    assert np.array_equal(on[1], off[1])
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_subtree_bitwise(precision):
    """Merged launches: one subtree workgroup per grid of a ragged batch."""
    torch, lap = need_gpu()
    probs = W.ragged_batch(count=10, lo=33, hi=257, seed=4)
    kw = dict(method="mg", precision=precision, tol=1e-10, max_iter=60)
    res = {}
    for sub in (0, -1):
        say("batch subtree", precision, sub)
        ctx = lap.Context(arena_bytes=1 << 30)
        ctx.set_subtree(sub)
        ctx.set_timing(True)
        gs = [ctx.grid(to_dev(torch, p.psi0), None if p.f is None else to_dev(torch, p.f), p.dx, p.dy)
              for p in probs]
        infos = ctx.solve_batch(gs, **kw)
        res[sub] = ([g.read().cpu().numpy() for g in gs], [i["iterations"] for i in infos],
                    ctx.kernel_stats(KC_SUBTREE)["launches"])
        ctx.close()
    assert res[0][2] == 0 and res[-1][2] > 0
    assert res[0][1] == res[-1][1]
    for a, b in zip(res[0][0], res[-1][0]):
        assert np.array_equal(a, b)
