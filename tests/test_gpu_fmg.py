"""Full multigrid start on the GPU against the oracle (oracle.multigrid.fmg):
the FMG pass alone and followed by V-cycles agree to 1e-10; on a smooth
problem the pass alone ends at discretisation accuracy; a solve to 1e-10
that starts with it meets the tolerance (oracle-recomputed residual) in no
more iterations than plain V-cycles."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, maxabs
from oracle import multigrid as omg, grid as ogrid, direct

pytestmark = pytest.mark.gpu

_CTX = {}


def _ctx(torch, lap):
    if "c" not in _CTX:
        _CTX["c"] = lap.Context(arena_bytes=1 << 30)
    return _CTX["c"]


def _smooth(N):
    h = 1.0 / (N - 1)
    x = np.arange(N) * h
    X, Y = np.meshgrid(x, x)
    ue = np.sin(np.pi * X) * np.sin(2 * np.pi * Y) + X * Y * Y
    f = -5.0 * np.pi ** 2 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y) + 2.0 * X
    psi = ue.copy()
    psi[1:-1, 1:-1] = 0.0
    return psi, f, h, ue


def _random(m, n, beta, seed, src=True):
    rng = np.random.default_rng(seed)
    dy = 1.0 / (n - 1)
    dx = beta * dy
    psi = W.random_boundary(m, n, rng)
    f = W.gaussian_bumps(m, n, dx, dy, rng) if src else None
    return psi, f, dx, dy


@pytest.mark.parametrize("m,n,beta,src", [(65, 33, 1.7, True), (129, 129, 1.0, False), (257, 129, 0.8, True),
                                          (49, 97, 1.2, True)])
@pytest.mark.parametrize("k", [0, 2])
def test_fmg_then_cycles_vs_oracle(m, n, beta, src, k):
    torch, lap = need_gpu()
    psi, f, dx, dy = _random(m, n, beta, m + n + k, src)
    say("fmg", m, n, beta, src, k)
    g = _ctx(torch, lap).grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)
    info = g.solve("mg", fmg=True, tol=0.0, max_iter=1 + k)
    assert info["iterations"] == 1 + k
    lv = omg.hierarchy(m, n, dx, dy)
    ref = omg.fmg(lv, psi, f)
    for _ in range(k):
        omg.vcycle(lv, 0, ref, f)
    assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10 * max(1.0, float(np.max(np.abs(ref))))
    g.destroy()


def test_fmg_pass_reaches_discretisation_accuracy():
    torch, lap = need_gpu()
    N = 257
    psi, f, h, ue = _smooth(N)
    g = _ctx(torch, lap).grid(to_dev(torch, psi), to_dev(torch, f), h, h)
    g.solve("mg", fmg=True, tol=0.0, max_iter=1)
    u = g.read().cpu().numpy()
    ud = direct.dst_solve(N, N, h, h, psi, f)
    e_disc = np.max(np.abs(ud - ue))
    assert np.max(np.abs(u - ue)) <= 1.5 * e_disc
    assert np.max(np.abs(u - ud)) <= 0.5 * e_disc
    g.destroy()


@pytest.mark.parametrize("N", [257, 513])
def test_fmg_solve_to_tolerance(N):
    torch, lap = need_gpu()
    p = W.square_problem(N, seed=2, bumps=True, bump_seed=3)
    say("fmg solve", N)
    ctx = _ctx(torch, lap)
    g = ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
    plain = g.solve("mg", tol=1e-10, max_iter=60)
    up = g.read().cpu().numpy()
    res = []
    for rep in range(2):                      # the second solve replays the cycle graph
        g.write(to_dev(torch, p.psi0))
        info = g.solve("mg", fmg=True, tol=1e-10, max_iter=60)
        res.append((info, g.read().cpu().numpy()))
    (i1, u1), (i2, u2) = res
    assert i1["status"] == 0 and i1["iterations"] == i2["iterations"] and np.array_equal(u1, u2)
    assert i1["iterations"] <= plain["iterations"]
    assert i1["res0_l2"] == pytest.approx(plain["res0_l2"], rel=1e-12)
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    assert ogrid.norm2(ogrid.residual(u1, p.f, p.dx, p.dy)) / r0 < 1e-10 * 1.0001
    # both stop at a relative residual of 1e-10, which bounds their error
    # against the exact discrete solution only through ||L_h^-1|| (about
    # 1e-9 here): compare each with that solution
    ex = direct.dst_solve(p.m, p.n, p.dx, p.dy, p.psi0, p.f)
    e_fmg, e_plain = maxabs(u1, ex), maxabs(up, ex)
    say("fmg error vs exact", e_fmg, "plain", e_plain)
    assert e_fmg <= 1e-8 and e_plain <= 1e-8
    say("fmg cycles", i1["iterations"], "plain", plain["iterations"])
    g.destroy()


def test_fmg_argument_errors():
    torch, lap = need_gpu()
    from paper_2208_02427_amd import LapError
    ctx = _ctx(torch, lap)
    g = ctx.grid(to_dev(torch, np.zeros((33, 33))), None, 0.1, 0.1)
    for kw in (dict(precision="mixed"), dict(smoother="zebra", nu1=1, nu2=1)):
        with pytest.raises(LapError):
            g.solve("mg", fmg=True, raise_on_fail=True, **kw)
    with pytest.raises(LapError):
        g.solve("sor", fmg=True, raise_on_fail=True)
    with pytest.raises(LapError):
        ctx.solve_batch([g], method="mg", fmg=True)
    g.destroy()
