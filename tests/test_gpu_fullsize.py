"""Parity at the benchmark's full size, in the launch configuration the
benchmark times (shipped tiling table, fused passes, small-level subtree):
the 8193 x 8193 unit-square problems, one GPU step each, against the oracle
run on the whole grid on the host.

* FP64 V(2,2) cycle (the headline workload): max-abs <= 1e-10;
* red-black SOR at the optimal omega, a block of sweeps, on sampled rows
  (bands the oracle sweeps on their own): max-abs <= 1e-10;
* one mixed-precision outer step on the 32-bump problem: the FP32 inner
  cycle differs from the oracle's float32 emulation by rounding only, gated
  at 2e-6 of the field scale as at the smaller sizes.

The whole-grid oracle steps take about a minute of host time each.
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, maxabs
from oracle import relax, multigrid as omg, grid as ogrid

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 8193


def _ctx():
    torch, lap = need_gpu()
    return torch, lap, lap.Context(arena_bytes=6 << 30)


@pytest.mark.timeout(900)
def test_fp64_vcycle_full_size():
    torch, lap, ctx = _ctx()
    p = W.square_problem(N, seed=2)
    say("full-size fp64 V-cycle", N)
    g = ctx.grid(to_dev(torch, p.psi0), None, p.dx, p.dy, alloc=lap.LAP_ALLOC_FP64)
    info = g.solve("mg", precision="fp64", tol=0.0, max_iter=1)
    assert info["iterations"] == 1
    got = g.read().cpu().numpy()
    g.destroy()
    ctx.close()
    lv = omg.hierarchy(N, N, p.dx, p.dy)
    ref = p.psi0.copy()
    omg.vcycle(lv, 0, ref, None)
    err = maxabs(got, ref)
    say("max-abs vs oracle", err)
    assert err <= 1e-10


def test_sor_sweeps_full_size():
    """k sweeps move information 2 rows per sweep, so a row of the result is
    fixed by the input rows within 2k of it: the oracle sweeps a band of
    rows (starting on an even row, so colours keep their global parity; the
    band's first and last rows held fixed) and its centre rows are exact."""
    torch, lap, ctx = _ctx()
    p = W.square_problem(N, seed=2)
    w = 2.0 / (1.0 + math.sin(math.pi * p.dx))
    k = 10
    say("full-size RB-SOR", N, k, w)
    g = ctx.grid(to_dev(torch, p.psi0), None, p.dx, p.dy, alloc=lap.LAP_ALLOC_FP64)
    info = g.solve("sor", omega=w, tol=0.0, max_iter=k, check_every=2)
    assert info["iterations"] == k
    got = g.read().cpu().numpy()
    g.destroy()
    ctx.close()
    R = 2 * k + 4
    rng = np.random.default_rng(11)
    rows = [1, 2, 3, 4, 64, 65, 4095, 4096, 4097, N - 5, N - 4, N - 3, N - 2] + list(rng.integers(1, N - 1, 8))
    worst = 0.0
    for c in rows:
        j0 = max(0, c - R) & ~1
        j1 = min(N - 1, c + R)
        band = p.psi0[j0:j1 + 1].copy()
        for _ in range(k):
            relax.rb_sweep(band, None, p.dx, p.dy, w)
        lo = 0 if j0 == 0 else 2 * k + 1
        hi = band.shape[0] - 1 if j1 == N - 1 else band.shape[0] - 2 * k - 2
        assert lo <= c - j0 <= hi
        worst = max(worst, maxabs(got[c], band[c - j0]))
    say("max-abs vs oracle over", len(rows), "rows", worst)
    assert worst <= 1e-10


@pytest.mark.timeout(900)
def test_mixed_step_full_size():
    torch, lap, ctx = _ctx()
    p = W.square_problem(N, seed=2, bumps=True, bump_seed=3)
    say("full-size mixed step", N)
    g = ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy, alloc=lap.LAP_ALLOC_MIXED)
    info = g.solve("mg", precision="mixed", tol=0.0, max_iter=1)
    assert info["iterations"] == 1
    got = g.read().cpu().numpy()
    g.destroy()
    ctx.close()
    lv = omg.hierarchy(N, N, p.dx, p.dy)
    ref = p.psi0.copy()
    omg.mixed_step(ref, p.f, lv)
    scale = float(np.max(np.abs(ref)))
    err = maxabs(got, ref)
    say("max-abs vs oracle", err, "scale", scale)
    assert err <= 2e-6 * scale
    # and the step reduced the FP64 residual as the oracle's did
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    rg = ogrid.norm2(ogrid.residual(got, p.f, p.dx, p.dy)) / r0
    rr = ogrid.norm2(ogrid.residual(ref, p.f, p.dx, p.dy)) / r0
    say("rel. residual gpu / oracle", rg, rr)
    assert rg == pytest.approx(rr, rel=1e-3)
