"""Iterate-level and converged parity of the GPU solvers (lap_solve_ex)
against the oracle, in the same ordering: red-black SOR sweeps, zebra ADI
iterations, FP64 V(2,2) cycles and mixed-precision outer steps.

Gate: FP64 results within 1e-10 max-abs of the oracle; the
error against the exact discrete solution is reported for converged runs.
Mixed precision is compared with the oracle's float32-emulated loop.
"""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev, rand_problem, maxabs
from oracle import relax, lines as olines, multigrid as omg, solve as osolve, direct, grid as ogrid

pytestmark = pytest.mark.gpu

_CTX = {}


def ctx():
    torch, lap = need_gpu()
    if "c" not in _CTX:
        _CTX["c"] = lap.Context(arena_bytes=2 << 30)
    return torch, lap, _CTX["c"]


def make_grid(psi, f, dx, dy):
    torch, lap, c = ctx()
    return c.grid(to_dev(torch, psi), None if f is None else to_dev(torch, f), dx, dy)


@pytest.mark.parametrize("m,n", [(3, 3), (4, 6), (33, 17), (129, 65), (130, 67), (257, 129)])
@pytest.mark.parametrize("k", [1, 5])
def test_sor_iterates(m, n, k):
    say("sor iterates", m, n, k)
    psi, f, dx, dy = rand_problem(m, n, m + n + k)
    g = make_grid(psi, f, dx, dy)
    info = g.solve("sor", omega=1.6, tol=0.0, max_iter=k)
    assert info["iterations"] == k
    ref = psi.copy()
    for _ in range(k):
        relax.rb_sweep(ref, f, dx, dy, 1.6)
    assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10
    g.destroy()


@pytest.mark.parametrize("m,n", [(33, 17), (129, 65), (130, 67), (257, 129)])
@pytest.mark.parametrize("ce", [2, 3, 5])
def test_sor_check_blocks(m, n, ce):
    """Check blocks of ce sweeps run as fused two-sweep passes (an odd block
    ends with a single sweep); two blocks against the oracle, and bitwise
    against one launch per sweep."""
    say("sor blocks", m, n, ce)
    psi, f, dx, dy = rand_problem(m, n, m + 3 * n + ce)
    torch, lap, c = ctx()
    outs = []
    for fuse in (True, False):
        c.set_fusion(fuse)
        g = make_grid(psi, f, dx, dy)
        info = g.solve("sor", omega=1.7, tol=0.0, max_iter=2 * ce, check_every=ce)
        assert info["iterations"] == 2 * ce
        outs.append(g.read().cpu().numpy())
        g.destroy()
    c.set_fusion(True)
    ref = psi.copy()
    for _ in range(2 * ce):
        relax.rb_sweep(ref, f, dx, dy, 1.7)
    assert maxabs(outs[0], ref) <= 1e-10
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("m,n", [(33, 17), (129, 65), (257, 257), (65, 129), (9, 9), (5, 5), (6, 6), (3, 3)])
@pytest.mark.parametrize("k", [1, 3])
def test_mg_fp64_cycles(m, n, k):
    say("mg64 cycles", m, n, k)
    psi, f, dx, dy = rand_problem(m, n, 7 * m + n + k)
    g = make_grid(psi, f, dx, dy)
    info = g.solve("mg", tol=0.0, max_iter=k)
    assert info["iterations"] == k
    lv = omg.hierarchy(m, n, dx, dy)
    assert g.levels() == [(a, b) for a, b, _, _ in lv]
    ref = psi.copy()
    for _ in range(k):
        omg.vcycle(lv, 0, ref, f)
    assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10
    g.destroy()


@pytest.mark.parametrize("use_graph", [True, False])
def test_mg_fp64_full_solve_matches_oracle(use_graph):
    """With graphs on, the first solve of a grid runs eagerly and a repeat
    with the same options replays the captured cycle: both are checked."""
    say("mg64 full", use_graph)
    torch, lap, c = ctx()
    p = W.square_problem(257, seed=2, bumps=True, bump_seed=3)
    g = make_grid(p.psi0, p.f, p.dx, p.dy)
    info = g.solve("mg", tol=1e-10, max_iter=50, use_graph=use_graph)
    first = g.read().cpu().numpy()
    g.write(to_dev(torch, p.psi0))
    info2 = g.solve("mg", tol=1e-10, max_iter=50, use_graph=use_graph)
    assert info2["iterations"] == info["iterations"]
    assert np.array_equal(g.read().cpu().numpy(), first)
    u_ref, k_ref, h_ref = osolve.mg_solve(p.psi0, p.f, p.dx, p.dy, tol=1e-10)
    assert info["status"] == 0
    assert info["iterations"] == k_ref
    assert info["rel_res_l2"] == pytest.approx(h_ref[-1], rel=1e-6)
    got = g.read().cpu().numpy()
    assert maxabs(got, u_ref) <= 1e-10
    # residual recomputed by the oracle from the returned field
    r = ogrid.residual(got, p.f, p.dx, p.dy)
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    assert ogrid.norm2(r) / r0 < 1e-10
    ex = direct.dst_solve(p.m, p.n, p.dx, p.dy, p.psi0, p.f)
    say("error vs exact discrete solution", maxabs(got, ex))
    g.destroy()


@pytest.mark.parametrize("m,n", [(65, 33), (129, 129), (257, 129)])
def test_mixed_steps(m, n):
    say("mixed steps", m, n)
    psi, f, dx, dy = rand_problem(m, n, 3 * m + n, interior=False)
    g = make_grid(psi, f, dx, dy)
    lv = omg.hierarchy(m, n, dx, dy)
    ref = psi.copy()
    for k in (1, 2, 3):
        g.write(to_dev(ctx()[0], psi))
        info = g.solve("mg", precision="mixed", tol=0.0, max_iter=k)
        assert info["iterations"] == k
        omg.mixed_step(ref, f, lv)
        scale = float(np.max(np.abs(ref)))
        # FP32 inner cycles differ by rounding only; the FP64 outer loop corrects it
        assert maxabs(g.read().cpu().numpy(), ref) <= 2e-6 * scale
    g.destroy()


def test_mixed_full_solve_reaches_fp64_accuracy():
    say("mixed full 513")
    p = W.square_problem(513, seed=2, bumps=True, bump_seed=3)
    g = make_grid(p.psi0, p.f, p.dx, p.dy)
    im = g.solve("mg", precision="mixed", tol=1e-10, max_iter=50)
    um = g.read().cpu().numpy()
    g.write(to_dev(ctx()[0], p.psi0))
    i64 = g.solve("mg", precision="fp64", tol=1e-10, max_iter=50)
    u64 = g.read().cpu().numpy()
    assert im["status"] == 0 and i64["status"] == 0
    assert abs(im["iterations"] - i64["iterations"]) <= 1
    r0 = ogrid.norm2(ogrid.residual(p.psi0, p.f, p.dx, p.dy))
    assert ogrid.norm2(ogrid.residual(um, p.f, p.dx, p.dy)) / r0 < 1e-10
    assert maxabs(um, u64) <= 1e-10 * max(1.0, np.max(np.abs(u64)))
    u_ref, k_ref, _ = osolve.mixed_solve(p.psi0, p.f, p.dx, p.dy, tol=1e-10)
    assert abs(im["iterations"] - k_ref) <= 1
    assert maxabs(um, u_ref) <= 1e-10
    say("mixed vs fp64 max-abs", maxabs(um, u64))
    g.destroy()


@pytest.mark.parametrize("form", ["after", "inside"])
@pytest.mark.parametrize("m,n", [(3, 3), (25, 17), (66, 35), (131, 200)])
def test_adi_iterates(form, m, n):
    say("adi iterates", m, n, form)
    psi, f, dx, dy = rand_problem(m, n, 5 * m + n, dx=0.1, dy=0.12)
    g = make_grid(psi, f, dx, dy)
    info = g.solve("adi", omega=1.2, tol=0.0, max_iter=3, adi_form=form)
    assert info["iterations"] == 3
    ref = psi.copy()
    for _ in range(3):
        olines.adi_zebra_iteration(ref, f, dx, dy, 1.2, "A" if form == "after" else "B")
    got = g.read().cpu().numpy()
    assert maxabs(got, ref) <= 1e-10
    g.destroy()


def test_chamber_all_gpu_methods():
    """Paper-sized chamber: every GPU method reaches max|r| < 1e-6 and the
    dense direct solution."""
    p = W.chamber(psi_ab=100.0)
    ex = direct.dense_solve(p.m, p.n, p.dx, p.dy, p.psi0, None)
    for method, kw in (("sor", dict(omega=1.0)), ("sor", dict(omega=1.7)), ("adi", dict(omega=1.0)),
                       ("adi", dict(omega=1.3, adi_form="inside")), ("mg", dict())):
        say("chamber", method, kw)
        g = make_grid(p.psi0, None, p.dx, p.dy)
        info = g.solve(method, tol=1e-6, stop="res_inf", max_iter=5000, **kw)
        assert info["status"] == 0, info
        got = g.read().cpu().numpy()
        assert ogrid.norm_inf(ogrid.residual(got, None, p.dx, p.dy)) < 1e-6
        assert maxabs(got, ex) < 1e-6
        # the oracle's own count for the same method / ordering
        if method == "sor":
            _, k, _ = osolve.iterate("rb", p.psi0, None, p.dx, p.dy, kw["omega"], "res_inf", 1e-6)
            assert info["iterations"] == k
        if method == "adi":
            mname = "adi_zebra_a" if kw.get("adi_form", "after") == "after" else "adi_zebra_b"
            _, k, _ = osolve.iterate(mname, p.psi0, None, p.dx, p.dy, kw["omega"], "res_inf", 1e-6)
            assert info["iterations"] == k
        if method == "mg":
            _, k, _ = osolve.mg_solve(p.psi0, None, p.dx, p.dy, tol=1e-6, stop="res_inf")
            assert info["iterations"] == k
        g.destroy()


@pytest.mark.parametrize("kind", ["x2-y2", "xy", "x3"])
def test_manufactured_reproduced_exactly(kind):
    say("manufactured", kind)
    p, exact = W.manufactured(kind, 25, 17, 0.25, 0.25)
    g = make_grid(p.psi0, p.f, p.dx, p.dy)
    info = g.solve("mg", tol=1e-13, max_iter=60)
    assert maxabs(g.read().cpu().numpy(), exact) <= 1e-10
    g.destroy()


def test_error_paths():
    torch, lap, c = ctx()
    say("error paths")
    psi, f, dx, dy = rand_problem(33, 33, 1)
    g = make_grid(psi, f, dx, dy)
    with pytest.raises(lap.LapError) as e:
        g.solve("sor", omega=2.0)
    assert e.value.status == -1
    info = g.solve("sor", omega=1.0, tol=1e-12, max_iter=3)
    assert info["status"] == -3 and info["iterations"] == 3
    with pytest.raises(lap.LapError):
        g.solve("sor", precision="mixed")
    with pytest.raises(lap.LapError):
        g.solve("mg", nu1=2, nu2=1)
    bad = psi.copy()
    bad[0, 3] = np.nan
    g.write(to_dev(torch, bad))
    info = g.solve("mg", tol=1e-10, max_iter=10)
    assert info["status"] == -4
    g.destroy()
    with pytest.raises(lap.LapError):
        make_grid(np.zeros((2, 5)), None, 1.0, 1.0)


def test_warm_start_continues():
    """k + k cycles equal 2k cycles bitwise (resume from the resident state)."""
    say("warm start")
    psi, f, dx, dy = rand_problem(129, 65, 9, interior=False)
    g1 = make_grid(psi, f, dx, dy)
    g1.solve("mg", tol=0.0, max_iter=2)
    g1.solve("mg", tol=0.0, max_iter=2)
    g2 = make_grid(psi, f, dx, dy)
    g2.solve("mg", tol=0.0, max_iter=4)
    assert np.array_equal(g1.read().cpu().numpy(), g2.read().cpu().numpy())
    g1.destroy()
    g2.destroy()


@pytest.mark.parametrize("m,n", [(6, 400), (401, 8), (3, 300), (130, 67), (4, 200)])
def test_separable_coarse_solve_single_level(m, n):
    """A grid that cannot coarsen and has more than 256 unknowns: multigrid
    is one separable direct solve (sine transform across the short side,
    tridiagonal solves along the long side), equal to the exact DST solution."""
    say("separable single level", m, n)
    psi, f, dx, dy = rand_problem(m, n, m * n, dx=0.01, dy=0.013, interior=False)
    g = make_grid(psi, f, dx, dy)
    assert g.levels() == [(m, n)]
    info = g.solve("mg", tol=0.0, max_iter=1)
    ex = direct.dst_solve(m, n, dx, dy, psi, f)
    assert maxabs(g.read().cpu().numpy(), ex) <= 1e-10 * max(1.0, np.max(np.abs(ex)))
    g.destroy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_separable_coarse_in_vcycle(precision):
    """9 x 1025 coarsens once to 5 x 513 (1533 unknowns, separable solve)."""
    say("separable coarse vcycle", precision)
    m, n = 9, 1025
    psi, f, dx, dy = rand_problem(m, n, 77, dx=1 / 1024, dy=1 / 1024, interior=False)
    g = make_grid(psi, f, dx, dy)
    assert g.levels() == [(9, 1025), (5, 513)]
    lv = omg.hierarchy(m, n, dx, dy)
    if precision == "fp64":
        info = g.solve("mg", tol=0.0, max_iter=1)
        ref = psi.copy()
        omg.vcycle(lv, 0, ref, f)
        assert maxabs(g.read().cpu().numpy(), ref) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
    info = g.solve("mg", precision=precision, tol=1e-10, max_iter=60)
    assert info["status"] == 0
    got = g.read().cpu().numpy()
    r0 = ogrid.norm2(ogrid.residual(psi, f, dx, dy))
    assert ogrid.norm2(ogrid.residual(got, f, dx, dy)) / r0 < 1e-10
    g.destroy()
