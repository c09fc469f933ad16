"""The paper's sequential methods on the GPU (one workgroup, grid in LDS)
against the oracle.

Methods: Jacobi (Eq. (5)), lexicographic Gauss-Seidel / SOR (Eqs. (6)-(7)),
SLORA / SLORB (Eqs. (8)-(10)) and ADI in the paper's order (rows ascending,
then columns ascending).  The GPU evaluates the same unfused expressions on
the same operands in the same order (lexicographic SOR by anti-diagonals,
the line methods line after line), so the iteration counts are the oracle's
and the fields agree bit for bit; the paper's own printed counts on the
25 x 17 chamber (SLORB 55 at w = 1.25, ADI 33 at w = 1.3, wall AB read as
psi = 1, Eq. (16) stopping rule) come out of the GPU as well."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev
from oracle import solve as osolve, direct

pytestmark = pytest.mark.gpu

# (GPU method, adi_form) -> oracle method name
ORACLE = {("jacobi", "after"): "jacobi", ("sor_lex", "after"): "sor_lex", ("slor_lex", "after"): "slora",
          ("slor_lex", "inside"): "slorb", ("adi_lex", "after"): "adi_lex_a", ("adi_lex", "inside"): "adi_lex_b"}

_CTX = {}


def _ctx(torch, lap):
    if "c" not in _CTX:
        _CTX["c"] = lap.Context(arena_bytes=256 << 20)
    return _CTX["c"]


def _gpu_solve(torch, lap, p, method, omega, form, stop, tol, max_iter=20000, f=None):
    g = _ctx(torch, lap).grid(to_dev(torch, p.psi0), None if f is None else to_dev(torch, f), p.dx, p.dy)
    info = g.solve(method, omega=omega, adi_form=form, stop=stop, tol=tol, max_iter=max_iter)
    u = g.read().cpu().numpy()
    g.destroy()
    return info, u


@pytest.mark.parametrize("method,form,omega", [("jacobi", "after", 1.0), ("sor_lex", "after", 1.0),
                                               ("sor_lex", "after", 1.75), ("slor_lex", "after", 1.0),
                                               ("slor_lex", "after", 1.6), ("slor_lex", "inside", 1.25),
                                               ("adi_lex", "inside", 1.3), ("adi_lex", "after", 1.0)])
def test_chamber_paper_rule_bitwise(method, form, omega, paper):
    """Chamber, psi_AB = 1, max|dpsi| < 1e-9 (Eq. (16)): the oracle's count
    and field, bit for bit."""
    torch, lap = need_gpu()
    p = W.chamber(psi_ab=1.0)
    tol = paper["stop"]["tol_delta"]
    say("paper method", method, form, omega)
    info, u = _gpu_solve(torch, lap, p, method, omega, form, "delta", tol)
    ref, k, h = osolve.iterate(ORACLE[(method, form)], p.psi0, None, p.dx, p.dy, omega, "delta", tol)
    assert info["status"] == 0
    assert info["iterations"] == k
    assert info["monitor"] == h[-1]
    assert np.array_equal(u, ref)


def test_paper_printed_counts_on_gpu(paper):
    """Figure 15 text: SLORB 55 iterations at w = 1.25 and ADI 33 at w = 1.3."""
    torch, lap = need_gpu()
    p = W.chamber(psi_ab=1.0)
    tol = paper["stop"]["tol_delta"]
    i_b, _ = _gpu_solve(torch, lap, p, "slor_lex", paper["omega_opt"]["slorb"], "inside", "delta", tol)
    i_a, _ = _gpu_solve(torch, lap, p, "adi_lex", paper["omega_opt"]["adi"], "inside", "delta", tol)
    assert i_b["iterations"] == paper["iterations_at_opt"]["slorb"]
    assert i_a["iterations"] == paper["iterations_at_opt"]["adi"]


def test_sor_lex_omega_sweep_matches_oracle():
    """The config-1 sweep w = 1.00 .. 1.95 of lexicographic SOR on the chamber
    (psi_AB = 100, max|r| < 1e-6): the oracle's count at every w, and the
    same best w."""
    torch, lap = need_gpu()
    p = W.chamber(psi_ab=100.0)
    gpu, orc = {}, {}
    for k in range(20):
        w = round(1.0 + 0.05 * k, 2)
        info, u = _gpu_solve(torch, lap, p, "sor_lex", w, "after", "res_inf", 1e-6)
        ref, kk, _ = osolve.iterate("sor_lex", p.psi0, None, p.dx, p.dy, w, "res_inf", 1e-6)
        gpu[w], orc[w] = info["iterations"], kk
        assert np.array_equal(u, ref), w
    say("sor_lex sweep", gpu)
    assert gpu == orc
    assert min(gpu, key=lambda w: (gpu[w], w)) == min(orc, key=lambda w: (orc[w], w))


@pytest.mark.parametrize("method,form", [("jacobi", "after"), ("sor_lex", "after"), ("slor_lex", "after"),
                                         ("adi_lex", "after"), ("adi_lex", "inside")])
def test_anisotropic_grid_with_source(method, form):
    """31 x 20, dx != dy, random boundary and source: fixed iteration counts
    bitwise against the oracle, then a converged solve against the dense
    direct solution."""
    torch, lap = need_gpu()
    rng = np.random.default_rng(3)
    m, n, dx, dy = 31, 20, 0.07, 0.05
    psi = W.random_boundary(m, n, rng)
    f = rng.standard_normal((n, m)) * 10.0
    p = W.Problem(m, n, dx, dy, psi, f, name="aniso")
    w = 1.2
    say("paper method aniso", method, form)
    info, u = _gpu_solve(torch, lap, p, method, w, form, "delta", 0.0, max_iter=7, f=f)
    assert info["iterations"] == 7
    ref = psi.copy()
    om = ORACLE[(method, form)]
    ref, _, _ = osolve.iterate(om, psi, f, dx, dy, w, "delta", 0.0, max_iter=7)
    assert np.array_equal(u, ref)
    info, u = _gpu_solve(torch, lap, p, method, w, form, "rel_l2", 1e-12, max_iter=20000, f=f)
    ex = direct.dense_solve(m, n, dx, dy, psi, f)
    assert info["status"] == 0
    assert np.max(np.abs(u - ex)) <= 1e-9 * max(1.0, np.max(np.abs(ex)))


def test_paper_method_errors():
    torch, lap = need_gpu()
    from paper_2208_02427_amd import LapError
    ctx = _ctx(torch, lap)
    big = ctx.grid(to_dev(torch, np.zeros((257, 257))), None, 0.1, 0.1)      # does not fit LDS
    with pytest.raises(LapError):
        big.solve("sor_lex", raise_on_fail=True)
    big.destroy()
    g = ctx.grid(to_dev(torch, np.zeros((17, 9))), None, 0.1, 0.2)          # beta^2 = cy / cx = 0.25
    with pytest.raises(LapError):
        ctx.solve_batch([g], method="jacobi")
    with pytest.raises(LapError):                                           # SLORB needs w < 1 + beta^2
        g.solve("slor_lex", omega=1.3, adi_form="inside", raise_on_fail=True)
    g.destroy()
