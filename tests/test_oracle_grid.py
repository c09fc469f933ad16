"""Pins for oracle.grid (operator, residual, norms) and oracle.direct
(dense elimination, DST solve): closed forms, library routines, invariants and
the grid counts the paper prints."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import grid, direct


def test_paper_grid_counts(paper):
    g = paper["grid"]
    p = W.chamber()
    # Eq. (4): m = Lx/dx + 1, n = Ly/dy + 1
    assert (p.m, p.n) == (g["m"], g["n"]) == (int(g["Lx"] / g["dx"]) + 1, int(g["Ly"] / g["dy"]) + 1)
    c = W.chamber_counts(p.m, p.n)
    assert c["total"] == g["total_points"]
    assert c["boundary_walls"] == g["boundary_points"]
    assert c["internal_paper"] == g["internal_points"]
    # the reading: 84 counts the four corners twice; the solver has 345 unknowns
    assert c["boundary_distinct"] == 80 and c["unknowns"] == 345
    assert c["unknowns"] + c["boundary_distinct"] == c["total"]


@pytest.mark.parametrize("kind", ["x2-y2", "xy", "x3-3xy2", "3x2y-y3"])
@pytest.mark.parametrize("dx,dy", [(0.25, 0.25), (0.3, 0.17), (1.0 / 40, 1.0 / 24)])
def test_operator_annihilates_harmonic_polynomials(kind, dx, dy):
    m, n = 23, 15
    u, _ = W.harmonic_field(kind, m, n, dx, dy, x0=-1.3, y0=0.7)
    Lu = grid.apply_L(u, dx, dy)
    cx, cy, d, _ = grid.coefficients(dx, dy)
    scale = d * np.max(np.abs(u))
    assert np.max(np.abs(Lu)) <= 1e-13 * scale


def test_printed_dx2_only_form_fails_on_anisotropic_grid():
    """Eq. (2)/(11) print dx^2 under the y term; with dx != dy that operator
    does not annihilate x^2 - y^2, while the dy^2 reading does."""
    dx, dy = 0.3, 0.17
    u, _ = W.harmonic_field("x2-y2", 9, 9, dx, dy)
    printed = grid.apply_L(u, dx, dx)          # cy = 1/dx^2
    assert np.max(np.abs(printed[1:-1, 1:-1])) > 1.0
    assert np.max(np.abs(grid.apply_L(u, dx, dy))) < 1e-10


def test_operator_on_cubic_gives_exact_laplacian():
    dx, dy = 0.2, 0.35
    u, lap = W.harmonic_field("x3", 17, 13, dx, dy, x0=0.4)
    Lu = grid.apply_L(u, dx, dy)
    assert np.allclose(Lu[1:-1, 1:-1], lap[1:-1, 1:-1], rtol=0, atol=1e-10)
    r = grid.residual(u, lap, dx, dy)
    assert np.max(np.abs(r)) < 1e-10


def test_operator_matches_dense_assembly():
    """-L_h on the interior (zero boundary) equals the assembled matrix,
    which is symmetric positive definite."""
    rng = np.random.default_rng(0)
    m, n, dx, dy = 8, 6, 0.3, 0.2
    A, rhs = direct.assemble(m, n, dx, dy, np.zeros((n, m)), None)
    assert np.array_equal(A, A.T)
    assert np.min(np.linalg.eigvalsh(A)) > 0
    x = rng.standard_normal((n - 2) * (m - 2))
    u = np.zeros((n, m))
    u[1:-1, 1:-1] = x.reshape(n - 2, m - 2)
    assert np.allclose(-grid.apply_L(u, dx, dy)[1:-1, 1:-1].ravel(), A @ x, rtol=1e-13, atol=1e-12)


def test_difference_form_residual():
    """residual_diff equals the assembled operator (as residual does) in FP64,
    reproduces the exact Laplacian of a cubic, and in FP32 on a smooth field
    of large values on a fine grid (h = 1/8192) stays within 1e-3 of the FP64
    residual of the stored values relative to its size, where the standard
    form is off by a quarter of the residual or more."""
    rng = np.random.default_rng(0)
    m, n, dx, dy = 8, 6, 0.3, 0.2
    A, _ = direct.assemble(m, n, dx, dy, np.zeros((n, m)), None)
    x = rng.standard_normal((n - 2) * (m - 2))
    u = np.zeros((n, m))
    u[1:-1, 1:-1] = x.reshape(n - 2, m - 2)
    assert np.allclose(grid.residual_diff(u, None, dx, dy)[1:-1, 1:-1].ravel(), A @ x, rtol=1e-13, atol=1e-12)
    dx, dy = 0.2, 0.35
    uc, lap = W.harmonic_field("x3", 17, 13, dx, dy, x0=0.4)
    assert np.max(np.abs(grid.residual_diff(uc, lap, dx, dy))) < 1e-10
    h = 1.0 / 8192
    i = np.arange(40)
    X, Y = np.meshgrid(0.3 + h * i, 0.6 + h * i)
    us = np.sin(np.pi * X) * np.sin(np.pi * Y)           # smooth, values near 0.8
    u32 = us.astype(np.float32)
    ref = grid.residual(u32.astype(np.float64), None, h, h)[1:-1, 1:-1]   # exact for the stored values
    scale = np.max(np.abs(ref))                            # about 2 pi^2 |u|
    d32 = grid.residual_diff(u32, None, h, h, np.float32)[1:-1, 1:-1]
    s32 = grid.residual(u32, None, h, h, np.float32)[1:-1, 1:-1]
    assert np.max(np.abs(d32 - ref)) < 1e-3 * scale
    assert np.max(np.abs(s32 - ref)) > 0.25 * scale


def test_norms_against_numpy():
    rng = np.random.default_rng(1)
    r = rng.standard_normal((11, 13))
    assert grid.norm2(r) == pytest.approx(np.linalg.norm(r[1:-1, 1:-1]), rel=1e-14)
    assert grid.norm_inf(r) == np.max(np.abs(r[1:-1, 1:-1]))


def test_gauss_solve_against_library():
    rng = np.random.default_rng(2)
    for N in (1, 5, 40):
        A = rng.standard_normal((N, N)) + N * np.eye(N) * rng.random()
        b = rng.standard_normal(N)
        x = direct.gauss_solve(A, b)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
        assert np.allclose(x, scipy.linalg.solve(A, b), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("m,n,dx,dy", [(3, 3, 1.0, 1.0), (5, 4, 0.5, 0.3), (9, 9, 0.125, 0.125),
                                         (9, 6, 0.1, 0.37), (25, 17, 0.25, 0.25)])
def test_dense_vs_dst_vs_numpy(m, n, dx, dy):
    rng = np.random.default_rng(m * 100 + n)
    psi = W.random_boundary(m, n, rng)
    f = rng.standard_normal((n, m))
    a = direct.dense_solve(m, n, dx, dy, psi, f)
    b = direct.dst_solve(m, n, dx, dy, psi, f)
    c = direct.dense_solve(m, n, dx, dy, psi, f, solver=np.linalg.solve)
    scale = max(1.0, np.max(np.abs(a)))
    assert np.max(np.abs(a - b)) <= 1e-12 * scale
    assert np.max(np.abs(a - c)) <= 1e-12 * scale
    # the solution satisfies the discrete equations
    assert np.max(np.abs(grid.residual(a, f, dx, dy))) <= 1e-9 * scale * (1 / dx ** 2 + 1 / dy ** 2)


@pytest.mark.parametrize("kind", ["x2-y2", "xy", "x3-3xy2", "3x2y-y3", "x3"])
def test_direct_solvers_reproduce_manufactured(kind):
    p, exact = W.manufactured(kind, 25, 17, 0.25, 0.25)
    for solver in (direct.dense_solve, direct.dst_solve):
        u = solver(p.m, p.n, p.dx, p.dy, p.psi0, p.f)
        assert np.max(np.abs(u - exact)) <= 1e-10
    # dx != dy too
    p, exact = W.manufactured(kind, 9, 9, 0.3, 0.17)
    u = direct.dense_solve(p.m, p.n, p.dx, p.dy, p.psi0, p.f)
    assert np.max(np.abs(u - exact)) <= 1e-11


def test_chamber_maximum_principle_and_symmetry():
    p = W.chamber(psi_ab=100.0)
    u = direct.dense_solve(p.m, p.n, p.dx, p.dy, p.psi0, None)
    inner = u[1:-1, 1:-1]
    assert inner.min() > 0.0 and inner.max() < 100.0
    assert np.max(np.abs(u - u[:, ::-1])) <= 1e-12
    v = direct.dst_solve(p.m, p.n, p.dx, p.dy, p.psi0, None)
    assert np.max(np.abs(u - v)) <= 1e-11


def test_linearity_superposition():
    rng = np.random.default_rng(3)
    m, n, dx, dy = 13, 9, 0.2, 0.3
    g1, g2 = W.random_boundary(m, n, rng), W.random_boundary(m, n, rng)
    f1, f2 = rng.standard_normal((n, m)), rng.standard_normal((n, m))
    s = direct.dst_solve(m, n, dx, dy, g1 + g2, f1 + f2)
    s12 = direct.dst_solve(m, n, dx, dy, g1, f1) + direct.dst_solve(m, n, dx, dy, g2, f2)
    assert np.max(np.abs(s - s12)) <= 1e-12
