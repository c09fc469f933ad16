"""Pins for oracle.lines (Thomas algorithm, SLORA, SLORB, ADI): library
banded solves, brute-force line-by-line ordering, closed-form line rates and
the SLOR/SLORB/ADI iteration counts the paper prints for the chamber."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import lines, solve, direct


def test_thomas_against_solve_banded():
    rng = np.random.default_rng(0)
    for K in (1, 2, 7, 64):
        a = rng.uniform(-1, 1, K)
        c = rng.uniform(-1, 1, K)
        b = np.abs(a) + np.abs(c) + rng.uniform(0.1, 2, K)
        r = rng.standard_normal(K)
        x = lines.thomas(a, b, c, r)
        ab = np.zeros((3, K))
        ab[0, 1:] = c[:-1]
        ab[1, :] = b
        ab[2, :-1] = a[1:]
        y = scipy.linalg.solve_banded((1, 1), ab, r)
        assert np.max(np.abs(x - y)) <= 1e-13 * max(1, np.max(np.abs(y)))
        # residual of the tridiagonal equations
        T = np.diag(b) + np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        assert np.max(np.abs(T @ x - r)) <= 1e-14 * 10 * np.max(np.abs(r)) * K


def test_thomas_rejects_non_dominant():
    with pytest.raises(ValueError):
        lines.thomas(-1.0, 1.5, -1.0, np.ones(5))


def test_thomas_many_equals_thomas():
    rng = np.random.default_rng(1)
    R = rng.standard_normal((23, 6))
    X = lines.thomas_many(-16.0, 64.0, -16.0, R)
    for l in range(6):
        assert np.array_equal(X[:, l], lines.thomas(-16.0, 64.0, -16.0, R[:, l]))


@pytest.mark.parametrize("form", ["A", "B"])
def test_zebra_group_equals_one_line_at_a_time(form):
    rng = np.random.default_rng(2)
    m, n, dx, dy = 12, 9, 0.2, 0.13
    psi = W.random_boundary(m, n, rng)
    psi[1:-1, 1:-1] = rng.random((n - 2, m - 2))
    f = rng.standard_normal((n, m))
    a = psi.copy()
    lines.adi_zebra_iteration(a, f, dx, dy, 1.2, form)
    b = psi.copy()
    for j in list(range(1, n - 1, 2)) + list(range(2, n - 1, 2)):
        lines.update_rows(b, f, [j], dx, dy, 1.2, form)
    for i in list(range(1, m - 1, 2)) + list(range(2, m - 1, 2)):
        lines.update_cols(b, f, [i], dx, dy, 1.2, form)
    assert np.array_equal(a, b)


def test_row_solution_satisfies_line_equations():
    """After a row update with w = 1 the 5-point equation holds exactly on that
    row given the (unchanged) neighbouring rows."""
    rng = np.random.default_rng(3)
    m, n, dx, dy = 10, 7, 0.3, 0.2
    psi = W.random_boundary(m, n, rng)
    psi[1:-1, 1:-1] = rng.random((n - 2, m - 2))
    f = rng.standard_normal((n, m))
    from oracle import grid
    for form in ("A", "B"):
        u = psi.copy()
        lines.update_rows(u, f, [3], dx, dy, 1.0, form)
        r = grid.residual(u, f, dx, dy)
        assert np.max(np.abs(r[3, 1:-1])) < 1e-10
        u = psi.copy()
        lines.update_cols(u, f, [4], dx, dy, 1.0, form)
        r = grid.residual(u, f, dx, dy)
        assert np.max(np.abs(r[1:-1, 4])) < 1e-10


@pytest.mark.parametrize("method", ["slora", "slorb", "adi_lex_a", "adi_lex_b", "adi_zebra_a", "adi_zebra_b"])
def test_line_methods_converge_to_exact(method):
    rng = np.random.default_rng(4)
    m, n, dx, dy = 13, 9, 0.1, 0.15
    psi = W.random_boundary(m, n, rng)
    f = rng.standard_normal((n, m))
    ex = direct.dense_solve(m, n, dx, dy, psi, f)
    u, k, h = solve.iterate(method, psi, f, dx, dy, 1.1, "delta", 1e-14, max_iter=5000)
    assert np.max(np.abs(u - ex)) <= 1e-10 * max(1, np.max(np.abs(ex)))


def test_line_gs_rate_closed_form():
    p = W.chamber(psi_ab=1.0)
    rho = lines.rate_line_jacobi_x(p.m, p.n, p.dx, p.dy) ** 2
    _, _, h = solve.iterate("slora", p.psi0, None, p.dx, p.dy, 1.0, "delta", 1e-13)
    h = np.asarray(h[-40:])
    ratio = float(np.exp(np.mean(np.log(h[1:] / h[:-1]))))
    assert ratio == pytest.approx(rho, rel=0.01)


def test_paper_counts_slor_w1(paper):
    """Figure 11 text: SLORA = SLORB = 326 iterations at w = 1 (both forms are
    line Gauss-Seidel there)."""
    p = W.chamber(psi_ab=1.0)
    tol = paper["stop"]["tol_delta"]
    _, ka, _ = solve.iterate("slora", p.psi0, None, p.dx, p.dy, 1.0, "delta", tol)
    _, kb, _ = solve.iterate("slorb", p.psi0, None, p.dx, p.dy, 1.0, "delta", tol)
    assert ka == kb
    assert ka == pytest.approx(paper["iterations_no_relaxation"]["slora"], rel=0.025)


def test_paper_counts_at_optimal_omega(paper):
    """Figure 15 text: ADI 33 iterations at w = 1.3, SLORB 55 at w = 1.25
    (ADI in the paper's order, rows then columns, relaxation inside the line
    system).  Reproduced exactly."""
    p = W.chamber(psi_ab=1.0)
    tol = paper["stop"]["tol_delta"]
    _, kb, _ = solve.iterate("slorb", p.psi0, None, p.dx, p.dy, paper["omega_opt"]["slorb"], "delta", tol)
    _, kadi, _ = solve.iterate("adi_lex_b", p.psi0, None, p.dx, p.dy, paper["omega_opt"]["adi"], "delta", tol)
    assert kb == paper["iterations_at_opt"]["slorb"]
    assert kadi == paper["iterations_at_opt"]["adi"]


@pytest.mark.slow
def test_paper_optimal_omega_slorb_and_adi(paper):
    """Figure 13 text: optimum w = 1.25 (SLORB) and 1.3 (ADI) among the
    convergent w of the 0.05 grid."""
    p = W.chamber(psi_ab=1.0)
    for method, key in (("slorb", "slorb"), ("adi_lex_b", "adi")):
        counts = {}
        for w in np.round(np.arange(1.0, 1.41, 0.05), 2):
            _, k, h = solve.iterate(method, p.psi0, None, p.dx, p.dy, float(w), "delta", 1e-9, max_iter=2000)
            if not solve.diverged(h) and k < 2000:
                counts[float(w)] = k
        best = min(counts, key=lambda w: (counts[w], w))
        assert best == paper["omega_opt"][key]


def _young_line_sor_rate(mu: float, w: float) -> float:
    """Spectral radius of SOR for a consistently ordered block matrix whose
    block Jacobi radius is mu (Young's theorem): below the optimum
    w_opt = 2 / (1 + sqrt(1 - mu^2)) it is ((w mu + sqrt(w^2 mu^2 - 4(w-1))) / 2)^2,
    from the optimum on it is w - 1."""
    w_opt = 2.0 / (1.0 + np.sqrt(1.0 - mu * mu))
    if w >= w_opt:
        return w - 1.0
    return ((w * mu + np.sqrt(w * w * mu * mu - 4.0 * (w - 1.0))) / 2.0) ** 2


def _rows_zebra_history(p, w, tol=1e-13, max_iter=3000):
    """delta history of repeated zebra row halves (odd rows, then even rows,
    relaxation after the line solve): x-line SOR in red-black line order."""
    u = p.psi0.copy()
    hist = []
    for _ in range(max_iter):
        old = u.copy()
        lines.adi_zebra_rows_half(u, None, p.dx, p.dy, w, "A")
        hist.append(float(np.max(np.abs(u - old))))
        if hist[-1] < tol:
            break
    return hist


@pytest.mark.parametrize("order", ["rows_ascending", "rows_zebra"])
@pytest.mark.parametrize("w,rel", [(1.3, 0.002), (1.5, 0.002), (1.8, 0.01), ("opt", 0.05)])
def test_relax_after_line_sor_rate_young(order, w, rel):
    """Relaxation after the line solve (SLORA, Eqs. (8)-(9); the zebra ADI
    default) at w != 1.  x-line SOR is block SOR on a block tridiagonal
    matrix, consistently ordered for ascending rows and for odd-then-even
    rows alike, so its asymptotic rate follows Young's formula with the
    x-line Jacobi radius; at the block optimum w_opt = 1.6220 (chamber) it is
    w - 1 up to the Jordan-block transient.  A misplaced relaxation (e.g.
    dividing by w, or relaxing toward the old row with the wrong sign) keeps
    the fixed point but changes this rate."""
    p = W.chamber(psi_ab=1.0)
    mu = lines.rate_line_jacobi_x(p.m, p.n, p.dx, p.dy)
    w_opt = 2.0 / (1.0 + np.sqrt(1.0 - mu * mu))
    assert w_opt == pytest.approx(1.6220, abs=1e-4)
    w = w_opt if w == "opt" else w
    if order == "rows_ascending":
        _, _, h = solve.iterate("slora", p.psi0, None, p.dx, p.dy, w, "delta", 1e-13, max_iter=5000)
    else:
        h = _rows_zebra_history(p, w)
    h = np.asarray(h[-40:])
    ratio = float(np.exp(np.mean(np.log(h[1:] / h[:-1]))))
    assert ratio == pytest.approx(_young_line_sor_rate(mu, w), rel=rel)
