"""Oracle: iteration drivers and stopping rules.

Paper passage: the solver iterates until the infinity-norm error
max|psi^{k+1} - psi^k| (Eq. (16)) falls below 1e-9.  Besides that rule
('delta'), two residual-based rules are offered: the max-abs residual
('res_inf', physical units of Eq. (11)) and the relative Euclidean residual
||r_k||_2 / ||r_0||_2 over the interior with r_0 taken at the start
('rel_l2').  Each driver returns the final field, the number of iterations
(cycles for multigrid, outer steps for the mixed loop) and the history of
the monitored quantity.
"""
from __future__ import annotations

import numpy as np

from . import relax, lines, multigrid
from .grid import residual, norm2, norm_inf, update_delta

POINT = ("jacobi", "gs_lex", "sor_lex", "rb")
DIVERGED = 1e30
LINE = ("slora", "slorb", "adi_lex_a", "adi_lex_b", "adi_zebra_a", "adi_zebra_b")


def _one_iteration(method, u, f, dx, dy, omega):
    if method == "jacobi":
        u[:, :] = relax.jacobi_sweep(u, f, dx, dy)
    elif method == "gs_lex":
        relax.gs_lex_sweep(u, f, dx, dy, 1.0)
    elif method == "sor_lex":
        relax.gs_lex_sweep(u, f, dx, dy, omega)
    elif method == "rb":
        relax.rb_sweep(u, f, dx, dy, omega)
    elif method == "slora":
        lines.slor_sweep(u, f, dx, dy, omega, "A")
    elif method == "slorb":
        lines.slor_sweep(u, f, dx, dy, omega, "B")
    elif method == "adi_lex_a":
        lines.adi_lex_iteration(u, f, dx, dy, omega, "A")
    elif method == "adi_lex_b":
        lines.adi_lex_iteration(u, f, dx, dy, omega, "B")
    elif method == "adi_zebra_a":
        lines.adi_zebra_iteration(u, f, dx, dy, omega, "A")
    elif method == "adi_zebra_b":
        lines.adi_zebra_iteration(u, f, dx, dy, omega, "B")
    else:
        raise ValueError(method)


def iterate(method: str, psi0: np.ndarray, f, dx: float, dy: float, omega: float = 1.0,
            stop: str = "delta", tol: float = 1e-9, max_iter: int = 100000):
    """Run a point or line method until the stopping rule holds.

    Returns (u, iterations, history); history[k] is the monitored quantity
    after iteration k+1."""
    u = np.array(psi0, dtype=np.float64, copy=True)
    r0 = norm2(residual(u, f, dx, dy)) if stop == "rel_l2" else None
    hist = []
    for k in range(1, max_iter + 1):
        old = u.copy() if stop == "delta" else None
        _one_iteration(method, u, f, dx, dy, omega)
        if stop == "delta":
            q = update_delta(u, old)
        elif stop == "res_inf":
            q = norm_inf(residual(u, f, dx, dy))
        elif stop == "rel_l2":
            q = norm2(residual(u, f, dx, dy)) / r0 if r0 > 0 else 0.0
        else:
            raise ValueError(stop)
        hist.append(q)
        if not np.isfinite(q) or q > DIVERGED:
            return u, k, hist
        if q < tol:
            return u, k, hist
    return u, max_iter, hist


def diverged(hist) -> bool:
    """True when the monitored quantity became non-finite or exceeded DIVERGED."""
    return bool(hist) and (not np.isfinite(hist[-1]) or hist[-1] > DIVERGED)


def mg_solve(psi0: np.ndarray, f, dx: float, dy: float, tol: float = 1e-10, max_cycles: int = 100,
             nu1: int = 2, nu2: int = 2, omega_s: float = 1.0, max_levels: int = 64,
             stop: str = "rel_l2", smoother: str = "rb"):
    """Repeat V-cycles until the stopping rule holds (rel_l2, res_inf or delta)."""
    n, m = psi0.shape
    levels = multigrid.hierarchy(m, n, dx, dy, max_levels)
    u = np.array(psi0, dtype=np.float64, copy=True)
    r0 = norm2(residual(u, f, dx, dy))
    hist = []
    for k in range(1, max_cycles + 1):
        old = u.copy() if stop == "delta" else None
        multigrid.vcycle(levels, 0, u, f, nu1, nu2, omega_s, np.float64, smoother)
        if stop == "delta":
            q = update_delta(u, old)
        elif stop == "res_inf":
            q = norm_inf(residual(u, f, dx, dy))
        else:
            q = norm2(residual(u, f, dx, dy)) / r0 if r0 > 0 else 0.0
        hist.append(q)
        if not np.isfinite(q) or q < tol:
            return u, k, hist
    return u, max_cycles, hist


# Safety factor of the one-cycle prediction below (a cycle's factor grows
# slowly as the FP32 rounding floor nears, about 10-15% between steps).
ONE_CYCLE_MARGIN = 1.5


def one_cycle_suffices(q: float, q_prev: float, ran: int, tol: float) -> bool:
    """Whether the step that opens with test value q (the one before it q_prev,
    after a step of `ran` FP32 cycles) takes one cycle instead of `inner`:
    with the per-cycle factor rho = (q / q_prev)^(1 / ran) measured on that
    step, one cycle is predicted to pass the test, 1.5 q rho < tol.  Written
    as q / q_prev < (tol / (1.5 q))^ran, with the power taken by repeated
    multiplication (no root)."""
    x = tol / (ONE_CYCLE_MARGIN * q)
    p = 1.0
    for _ in range(ran):
        p *= x
    return q / q_prev < p


def mixed_solve(psi0: np.ndarray, f, dx: float, dy: float, tol: float = 1e-10, max_steps: int = 100,
                nu1: int = 2, nu2: int = 2, omega_s: float = 1.0, max_levels: int = 64, smoother: str = "rb",
                inner: int = 1, schedule: list | None = None):
    """Mixed-precision defect correction until ||r||_2/||r_0||_2 < tol (the
    test is taken on the FP64 residual before each step).  With inner > 1 a
    step runs `inner` FP32 V-cycles, or one where one_cycle_suffices() holds
    for its test and the two before it (not for the first step); the cycles
    each step ran are appended to `schedule` if given."""
    n, m = psi0.shape
    levels = multigrid.hierarchy(m, n, dx, dy, max_levels)
    u = np.array(psi0, dtype=np.float64, copy=True)
    r0 = norm2(residual(u, f, dx, dy))
    hist = []
    q_prev, ran = None, 0
    for k in range(0, max_steps + 1):
        q = norm2(residual(u, f, dx, dy)) / r0 if r0 > 0 else 0.0
        if k > 0:
            hist.append(q)
        if not np.isfinite(q) or q < tol or k == max_steps:
            return u, k, hist
        c = inner
        if inner > 1 and q_prev is not None and one_cycle_suffices(q, q_prev, ran, tol):
            c = 1
        multigrid.mixed_step(u, f, levels, nu1, nu2, omega_s, smoother, c)
        if schedule is not None:
            schedule.append(c)
        q_prev, ran = q, c
    return u, max_steps, hist
