"""Oracle: point relaxation methods.

Paper passages: Jacobi (Eq. (5)), Gauss-Seidel (Eq. (6)), SOR applied to
Gauss-Seidel (Eq. (7)), all in the "Iterative Methods" section.

Every update is written with the same expression tree

    t_ij  = (cx (W + E) + cy (S + N) - f_ij) * inv_d        (point solution)
    psi_ij <- psi_ij + omega (t_ij - psi_ij)                 (relaxation)

With f = 0, t is Eq. (5)'s right-hand side (divide numerator and
denominator by cx; cy/cx = (dx/dy)^2 = beta^2), and psi + omega (t - psi)
is Eq. (7)'s (1 - w) psi + w t rearranged ("u" in Eq. (7) read as psi).

Red-black SOR is the GPU ordering, not the paper's: colour (i + j) mod 2 on
global indices, colour 0 first, then colour 1.  Within one colour no node
depends on another node of that colour, so updating a whole colour at once
equals updating its nodes one after another in any order.

Pins (tests/test_oracle_relax.py): fixed point of every method on discretely
harmonic fields; maximum principle for Jacobi/GS iterates; brute-force
per-node loop equals the vectorised red-black colour update bitwise; closed
form asymptotic rates rho_J, rho_GS = rho_J^2 and SOR at the Young optimum;
the paper's printed iteration counts for Jacobi and GS on the chamber.
"""
from __future__ import annotations

import numpy as np

from .grid import coefficients, colour_mask


def _zero_source(u, f):
    return np.zeros_like(u) if f is None else f.astype(u.dtype)


def point_solution(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
                   dtype=np.float64) -> np.ndarray:
    """t = (cx (W+E) + cy (S+N) - f) * inv_d at every interior node, computed
    from the current u (the Jacobi value of Eq. (5) with a source term)."""
    cx, cy, _, inv_d = coefficients(dx, dy, dtype)
    ff = _zero_source(u, f)
    t = u.copy()
    W = u[1:-1, :-2]
    E = u[1:-1, 2:]
    S = u[:-2, 1:-1]
    N = u[2:, 1:-1]
    t[1:-1, 1:-1] = ((cx * (W + E) + cy * (S + N)) - ff[1:-1, 1:-1]) * inv_d
    return t


def jacobi_sweep(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float) -> np.ndarray:
    """One Jacobi iteration (Eq. (5)): every interior node from the old
    values of its neighbours.  Returns the new array; u is not modified."""
    return point_solution(u, f, dx, dy)


def gs_lex_sweep(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
                 omega: float = 1.0) -> None:
    """One lexicographic Gauss-Seidel (omega = 1, Eq. (6)) or SOR (Eq. (7))
    sweep, in place.  Rows j = 1..n-2 ascending, in each row i = 1..m-2
    ascending, so the (i-1, j) and (i, j-1) neighbours are already new.
    Plain Python loops: this is the sequential method itself."""
    n, m = u.shape
    cx, cy, _, inv_d = (float(v) for v in coefficients(dx, dy))
    rows = u.tolist()
    frows = None if f is None else f.tolist()
    for j in range(1, n - 1):
        rm, r0, rp = rows[j - 1], rows[j], rows[j + 1]
        fr = None if frows is None else frows[j]
        for i in range(1, m - 1):
            fij = 0.0 if fr is None else fr[i]
            t = ((cx * (r0[i - 1] + r0[i + 1]) + cy * (rm[i] + rp[i])) - fij) * inv_d
            r0[i] = r0[i] + omega * (t - r0[i])
    u[:, :] = np.asarray(rows, dtype=np.float64)


def rb_sweep(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
             omega: float, dtype=np.float64) -> None:
    """One red-black SOR sweep, in place: all colour-0 interior nodes
    ((i + j) even) from the current values, then all colour-1 nodes from the
    just-updated colour-0 values.  dtype float32 emulates the FP32 smoother
    (u must then be float32; coefficients and omega rounded once)."""
    n, m = u.shape
    om = np.dtype(dtype).type(omega)
    for colour in (0, 1):
        mask = colour_mask(m, n, colour)
        t = point_solution(u, f, dx, dy, dtype)
        u[mask] = u[mask] + om * (t[mask] - u[mask])


def rb_sweep_loops(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
                   omega: float) -> None:
    """Brute-force red-black sweep: the same colour order, but node by node
    in Python loops.  Used only to pin rb_sweep on small grids."""
    n, m = u.shape
    cx, cy, _, inv_d = (float(v) for v in coefficients(dx, dy))
    for colour in (0, 1):
        new = u.copy()
        for j in range(1, n - 1):
            for i in range(1, m - 1):
                if (i + j) % 2 != colour:
                    continue
                fij = 0.0 if f is None else float(f[j, i])
                t = ((cx * (u[j, i - 1] + u[j, i + 1]) + cy * (u[j - 1, i] + u[j + 1, i])) - fij) * inv_d
                new[j, i] = u[j, i] + omega * (t - u[j, i])
        u[:, :] = new


def rate_jacobi(m: int, n: int, dx: float, dy: float) -> float:
    """Spectral radius of point Jacobi for the Dirichlet 5-point Laplacian:
    (cx cos(pi/(m-1)) + cy cos(pi/(n-1))) / (cx + cy)."""
    cx, cy = 1.0 / dx ** 2, 1.0 / dy ** 2
    return (cx * np.cos(np.pi / (m - 1)) + cy * np.cos(np.pi / (n - 1))) / (cx + cy)


def omega_opt(rho_j: float) -> float:
    """Young's optimal SOR factor 2 / (1 + sqrt(1 - rho_J^2)) for a
    consistently ordered matrix (lexicographic and red-black both are)."""
    return 2.0 / (1.0 + np.sqrt(1.0 - rho_j * rho_j))
