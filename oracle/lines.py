"""Oracle: line relaxation (SLOR), ADI and the Thomas algorithm.

Paper passages: the Thomas algorithm for tridiagonal systems (Introduction,
direct methods; SLOR section); SLOR by rows with relaxation after the line
solve, SLORA (Eqs. (8)-(9)); relaxation inside the line system, SLORB
(Eq. (10)); ADI = a sweep by rows followed by a sweep by columns (ADI section).

Readings:
* Eq. (8): the missing parenthesis closes after psi^{k+1}_{i,j-1}; rows are
  visited j ascending, so row j-1 is already new and row j+1 is old; the
  unrelaxed line solution psi^{k'+1} is called psi~ here.
* Eq. (10) prints the tridiagonal coefficients swapped; the system used is
  -w cx psi_{i-1} + d psi_i - w cx psi_{i+1}
        = (1-w) d psi^k_ij + w [cy (psi^k_{i,j+1} + psi^{k+1}_{i,j-1}) - f_ij],
  i.e. point SOR written for a whole row (Eq. (10) times cx, with the two
  coefficients exchanged; only this form has the 5-point equation as its
  fixed point).  It is diagonally dominant only for w < 1 + beta^2.
* The column half of ADI mirrors the row half (x and y exchanged).
* "ADI-zebra" is the GPU ordering: in the row half all odd rows j are solved
  from the current neighbours, then all even rows; in the column half odd
  columns, then even columns.  Lines of one parity share no unknowns and
  read only lines of the other parity, so solving them together equals
  solving them one after another.

Pins (tests/test_oracle_lines.py): Thomas against scipy.linalg.solve_banded
and against its own residual; every line method leaves a discretely harmonic
field unchanged; closed-form asymptotic rate of line Gauss-Seidel; the rate
of relaxation after the line solve (form 'A', ascending and zebra rows) at
w = 1.3, 1.5, 1.8 and the block optimum against Young's formula; converged
solutions against the dense direct solve; the paper's printed iteration count
for SLOR at w = 1 on the chamber; the paper's ADI and SLORB counts at their
optimal w (33 at 1.3, 55 at 1.25), reproduced exactly with the relaxation
inside the line system (the ADI placement the paper does not print; the
placement after the solve does not reproduce 33).
"""
from __future__ import annotations

import numpy as np

from .grid import coefficients


# --------------------------------------------------------------------------
# Thomas algorithm
# --------------------------------------------------------------------------
def thomas(a, b, c, r):
    """Solve a_k x_{k-1} + b_k x_k + c_k x_{k+1} = r_k, k = 0..K-1 (a_0 and
    c_{K-1} unused) by Gaussian elimination without pivoting specialised to
    the tridiagonal band: forward sweep c'_k, r'_k, then back substitution.
    Scalars broadcast.  Raises ValueError if a row is not diagonally dominant
    (|b| <= |a| + |c|), where the method may break down."""
    r = [float(v) for v in r]
    K = len(r)
    a = [float(a)] * K if np.isscalar(a) else [float(v) for v in a]
    b = [float(b)] * K if np.isscalar(b) else [float(v) for v in b]
    c = [float(c)] * K if np.isscalar(c) else [float(v) for v in c]
    for k in range(K):
        off = (abs(a[k]) if k > 0 else 0.0) + (abs(c[k]) if k < K - 1 else 0.0)
        if K > 1 and abs(b[k]) <= off:
            raise ValueError("tridiagonal system not diagonally dominant")
    cp = [0.0] * K
    rp = [0.0] * K
    cp[0] = c[0] / b[0]
    rp[0] = r[0] / b[0]
    for k in range(1, K):
        piv = b[k] - a[k] * cp[k - 1]
        cp[k] = c[k] / piv
        rp[k] = (r[k] - a[k] * rp[k - 1]) / piv
    x = [0.0] * K
    x[K - 1] = rp[K - 1]
    for k in range(K - 2, -1, -1):
        x[k] = rp[k] - cp[k] * x[k + 1]
    return np.asarray(x)


def thomas_many(a: float, b: float, c: float, R: np.ndarray) -> np.ndarray:
    """The same recurrences for many independent systems with constant
    coefficients: R has shape (K, L), one system per column; the loop runs
    along k with numpy operations across the L systems.  The arithmetic is
    done in R's precision (float32 R: coefficients rounded to float32 and
    every operation rounded to float32, as in the mixed inner cycle)."""
    K = R.shape[0]
    if K > 1 and abs(b) <= abs(a) + abs(c):
        raise ValueError("tridiagonal system not diagonally dominant")
    dt = R.dtype.type
    a, b, c = dt(a), dt(b), dt(c)
    cp = np.zeros(K, dtype=R.dtype)
    rp = np.zeros_like(R)
    cp[0] = c / b
    rp[0] = R[0] / b
    for k in range(1, K):
        piv = b - a * cp[k - 1]
        cp[k] = c / piv
        rp[k] = (R[k] - a * rp[k - 1]) / piv
    X = np.zeros_like(R)
    X[K - 1] = rp[K - 1]
    for k in range(K - 2, -1, -1):
        X[k] = rp[k] - cp[k] * X[k + 1]
    return X


# --------------------------------------------------------------------------
# Line updates
# --------------------------------------------------------------------------
def _src(u, f):
    return np.zeros_like(u) if f is None else f


def update_rows(u: np.ndarray, f: np.ndarray | None, rows, dx: float, dy: float,
                omega: float, form: str) -> None:
    """Solve the row systems of the listed interior rows j (which must share
    no neighbours, or be a single row) from the current u, in place.

    form 'A' (SLORA, Eqs. (8)-(9)): solve
        -cx t_{i-1} + d t_i - cx t_{i+1} = cy (u_{i,j-1} + u_{i,j+1}) - f_ij
    with t = u on the row ends, then u_row <- u_row + w (t - u_row).
    form 'B' (SLORB, Eq. (10) as read in the header): solve
        -w cx t_{i-1} + d t_i - w cx t_{i+1}
            = (1-w) d u_ij + w (cy (u_{i,j-1} + u_{i,j+1}) - f_ij)
    and store t."""
    n, m = u.shape
    cx, cy, d, _ = (float(v) for v in coefficients(dx, dy))
    ff = _src(u, f)
    rows = np.asarray(list(rows), dtype=np.int64)
    if rows.size == 0:
        return
    # right-hand sides, one system per listed row: shape (K = m-2, L)
    S = u[rows - 1, 1:m - 1]
    N = u[rows + 1, 1:m - 1]
    base = (cy * (S + N) - ff[rows, 1:m - 1])
    if form == "A":
        R = base.copy()
        R[:, 0] = R[:, 0] + cx * u[rows, 0]
        R[:, -1] = R[:, -1] + cx * u[rows, m - 1]
        T = thomas_many(-cx, d, -cx, R.T).T
        old = u[rows, 1:m - 1]
        u[rows, 1:m - 1] = old + omega * (T - old)
    elif form == "B":
        R = (1.0 - omega) * d * u[rows, 1:m - 1] + omega * base
        R[:, 0] = R[:, 0] + omega * cx * u[rows, 0]
        R[:, -1] = R[:, -1] + omega * cx * u[rows, m - 1]
        T = thomas_many(-omega * cx, d, -omega * cx, R.T).T
        u[rows, 1:m - 1] = T
    else:
        raise ValueError(form)


def update_cols(u: np.ndarray, f: np.ndarray | None, cols, dx: float, dy: float,
                omega: float, form: str) -> None:
    """The column mirror of update_rows: unknowns j = 1..n-2 of each listed
    interior column i, coupling -cy along the column, cx (u_{i-1,j} +
    u_{i+1,j}) on the right-hand side."""
    ut = u.T.copy()
    ft = None if f is None else f.T.copy()
    update_rows(ut, ft, cols, dy, dx, omega, form)
    u[:, :] = ut.T


def slor_sweep(u, f, dx, dy, omega, form="A"):
    """One SLOR iteration by rows, j = 1..n-2 ascending, one row at a time
    (SLORA: form 'A', Eqs. (8)-(9); SLORB: form 'B', Eq. (10))."""
    n = u.shape[0]
    for j in range(1, n - 1):
        update_rows(u, f, [j], dx, dy, omega, form)


def adi_lex_iteration(u, f, dx, dy, omega, form="B"):
    """One ADI iteration in the paper's ordering: a row sweep (j ascending)
    followed by a column sweep (i ascending)."""
    n, m = u.shape
    for j in range(1, n - 1):
        update_rows(u, f, [j], dx, dy, omega, form)
    for i in range(1, m - 1):
        update_cols(u, f, [i], dx, dy, omega, form)


def adi_zebra_iteration(u, f, dx, dy, omega, form="A"):
    """One ADI iteration in zebra order (the GPU ordering): odd rows, even
    rows, odd columns, even columns; each group solved together."""
    n, m = u.shape
    update_rows(u, f, range(1, n - 1, 2), dx, dy, omega, form)
    update_rows(u, f, range(2, n - 1, 2), dx, dy, omega, form)
    update_cols(u, f, range(1, m - 1, 2), dx, dy, omega, form)
    update_cols(u, f, range(2, m - 1, 2), dx, dy, omega, form)


def adi_zebra_rows_half(u, f, dx, dy, omega, form="A"):
    """The row half of adi_zebra_iteration alone (odd rows, then even rows)."""
    n = u.shape[0]
    update_rows(u, f, range(1, n - 1, 2), dx, dy, omega, form)
    update_rows(u, f, range(2, n - 1, 2), dx, dy, omega, form)


def adi_zebra_cols_half(u, f, dx, dy, omega, form="A"):
    """The column half of adi_zebra_iteration alone (odd, then even columns)."""
    m = u.shape[1]
    update_cols(u, f, range(1, m - 1, 2), dx, dy, omega, form)
    update_cols(u, f, range(2, m - 1, 2), dx, dy, omega, form)


def rate_line_jacobi_x(m: int, n: int, dx: float, dy: float) -> float:
    """Spectral radius of x-line Jacobi for the Dirichlet 5-point Laplacian:
    cy cos(pi/(n-1)) / (cx + cy - cx cos(pi/(m-1))).  Line Gauss-Seidel by
    rows converges at the square of it."""
    cx, cy = 1.0 / dx ** 2, 1.0 / dy ** 2
    return cy * np.cos(np.pi / (n - 1)) / (cx + cy - cx * np.cos(np.pi / (m - 1)))
