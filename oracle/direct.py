"""Oracle: exact solutions of the discrete problem.

Paper passage: the direct methods named in the Introduction (Cramer's rule,
Gauss elimination, the Thomas algorithm).  Every iterative method of the
paper converges to the unique solution of the linear system L_h psi = f on
the interior with psi = g on the perimeter; this module computes that
solution without iterating, two independent ways:

* dense Gaussian elimination with partial pivoting on the assembled system
  (own code; small grids only), and
* the DST-I spectral solve: sin(p pi i/(m-1)) sin(q pi j/(n-1)) are the
  eigenvectors of the Dirichlet 5-point operator on any rectangle, with
  eigenvalues -2cx(1 - cos(p pi/(m-1))) - 2cy(1 - cos(q pi/(n-1))); the
  transform itself is scipy.fft.dstn (a library routine sharing nothing with
  the iterative code).

Pins (tests/test_oracle_grid.py): dense GE against numpy.linalg.solve;
dense GE against DST on rectangles with dx != dy; both reproduce the
discretely harmonic fields exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .grid import coefficients


def assemble(m: int, n: int, dx: float, dy: float, psi_b: np.ndarray,
             f: np.ndarray | None):
    """The SPD system A x = rhs for the (m-2)(n-2) interior unknowns,
    A = -L_h restricted to the interior, numbered k = (j-1)(m-2) + (i-1).
    Boundary values from psi_b's perimeter are moved to the right-hand side:
        d x_ij - sum_{interior nbrs} c x_nbr = -f_ij + sum_{boundary nbrs} c g."""
    cx, cy, d, _ = (float(v) for v in coefficients(dx, dy))
    mi, ni = m - 2, n - 2
    N = mi * ni
    A = np.zeros((N, N))
    rhs = np.zeros(N)
    for j in range(1, n - 1):
        for i in range(1, m - 1):
            k = (j - 1) * mi + (i - 1)
            A[k, k] = d
            rhs[k] = -(0.0 if f is None else float(f[j, i]))
            for (ii, jj, c) in ((i - 1, j, cx), (i + 1, j, cx), (i, j - 1, cy), (i, j + 1, cy)):
                if 1 <= ii <= m - 2 and 1 <= jj <= n - 2:
                    A[k, (jj - 1) * mi + (ii - 1)] = -c
                else:
                    rhs[k] += c * float(psi_b[jj, ii])
    return A, rhs


def gauss_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Gaussian elimination with partial pivoting, then back substitution.
    Each elimination step is one row pivot search and a rank-one update of
    the trailing block."""
    A = np.array(A, dtype=np.float64)
    b = np.array(b, dtype=np.float64)
    N = A.shape[0]
    for k in range(N):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if A[p, k] == 0.0:
            raise ValueError("singular matrix")
        if p != k:
            A[[k, p]] = A[[p, k]]
            b[[k, p]] = b[[p, k]]
        l = A[k + 1:, k] / A[k, k]
        A[k + 1:, k:] -= np.outer(l, A[k, k:])
        b[k + 1:] -= l * b[k]
    x = np.zeros(N)
    for k in range(N - 1, -1, -1):
        x[k] = (b[k] - A[k, k + 1:] @ x[k + 1:]) / A[k, k]
    return x


def dense_solve(m: int, n: int, dx: float, dy: float, psi_b: np.ndarray,
                f: np.ndarray | None, solver=gauss_solve) -> np.ndarray:
    """Exact discrete solution on the full (n, m) array (perimeter copied
    from psi_b) by assembling the system and eliminating."""
    A, rhs = assemble(m, n, dx, dy, psi_b, f)
    x = solver(A, rhs)
    out = np.array(psi_b, dtype=np.float64, copy=True)
    out[1:-1, 1:-1] = x.reshape(n - 2, m - 2)
    return out


def dst_solve(m: int, n: int, dx: float, dy: float, psi_b: np.ndarray,
              f: np.ndarray | None) -> np.ndarray:
    """Exact discrete solution by diagonalising the Dirichlet 5-point
    operator with the type-I sine transform in x and y."""
    cx, cy, _, _ = (float(v) for v in coefficients(dx, dy))
    mi, ni = m - 2, n - 2
    # right-hand side of L_h x = b on the interior with the boundary lifted
    b = np.zeros((ni, mi)) if f is None else np.array(f[1:-1, 1:-1], dtype=np.float64)
    b[:, 0] -= cx * psi_b[1:-1, 0]
    b[:, -1] -= cx * psi_b[1:-1, m - 1]
    b[0, :] -= cy * psi_b[0, 1:-1]
    b[-1, :] -= cy * psi_b[n - 1, 1:-1]
    p = np.arange(1, mi + 1)
    q = np.arange(1, ni + 1)
    lam = (-2.0 * cx * (1.0 - np.cos(p * np.pi / (m - 1)))[None, :]
           - 2.0 * cy * (1.0 - np.cos(q * np.pi / (n - 1)))[:, None])
    bh = scipy.fft.dstn(b, type=1, norm="ortho")
    x = scipy.fft.idstn(bh / lam, type=1, norm="ortho")
    out = np.array(psi_b, dtype=np.float64, copy=True)
    out[1:-1, 1:-1] = x
    return out
