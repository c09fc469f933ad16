"""Oracle: the 5-point operator, the residual and the norms.

Paper passages: the five-point formula (Eq. (2)); the linear operator L of the
multigrid section (Eq. (11)); the residual R = L(psi) (Eq. (12)); the
infinity-norm update error used as the stopping rule (Eq. (16)).

Reading: Eq. (2) and Eq. (11) print dx^2 under the y second difference; the
Jacobi formula (Eq. (5)) with beta = dx/dy only follows from dy^2 there, so
L_h uses 1/dy^2 for the y term.  With dx = dy (the paper's chamber) the two
forms coincide.

Sign convention: the discrete problem is L_h psi = f (f = 0 is Laplace);
the residual is r = f - L_h psi, so L_h e = r for the error e.  The paper's
R = L(psi) with L(dpsi) = -R is the same algebra with f = 0 (Eqs. (12)-(15)).

Pins (tests/test_oracle_grid.py): discretely harmonic polynomials give
L_h psi = 0 to rounding for dx != dy (fails for the dx^2-only form);
L_h(x^3) = 6x; symmetric negative-definite check of -L_h against a dense
assembly; norms against numpy.linalg.norm.
"""
from __future__ import annotations

import numpy as np


def coefficients(dx: float, dy: float, dtype=np.float64):
    """(cx, cy, d, inv_d) with cx = 1/dx^2, cy = 1/dy^2, d = 2(cx+cy), inv_d = 1/d.

    All four are formed in FP64 and then rounded once to `dtype`, so an FP32
    computation uses the correctly rounded FP64 coefficients."""
    cx = 1.0 / (dx * dx)
    cy = 1.0 / (dy * dy)
    d = 2.0 * (cx + cy)
    inv_d = 1.0 / d
    t = np.dtype(dtype).type
    return t(cx), t(cy), t(d), t(inv_d)


def apply_L(u: np.ndarray, dx: float, dy: float, dtype=np.float64) -> np.ndarray:
    """L_h u at the interior nodes (zero on the perimeter):

        (L_h u)_ij = cx (u_{i-1,j} + u_{i+1,j}) + cy (u_{i,j-1} + u_{i,j+1}) - d u_ij

    which is Eq. (2)/(11) multiplied out.  u has shape (n, m) indexed [j, i]."""
    cx, cy, d, _ = coefficients(dx, dy, dtype)
    out = np.zeros_like(u)
    W = u[1:-1, :-2]
    E = u[1:-1, 2:]
    S = u[:-2, 1:-1]
    N = u[2:, 1:-1]
    C = u[1:-1, 1:-1]
    out[1:-1, 1:-1] = (cx * (W + E) + cy * (S + N)) - d * C
    return out


def residual(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
             dtype=np.float64) -> np.ndarray:
    """r = f - L_h u on the interior, 0 on the perimeter (Eq. (12) with a
    source term and the sign convention of the module header)."""
    Lu = apply_L(u, dx, dy, dtype)
    r = -Lu
    if f is not None:
        r[1:-1, 1:-1] = f[1:-1, 1:-1].astype(u.dtype) - Lu[1:-1, 1:-1]
    return r


def residual_diff(u: np.ndarray, f: np.ndarray | None, dx: float, dy: float,
                  dtype=np.float64) -> np.ndarray:
    """The same residual with L_h in difference form,
        cx ((u_{i-1,j} - u_ij) + (u_{i+1,j} - u_ij)) + cy ((u_{i,j-1} - u_ij) + (u_{i,j+1} - u_ij)),
    algebraically equal to apply_L (d = 2 (cx + cy)).  In floating point the
    neighbour differences are formed first, so for a smooth u of large values
    the result keeps the accuracy of the second differences instead of that
    of terms of size 8|u|/h^2."""
    cx, cy, _, _ = coefficients(dx, dy, dtype)
    W = u[1:-1, :-2]
    E = u[1:-1, 2:]
    S = u[:-2, 1:-1]
    N = u[2:, 1:-1]
    C = u[1:-1, 1:-1]
    Lu = cx * ((W - C) + (E - C)) + cy * ((S - C) + (N - C))
    r = np.zeros_like(u)
    r[1:-1, 1:-1] = -Lu if f is None else f[1:-1, 1:-1].astype(u.dtype) - Lu
    return r


def interior(a: np.ndarray) -> np.ndarray:
    return a[1:-1, 1:-1]


def norm2(r: np.ndarray) -> float:
    """Unweighted Euclidean norm over the interior nodes."""
    v = interior(r).astype(np.float64)
    return float(np.sqrt(np.sum(v * v)))


def norm_inf(r: np.ndarray) -> float:
    """Max-abs over the interior nodes."""
    v = interior(r)
    return float(np.max(np.abs(v))) if v.size else 0.0


def update_delta(new: np.ndarray, old: np.ndarray) -> float:
    """The paper's iteration error max|psi^{k+1} - psi^k| (Eq. (16))."""
    return float(np.max(np.abs(new.astype(np.float64) - old.astype(np.float64))))


def colour_mask(m: int, n: int, colour: int) -> np.ndarray:
    """Boolean (n, m) mask of the interior nodes with (i + j) mod 2 == colour."""
    j, i = np.mgrid[0:n, 0:m]
    mask = ((i + j) % 2) == colour
    mask[0, :] = False
    mask[-1, :] = False
    mask[:, 0] = False
    mask[:, -1] = False
    return mask
