"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only *builds inputs*: grid sizes, spacings, Dirichlet boundary
values, source terms, request streams.  It holds none of the solvers'
arithmetic (no stencil, no relaxation, no transfer operator), so the CPU oracle
and the HIP path can both consume it without sharing any method code.

Array convention everywhere: a field on an m x n vertex grid is a float64 numpy
array of shape (n, m), indexed [j, i], i.e. row-major with element (i, j) at
flat offset j*m + i (x runs along a row, y across rows).  The perimeter holds
the Dirichlet data; the interior holds the initial guess.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Problem", "coords", "chamber", "chamber_counts", "harmonic_field",
    "manufactured", "random_boundary", "gaussian_bumps", "square_problem",
    "snap_size", "ragged_batch", "poisson_requests", "HARMONIC_KINDS",
]


@dataclass
class Problem:
    """One Dirichlet problem  L_h psi = f  on an m x n vertex grid."""
    m: int
    n: int
    dx: float
    dy: float
    psi0: np.ndarray          # (n, m) float64: perimeter = boundary data, interior = start
    f: np.ndarray | None      # (n, m) float64 source, or None for f == 0
    name: str = ""

    @property
    def beta(self) -> float:
        return self.dx / self.dy


def coords(m: int, n: int, dx: float, dy: float, x0: float = 0.0, y0: float = 0.0):
    """Node coordinates x_i = x0 + i*dx, y_j = y0 + j*dy (uniform grid of the
    paper's problem definition, Eq. (4))."""
    x = x0 + dx * np.arange(m, dtype=np.float64)
    y = y0 + dy * np.arange(n, dtype=np.float64)
    return x, y


# --------------------------------------------------------------------------
# Paper-sized chamber (Problem Definition section, Eq. (4)).
# --------------------------------------------------------------------------
def chamber(psi_ab: float = 100.0, gap_j0: int = 1, lx: float = 6.0, ly: float = 4.0,
            h: float = 0.25) -> Problem:
    """The 25 x 17 chamber.

    Lx = 6, Ly = 4, dx = dy = 0.25 gives m = Lx/dx + 1 = 25, n = Ly/dy + 1 = 17
    (Eq. (4)).  Boundary reading (the grid/BC figure is not available): the
    bottom wall and the side walls up to node j = gap_j0 hold psi = 0; the wall
    from the top of the inlet gap, across the top, down to the top of the
    outlet gap holds psi = psi_ab; across each 0.25 m gap psi ramps linearly
    0 -> psi_ab, which with dy = 0.25 puts no node strictly inside the gap.
    """
    m = int(round(lx / h)) + 1
    n = int(round(ly / h)) + 1
    psi = np.zeros((n, m), dtype=np.float64)
    gap_len = 0.25
    y = h * np.arange(n)
    y_c = gap_j0 * h                 # bottom of the gap (point C / D)
    y_a = y_c + gap_len              # top of the gap (point A / B)
    side = np.where(y <= y_c, 0.0, np.where(y >= y_a - 1e-12, psi_ab,
                                            psi_ab * (y - y_c) / gap_len))
    psi[:, 0] = side
    psi[:, m - 1] = side
    psi[n - 1, :] = psi_ab           # top wall
    psi[0, :] = 0.0                  # bottom wall
    return Problem(m, n, h, h, psi, None, name=f"chamber(psi_ab={psi_ab},gap_j0={gap_j0})")


def chamber_counts(m: int, n: int) -> dict:
    """Point counts of an m x n vertex grid in the bookkeeping of the problem
    definition: total m*n, 'boundary' 2(m+n) (four walls, corners counted on
    both walls), 'internal' = total - 2(m+n); plus the distinct boundary nodes
    and the true number of unknowns (m-2)(n-2)."""
    return {
        "total": m * n,
        "boundary_walls": 2 * (m + n),
        "internal_paper": m * n - 2 * (m + n),
        "boundary_distinct": 2 * (m + n) - 4,
        "unknowns": (m - 2) * (n - 2),
    }


# --------------------------------------------------------------------------
# Manufactured fields (discretely harmonic polynomials and a cubic with source)
# --------------------------------------------------------------------------
HARMONIC_KINDS = ("x2-y2", "xy", "x3-3xy2", "3x2y-y3", "x3")


def harmonic_field(kind: str, m: int, n: int, dx: float, dy: float,
                   x0: float = 0.0, y0: float = 0.0):
    """Return (psi, lap) for a polynomial field sampled at the nodes.

    psi is the exact field at every node; lap is its continuous Laplacian
    (zero for the harmonic kinds, 6x for 'x3').  Second differences of
    polynomials of degree <= 3 are exact, so these fields satisfy the 5-point
    equation exactly for any dx, dy.
    """
    x, y = coords(m, n, dx, dy, x0, y0)
    X, Y = np.meshgrid(x, y)          # shape (n, m), [j, i]
    if kind == "x2-y2":
        return X * X - Y * Y, np.zeros_like(X)
    if kind == "xy":
        return X * Y, np.zeros_like(X)
    if kind == "x3-3xy2":
        return X ** 3 - 3.0 * X * Y * Y, np.zeros_like(X)
    if kind == "3x2y-y3":
        return 3.0 * X * X * Y - Y ** 3, np.zeros_like(X)
    if kind == "x3":
        return X ** 3, 6.0 * X
    raise ValueError(kind)


def manufactured(kind: str, m: int, n: int, dx: float, dy: float,
                 x0: float = 0.0, y0: float = 0.0) -> tuple[Problem, np.ndarray]:
    """A Dirichlet problem whose exact discrete solution is a polynomial field:
    boundary = field on the perimeter, interior start 0, f = its Laplacian
    (None when harmonic).  Returns (problem, exact field)."""
    exact, lap = harmonic_field(kind, m, n, dx, dy, x0, y0)
    psi0 = exact.copy()
    psi0[1:-1, 1:-1] = 0.0
    f = None if not np.any(lap) else lap.copy()
    return Problem(m, n, dx, dy, psi0, f, name=f"manufactured({kind})"), exact


# --------------------------------------------------------------------------
# Random Dirichlet data, Gaussian-bump sources
# --------------------------------------------------------------------------
def random_boundary(m: int, n: int, rng: np.random.Generator | int) -> np.ndarray:
    """psi0 with U[0,1) boundary values and a zero interior.

    Draw order along the perimeter: row j=0 (i ascending), row j=n-1, column
    i=0 (j = 1..n-2), column i=m-1 (j = 1..n-2)."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    psi = np.zeros((n, m), dtype=np.float64)
    psi[0, :] = rng.random(m)
    psi[n - 1, :] = rng.random(m)
    psi[1:n - 1, 0] = rng.random(n - 2)
    psi[1:n - 1, m - 1] = rng.random(n - 2)
    return psi


def gaussian_bumps(m: int, n: int, dx: float, dy: float, rng: np.random.Generator | int,
                   count: int = 32) -> np.ndarray:
    """Source f = sum_k a_k exp(-((x-x_k)^2 + (y-y_k)^2) / (2 s_k^2)), with
    a_k ~ N(0,1), centres uniform in the domain, s_k = u_k * L, u_k ~ U[0.01, 0.1]
    and L the longer side of the domain."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.default_rng(rng)
    lx, ly = dx * (m - 1), dy * (n - 1)
    big = max(lx, ly)
    amp = rng.standard_normal(count)
    cx = rng.random(count) * lx
    cy = rng.random(count) * ly
    sig = rng.uniform(0.01, 0.1, count) * big
    x, y = coords(m, n, dx, dy)
    f = np.zeros((n, m), dtype=np.float64)
    for k in range(count):
        gx = np.exp(-((x - cx[k]) ** 2) / (2.0 * sig[k] ** 2))
        gy = np.exp(-((y - cy[k]) ** 2) / (2.0 * sig[k] ** 2))
        f += amp[k] * np.outer(gy, gx)
    return f


def square_problem(N: int, seed: int = 2, bumps: bool = False, bump_seed: int = 3) -> Problem:
    """Unit square, N x N vertices, h = 1/(N-1), beta = 1, U[0,1) boundary
    drawn from `seed`, zero start; f = 0 or 32 Gaussian bumps from `bump_seed`."""
    h = 1.0 / (N - 1)
    psi0 = random_boundary(N, N, seed)
    f = gaussian_bumps(N, N, h, h, bump_seed) if bumps else None
    return Problem(N, N, h, h, psi0, f, name=f"square{N}{'+bumps' if bumps else ''}")


# --------------------------------------------------------------------------
# Ragged batches and request streams
# --------------------------------------------------------------------------
_SNAP = None


def _snap_table(limit: int = 1 << 16) -> np.ndarray:
    global _SNAP
    if _SNAP is None:
        vals = sorted({c * (1 << k) + 1 for c in (4, 5, 6, 7) for k in range(0, 15)
                       if c * (1 << k) + 1 <= limit})
        _SNAP = np.array(vals, dtype=np.int64)
    return _SNAP


def snap_size(v: float) -> int:
    """Nearest size of the form c*2^k + 1 with c in {4,5,6,7}: such sizes can
    be vertex-coarsened k times."""
    t = _snap_table()
    return int(t[np.argmin(np.abs(t - v))])


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def ragged_batch(count: int = 512, lo: int = 33, hi: int = 1025, seed: int = 4,
                 max_aspect: float = 3.0, beta_range=(0.5, 2.0), bumps: bool = False) -> list[Problem]:
    """`count` independent grids: m, n log-uniform in [lo, hi] snapped to
    c*2^k+1, aspect max(m,n)/min(m,n) <= max_aspect (resampled), dy = 1/(n-1),
    dx = beta*dy with beta ~ U[beta_range], U[0,1) boundary, zero start."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        m = snap_size(_log_uniform(rng, lo, hi))
        n = snap_size(_log_uniform(rng, lo, hi))
        m = min(max(m, snap_size(lo)), snap_size(hi))
        n = min(max(n, snap_size(lo)), snap_size(hi))
        if max(m, n) / min(m, n) > max_aspect:
            continue
        beta = rng.uniform(*beta_range)
        dy = 1.0 / (n - 1)
        dx = beta * dy
        psi0 = random_boundary(m, n, rng)
        f = gaussian_bumps(m, n, dx, dy, rng) if bumps else None
        out.append(Problem(m, n, dx, dy, psi0, f, name=f"ragged[{len(out)}]"))
    return out


@dataclass
class Request:
    rid: int
    arrival: float            # seconds since stream start
    m: int
    n: int
    tol: float
    seed: int


def poisson_requests(rate: float, count: int, seed: int = 5, lo: int = 17, hi: int = 4097,
                     tols=(1e-8, 1e-10)) -> list[Request]:
    """A Poisson request stream: exponential inter-arrival times with mean
    1/rate; per request m, n log-uniform in [lo, hi] snapped to c*2^k+1; the
    tolerance uniform over `tols`; a per-request seed for its boundary and
    source (beta = 1)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        m = snap_size(_log_uniform(rng, lo, hi))
        n = snap_size(_log_uniform(rng, lo, hi))
        tol = float(tols[rng.integers(len(tols))])
        out.append(Request(r, t, m, n, tol, int(rng.integers(1 << 31))))
    return out


def request_problem(req: Request) -> Problem:
    """The grid of one request: unit spacing in y (dy = 1/(n-1)), beta = 1,
    U[0,1) boundary and a 32-bump source drawn from the request's seed."""
    rng = np.random.default_rng(req.seed)
    h = 1.0 / (max(req.m, req.n) - 1)
    psi0 = random_boundary(req.m, req.n, rng)
    f = gaussian_bumps(req.m, req.n, h, h, rng)
    return Problem(req.m, req.n, h, h, psi0, f, name=f"req{req.rid}")
