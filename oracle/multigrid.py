"""Oracle: multigrid V-cycle and mixed-precision defect correction.

Paper passages: the "Multigrid Method (V-Cycle)" section: operator (Eq. (11)),
residual (Eq. (12)), correction psi = dpsi + psi^k (Eq. (13)), error
equation L dpsi = -R (Eqs. (14)-(15)), the three mesh levels 25x17 / 13x9 /
7x5 and the eleven-step cycle; repeated until converged.

Readings (the V-cycle figure is not available):
* Levels are vertex-coarsened: m_{l+1} = (m_l - 1)/2 + 1, spacing doubled, and
  the coarse operator is the 5-point operator rediscretised at the coarse
  spacing (the three mesh sizes are exactly this).  Coarsening continues
  while both sides are odd and stay >= 5.
* Residual transfer: 9-point full weighting; correction transfer: bilinear
  interpolation; the correction is zero on every coarse boundary.  The paper
  names neither operator.
* The coarsest level is solved "till convergence", i.e. exactly: here by the
  dense elimination of oracle.direct.
* Smoother: red-black SOR (oracle.relax.rb_sweep) with nu1 pre- and nu2
  post-sweeps; the paper's own variant is 3 lexicographic GS sweeps per visit
  and is available with smoother='gs_lex'.  smoother='zebra' smooths with the
  paper's line relaxation instead: one smoothing step is one ADI iteration in
  zebra order (oracle.lines.adi_zebra_iteration: odd rows, even rows, odd
  columns, even columns, each line solved exactly, relaxation after the
  solve with omega_s), which stays a good smoother when dx != dy makes the
  5-point operator anisotropic.
* Sign: r = f - L_h u and L_h e = r (equivalent to Eqs. (12)-(15)).

Mixed precision (not in the paper): psi and the residual stay FP64; each
outer step solves the error equation approximately by one FP32 V-cycle from
a zero start (or `inner` cycles, each next from the previous correction,
forming its level-0 residual with the operator in difference form) and adds
the FP32 correction to the FP64 iterate.  How many cycles a step runs
is the driver's choice (oracle.solve.mixed_solve).

Pins (tests/test_oracle_multigrid.py): full weighting and bilinear
interpolation reproduce linear fields exactly and satisfy the adjoint
identity 4 <FW r, e>_c = <r, P e>_f; the V-cycle leaves discretely harmonic
fields unchanged and converges to the DST solution; its asymptotic factor is
below 0.15 and its cycle count to 1e-10 does not grow with the grid
(h-independence); the mixed loop reaches the FP64 solution; with several
FP32 cycles per defect correction its residual after each step follows the
FP64 cycle history at the cycles run so far, and one step of two cycles
lands within FP32 storage noise of two FP64 cycles (with the later cycle's
level-0 residual in the standard form it is 20x farther on 513^2); the
difference form equals the standard one in FP64 and is the more accurate in
FP32 for a smooth field; a last step shortened to one
cycle (oracle.solve.one_cycle_suffices, pinned against its closed form)
lands on the history one cycle further, with no more steps than without it.
"""
from __future__ import annotations

import numpy as np

from .grid import coefficients, residual, residual_diff, norm2
from .relax import rb_sweep, gs_lex_sweep
from .lines import adi_zebra_iteration
from .direct import dense_solve


def hierarchy(m: int, n: int, dx: float, dy: float, max_levels: int = 64, min_side: int = 5):
    """Level list [(m, n, dx, dy), ...] from fine to coarse."""
    levels = [(m, n, dx, dy)]
    while len(levels) < max_levels:
        mm, nn, hx, hy = levels[-1]
        if (mm - 1) % 2 or (nn - 1) % 2:
            break
        mc, nc = (mm - 1) // 2 + 1, (nn - 1) // 2 + 1
        if mc < min_side or nc < min_side:
            break
        levels.append((mc, nc, 2.0 * hx, 2.0 * hy))
    return levels


def restrict_fw(r: np.ndarray) -> np.ndarray:
    """Full weighting of a fine field r (zero perimeter) to the coarse grid:
        b(I,J) = [4 r(2I,2J) + 2 (r(2I±1,2J) + r(2I,2J±1)) + r(2I±1,2J±1)] / 16
    at coarse interior nodes, 0 on the coarse perimeter."""
    n, m = r.shape
    mc, nc = (m - 1) // 2 + 1, (n - 1) // 2 + 1
    dt = r.dtype.type
    b = np.zeros((nc, mc), dtype=r.dtype)
    C = r[2:-2:2, 2:-2:2]
    W = r[2:-2:2, 1:-3:2]
    E = r[2:-2:2, 3:-1:2]
    S = r[1:-3:2, 2:-2:2]
    N = r[3:-1:2, 2:-2:2]
    SW = r[1:-3:2, 1:-3:2]
    SE = r[1:-3:2, 3:-1:2]
    NW = r[3:-1:2, 1:-3:2]
    NE = r[3:-1:2, 3:-1:2]
    b[1:-1, 1:-1] = ((dt(4) * C + dt(2) * ((W + E) + (S + N))) + ((SW + SE) + (NW + NE))) * dt(0.0625)
    return b


def prolong(e: np.ndarray, m: int, n: int) -> np.ndarray:
    """Bilinear interpolation of a coarse correction (zero perimeter) to the
    fine m x n grid: coincident nodes copy, edge midpoints average two, cell
    centres average four."""
    dt = e.dtype.type
    p = np.zeros((n, m), dtype=e.dtype)
    p[0::2, 0::2] = e
    p[0::2, 1::2] = (e[:, :-1] + e[:, 1:]) * dt(0.5)
    p[1::2, 0::2] = (e[:-1, :] + e[1:, :]) * dt(0.5)
    p[1::2, 1::2] = ((e[:-1, :-1] + e[:-1, 1:]) + (e[1:, :-1] + e[1:, 1:])) * dt(0.25)
    return p


def coarse_solve(u: np.ndarray, b: np.ndarray | None, dx: float, dy: float) -> None:
    """Exact solve of L_h u = b on a (small) level with u's perimeter as the
    boundary, in place (done in FP64 and rounded to u's dtype)."""
    n, m = u.shape
    bb = None if b is None else b.astype(np.float64)
    sol = dense_solve(m, n, dx, dy, u.astype(np.float64), bb)
    u[1:-1, 1:-1] = sol[1:-1, 1:-1].astype(u.dtype)


def vcycle(levels, l: int, u: np.ndarray, b: np.ndarray | None, nu1: int = 2, nu2: int = 2,
           omega_s: float = 1.0, dtype=np.float64, smoother: str = "rb", top_residual_diff: bool = False) -> None:
    """One V-cycle on level l, in place on u (u's perimeter is the boundary:
    g on level 0, zero on coarse levels; b is the right-hand side):
        nu1 smoothing sweeps; r = b - L u; b' = FW(r); e' = 0;
        V(l+1, e', b'); u += P e'; nu2 smoothing sweeps.
    The coarsest level is solved exactly.  With top_residual_diff the
    residual of level l is formed with L_h in difference form
    (grid.residual_diff; the coarser levels as usual)."""
    m, n, dx, dy = levels[l]
    if l == len(levels) - 1:
        coarse_solve(u, b, dx, dy)
        return

    def smooth():
        if smoother == "rb":
            rb_sweep(u, b, dx, dy, omega_s, dtype)
        elif smoother == "gs_lex":
            gs_lex_sweep(u, b, dx, dy, omega_s)
        elif smoother == "zebra":
            adi_zebra_iteration(u, b, dx, dy, omega_s, "A")
        else:
            raise ValueError(smoother)

    for _ in range(nu1):
        smooth()
    r = (residual_diff if top_residual_diff else residual)(u, b, dx, dy, dtype)
    bc = restrict_fw(r)
    mc, nc, _, _ = levels[l + 1]
    ec = np.zeros((nc, mc), dtype=u.dtype)
    vcycle(levels, l + 1, ec, bc, nu1, nu2, omega_s, dtype, smoother)
    u += prolong(ec, m, n)
    for _ in range(nu2):
        smooth()


def mixed_step(psi: np.ndarray, f: np.ndarray | None, levels, nu1=2, nu2=2, omega_s=1.0, smoother="rb",
               inner: int = 1):
    """One outer step of the mixed-precision defect correction:
        r64 = f - L_h psi64;  b32 = fl32(r64);
        e32 = `inner` FP32 V-cycles on L_h e = b32, the first from 0;
        psi64 += fl64(e32).
    (Eqs. (13)-(15) solve the error equation with the cycle; more cycles per
    correction solve it more accurately before the FP64 update.)  A cycle
    after the first starts from a smooth correction of large values: the
    standard form of its level-0 residual b32 - L_h e32 adds terms of size
    8|e|/h^2 whose FP32 rounding swamps the smooth part the coarse levels must
    see (on 8193^2 the second cycle then no longer reduces smooth error), so
    those cycles form it with L_h in difference form (vcycle's
    top_residual_diff), still in FP32.  Returns the FP64 residual taken at
    the start of the step."""
    m, n, dx, dy = levels[0]
    r = residual(psi, f, dx, dy)
    b32 = r.astype(np.float32)
    e32 = np.zeros_like(b32)
    for c in range(inner):
        vcycle(levels, 0, e32, b32, nu1, nu2, omega_s, np.float32, smoother, top_residual_diff=c > 0)
    psi += e32.astype(np.float64)
    return r


def mixed_residual_after(psi, f, levels):
    m, n, dx, dy = levels[0]
    return norm2(residual(psi, f, dx, dy))


def boundary_on_level(psi_b: np.ndarray, l: int) -> np.ndarray:
    """The Dirichlet data of level l: the fine perimeter values at the nodes
    the level keeps (every 2^l-th node), on an otherwise zero array."""
    s = 1 << l
    g = psi_b[::s, ::s].copy()
    g[1:-1, 1:-1] = 0.0
    return g


def fmg(levels, psi_b: np.ndarray, f: np.ndarray | None, nu1: int = 2, nu2: int = 2,
        omega_s: float = 1.0, smoother: str = "rb") -> np.ndarray:
    """Full multigrid start (not in the paper; it follows the paper's argument
    for multigrid, that the low-frequency error a fine grid removes slowly is
    removed cheaply on coarse grids): the problem itself, not its error
    equation, is posed on every level, with the boundary data of the level's
    nodes and the source full-weighted down the hierarchy; the coarsest level
    is solved exactly, and each finer level starts from the bilinear
    interpolation of the coarser level's solution (boundary included) and
    takes one V(nu1, nu2) cycle.  Returns the level-0 field."""
    L = len(levels)
    fs = [None] * L
    fs[0] = np.zeros_like(psi_b) if f is None else np.array(f, dtype=np.float64)
    for l in range(1, L):
        fs[l] = restrict_fw(fs[l - 1])
    m, n, dx, dy = levels[L - 1]
    u = boundary_on_level(psi_b, L - 1)
    coarse_solve(u, fs[L - 1], dx, dy)
    for l in range(L - 2, -1, -1):
        m, n, dx, dy = levels[l]
        v = boundary_on_level(psi_b, l)
        v[1:-1, 1:-1] = prolong(u, m, n)[1:-1, 1:-1]
        vcycle(levels[l:], 0, v, fs[l], nu1, nu2, omega_s, np.float64, smoother)
        u = v
    return u
