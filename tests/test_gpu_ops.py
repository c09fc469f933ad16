"""Kernel-level parity: each lap_op_* kernel against the oracle function on
the same seeded inputs (sizes span several 64-lane windows and row chunks
with ragged tails, odd and even sizes, the 3 x 3 minimum).

Tolerances: FP64 kernels 1e-13 x max|field| (one kernel application, FMA
vs separate rounding); FP32 kernels 2e-6 x max|field| against the oracle's
float32 emulation (a few ulp over one expression chain).  ADI lines follow
the definition's operation order exactly and are compared bitwise.
"""
import numpy as np
import pytest

from gpu_helpers import need_gpu, say, to_dev, rand_problem, maxabs
from oracle import relax, grid as ogrid, multigrid as omg, lines as olines

pytestmark = pytest.mark.gpu

SIZES = [(3, 3), (5, 4), (4, 9), (7, 7), (65, 33), (130, 67), (257, 193), (300, 131), (513, 9)]
ODD = [(5, 5), (9, 17), (65, 33), (129, 65), (257, 193), (515, 131)]


@pytest.mark.parametrize("m,n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("variant", ["plain", "source", "zero"])
def test_rb_sweep(m, n, dtype, variant):
    torch, lap = need_gpu()
    say("rb_sweep", m, n, dtype, variant)
    psi, f, dx, dy = rand_problem(m, n, m * 1000 + n, source=(variant != "plain"))
    np_dt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    omega = 1.37
    if variant == "zero":
        psi = np.zeros_like(psi)
    u_in = lap.pitched(to_dev(torch, psi), tdt)
    u_out = u_in.clone()
    fd = lap.pitched(to_dev(torch, f), tdt) if f is not None else None
    lap.op_rb_sweep(m, n, dx, dy, omega, None if variant == "zero" else u_in, fd, u_out)
    torch.cuda.synchronize()
    got = u_out[:, :m].cpu().numpy()
    ref = psi.astype(np_dt)
    relax.rb_sweep(ref, None if f is None else f.astype(np_dt), dx, dy, omega, np_dt)
    scale = max(1.0, float(np.max(np.abs(ref))))
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert maxabs(got, ref) <= tol * scale
    # the input is untouched (out of place)
    if variant != "zero":
        assert np.array_equal(u_in[:, :m].cpu().numpy(), psi.astype(np_dt))


@pytest.mark.parametrize("m,n", ODD)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rb_sweep_with_prolongation(m, n, dtype):
    torch, lap = need_gpu()
    say("rb_sweep+prolong", m, n, dtype)
    psi, f, dx, dy = rand_problem(m, n, m + 7 * n)
    mc, nc = (m - 1) // 2 + 1, (n - 1) // 2 + 1
    rng = np.random.default_rng(5)
    ec = np.zeros((nc, mc))
    ec[1:-1, 1:-1] = rng.standard_normal((nc - 2, mc - 2))
    np_dt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u_in = lap.pitched(to_dev(torch, psi), tdt)
    u_out = u_in.clone()
    lap.op_rb_sweep(m, n, dx, dy, 1.0, u_in, lap.pitched(to_dev(torch, f), tdt), u_out,
                    ec=lap.pitched(to_dev(torch, ec), tdt))
    torch.cuda.synchronize()
    ref = psi.astype(np_dt) + omg.prolong(ec.astype(np_dt), m, n)
    relax.rb_sweep(ref, f.astype(np_dt), dx, dy, 1.0, np_dt)
    scale = max(1.0, float(np.max(np.abs(ref))))
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert maxabs(u_out[:, :m].cpu().numpy(), ref) <= tol * scale


@pytest.mark.parametrize("m,n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_residual_and_norms(m, n, dtype):
    torch, lap = need_gpu()
    say("residual", m, n, dtype)
    psi, f, dx, dy = rand_problem(m, n, 3 * m + n)
    np_dt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = lap.pitched(to_dev(torch, psi), tdt)
    r = torch.zeros_like(u)
    norms = lap.op_residual(m, n, dx, dy, u, lap.pitched(to_dev(torch, f), tdt), r)
    torch.cuda.synchronize()
    ref = ogrid.residual(psi.astype(np_dt), f.astype(np_dt), dx, dy, np_dt)
    scale = max(1.0, float(np.max(np.abs(ref))))
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert maxabs(r[:, :m].cpu().numpy(), ref) <= tol * scale
    s2, mx = norms.cpu().numpy()
    ref64 = ogrid.residual(psi.astype(np_dt).astype(np.float64), f.astype(np_dt).astype(np.float64), dx, dy)
    assert np.sqrt(s2) == pytest.approx(ogrid.norm2(ref64), rel=1e-12 if dtype == "f64" else 1e-5)
    assert mx == pytest.approx(ogrid.norm_inf(ref64), rel=1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("m,n", ODD)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_restrict(m, n, dtype):
    torch, lap = need_gpu()
    say("restrict", m, n, dtype)
    psi, f, dx, dy = rand_problem(m, n, 11 * m + n)
    np_dt = np.float64 if dtype == "f64" else np.float32
    tdt = torch.float64 if dtype == "f64" else torch.float32
    mc, nc = (m - 1) // 2 + 1, (n - 1) // 2 + 1
    bc = torch.zeros((nc, lap.pitch(mc)), dtype=tdt, device="cuda")
    lap.op_restrict(m, n, dx, dy, lap.pitched(to_dev(torch, psi), tdt), lap.pitched(to_dev(torch, f), tdt), bc)
    torch.cuda.synchronize()
    r = ogrid.residual(psi.astype(np_dt), f.astype(np_dt), dx, dy, np_dt)
    ref = omg.restrict_fw(r)
    scale = max(1.0, float(np.max(np.abs(ref))))
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert maxabs(bc[:, :mc].cpu().numpy(), ref) <= tol * scale


def _seg_fits(direction, K):
    """Whether the library solves these lines with the segmented solver
    (blocks of 15 unknowns + separators, at most 256 blocks); longer lines
    use the sequential recurrence."""
    S = 0 if K <= 0 else (K + 16) // 16
    return K >= 1 and S <= 256


# sizes: tiny; one block (K = 15); a separator as the last unknown (K = 16,
# 32); several blocks with ragged tails; long lines (K = 1023, 1024, 4095);
# lines past the segmented solver (sequential solver)
@pytest.mark.parametrize("m,n", [(3, 3), (4, 7), (17, 18), (18, 34), (35, 19), (25, 17), (66, 35), (200, 131),
                                 (131, 260), (1025, 24), (24, 1025), (9, 1026), (6, 4097), (4200, 5), (5, 4200)])
@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("form", [0, 1])
def test_adi_half(m, n, direction, form):
    torch, lap = need_gpu()
    say("adi_half", m, n, direction, form)
    psi, f, dx, dy = rand_problem(m, n, 17 * m + n, dx=0.1, dy=0.13)
    omega = 1.15
    u = lap.pitched(to_dev(torch, psi))
    lap.op_adi_half(m, n, dx, dy, omega, direction, form, u, lap.pitched(to_dev(torch, f)))
    ref = psi.copy()
    fn = olines.adi_zebra_rows_half if direction == 0 else olines.adi_zebra_cols_half
    fn(ref, f, dx, dy, omega, "A" if form == 0 else "B")
    got = u[:, :m].cpu().numpy()
    assert maxabs(got, ref) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    if not _seg_fits(direction, (m if direction == 0 else n) - 2):
        # the sequential solver evaluates the oracle's recurrence in its order
        assert np.array_equal(got, ref)


def test_op_argument_errors():
    torch, lap = need_gpu()
    say("op errors")
    u = torch.zeros((5, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(lap.LapError):
        lap.op_rb_sweep(5, 5, 0.1, 0.1, 2.0, u, None, u.clone())        # omega outside (0, 2)
    with pytest.raises(lap.LapError):
        lap.op_rb_sweep(2, 5, 0.1, 0.1, 1.0, u, None, u.clone())        # m < 3
    bad = torch.zeros((5, 70), dtype=torch.float64, device="cuda")
    with pytest.raises(lap.LapError):
        lap.op_rb_sweep(5, 5, 0.1, 0.1, 1.0, bad, None, bad.clone())    # ld not a multiple of 64
