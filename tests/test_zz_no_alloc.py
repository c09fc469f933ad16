"""lap_op_residual_static (no work buffer, nothing allocated) against
lap_op_residual (caller's work buffer): the same kernels, so the residual
field and both norms must agree bit for bit; two calls in a row, the second
on a smaller grid (the shared per-GPU partials array keeps the first call's
contents, which the second must fully overwrite), FP64 then FP32.  The norms
are also checked against the oracle's residual."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import need_gpu, say, rand_problem
from oracle import grid as ogrid

pytestmark = pytest.mark.gpu


def _case(torch, lap, m, n, dtype, seed):
    psi, f, dx, dy = rand_problem(m, n, seed)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = lap.pitched(torch.as_tensor(psi, device="cuda"), tdt)
    ft = lap.pitched(torch.as_tensor(f, device="cuda"), tdt)
    r_ref = torch.zeros_like(u)
    r_new = torch.zeros_like(u)
    say("no-alloc residual", m, n, dtype)
    n_ref = lap.op_residual(m, n, dx, dy, u, ft, r_ref)
    n_new = lap.op_residual_static(m, n, dx, dy, u, ft, r_new)
    torch.cuda.synchronize()
    assert torch.equal(n_ref, n_new), (n_ref, n_new)
    assert torch.equal(r_ref, r_new)
    # the oracle's residual of the same (rounded) inputs
    uu = u[:, :m].double().cpu().numpy()
    ff = ft[:, :m].double().cpu().numpy()
    ro = ogrid.residual(uu, ff, dx, dy)
    s2 = float(np.sum(ro[1:-1, 1:-1] ** 2))
    mx = float(np.max(np.abs(ro[1:-1, 1:-1])))
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert abs(n_new[0].item() - s2) <= tol * s2
    assert abs(n_new[1].item() - mx) <= tol * mx
    return n_new


def test_static_residual_matches_work_buffer_version_twice():
    torch, lap = need_gpu()
    a = _case(torch, lap, 1027, 517, "f64", 1)
    b = _case(torch, lap, 131, 67, "f64", 2)        # smaller: fewer tiles than the first call
    assert not torch.equal(a, b)
    _case(torch, lap, 515, 300, "f32", 3)
    _case(torch, lap, 70, 35, "f32", 4)


def test_static_residual_rejects_oversized_grid_before_launch():
    torch, lap = need_gpu()
    from paper_2208_02427_amd import _native as N
    u = torch.zeros(256, dtype=torch.float64, device="cuda")
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    m = n = 16385                   # 68096 FP64 norm tiles > 65536
    ld = lap.pitch(m)
    st = lap.lib().lap_op_residual_static(0, m, n, ld, 1.0, 1.0, ctypes.c_void_p(u.data_ptr()), None, None,
                                          ctypes.c_void_p(norms.data_ptr()), None)
    assert st == N.LAP_EINVAL
    assert b"too large" in lap.lib().lap_last_error()
