"""MI355X (gfx950) solvers for the 5-point 2D Laplace / Poisson equation:
red-black SOR, line ADI with batched Thomas solves, multigrid V-cycles in
FP64 and mixed FP32/FP64 precision, batched and served solves.

This module is a thin binding over liblap.so (include/lap.h): it marshals
arguments and owns the device memory (a torch uint8 arena) and the HIP stream
(a torch stream); every step of every method runs in the library's kernels.
Fields are torch float64 tensors of shape (n, m) on the GPU, indexed [j, i]
(row-major, element (i, j) at j*m + i).
"""
from __future__ import annotations

import ctypes
import json
import os

from . import _native as N
from ._native import (LAP_SOR_RB, LAP_ADI, LAP_MG, LAP_JACOBI, LAP_SOR_LEX, LAP_SLOR_LEX,  # noqa: F401
                      LAP_ADI_LEX, LAP_STOP_DELTA, LAP_FP64, LAP_MIXED, LAP_STOP_REL_L2,
                      LAP_STOP_RES_INF, LAP_ADI_RELAX_AFTER, LAP_ADI_RELAX_INSIDE, LAP_SMOOTH_RB,
                      LAP_SMOOTH_ZEBRA, LAP_ALLOC_FP64,
                      LAP_ALLOC_MIXED, LAP_ALLOC_ADI, LAP_ALLOC_ALL, LapInfo, LapOpts)

# tilings measured by the autotuner on MI355X (applied to every new Context)
DEFAULT_TUNING = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")

METHODS = {"sor": LAP_SOR_RB, "rb": LAP_SOR_RB, "adi": LAP_ADI, "mg": LAP_MG,
           # the paper's sequential orderings (one workgroup, grid in LDS)
           "jacobi": LAP_JACOBI, "sor_lex": LAP_SOR_LEX, "gs_lex": LAP_SOR_LEX, "slor_lex": LAP_SLOR_LEX,
           "adi_lex": LAP_ADI_LEX}
PRECISIONS = {"fp64": LAP_FP64, "mixed": LAP_MIXED}


class LapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{N.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    return N.load()


def _check(status: int, allow=()):
    if status != 0 and status not in allow:
        raise LapError(status, lib().lap_last_error().decode())
    return status


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblap needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


SMOOTHERS = {"rb": LAP_SMOOTH_RB, "zebra": LAP_SMOOTH_ZEBRA}


def opts(method="mg", precision="fp64", omega=1.0, tol=1e-10, max_iter=100, stop="rel_l2", nu1=2, nu2=2,
         check_every=1, adi_form="after", use_graph=True, smoother="rb", fmg=False, inner=1) -> LapOpts:
    o = LapOpts()
    lib().lap_opts_default(ctypes.byref(o))
    o.method = METHODS[method] if isinstance(method, str) else int(method)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.omega = float(omega)
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.stop = {"rel_l2": LAP_STOP_REL_L2, "res_inf": LAP_STOP_RES_INF, "delta": LAP_STOP_DELTA}[stop] \
        if isinstance(stop, str) else int(stop)
    o.nu1 = int(nu1)
    o.nu2 = int(nu2)
    o.check_every = int(check_every)
    o.adi_form = {"after": LAP_ADI_RELAX_AFTER, "inside": LAP_ADI_RELAX_INSIDE}[adi_form] \
        if isinstance(adi_form, str) else int(adi_form)
    o.use_graph = 1 if use_graph else 0
    o.smoother = SMOOTHERS[smoother] if isinstance(smoother, str) else int(smoother)
    o.fmg = 1 if fmg else 0
    o.inner = int(inner)
    return o


class Context:
    """A device arena (torch uint8 tensor) and a HIP stream (torch stream)
    handed to lap_ctx_create.  Library work is ordered after the caller's
    current stream on entry and the current stream waits for it on exit."""

    def __init__(self, arena_bytes: int = 1 << 30, device: str = "cuda:0", tuning: str | None = "default"):
        torch = _torch()
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        _check(lib().lap_ctx_create(_ptr(self.arena), int(arena_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h)))
        self.handle = h
        self.grids = []
        if tuning == "default":
            tuning = DEFAULT_TUNING if os.path.exists(DEFAULT_TUNING) else None
        if tuning:
            with open(tuning) as fh:
                for rep in json.load(fh)["reports"]:
                    self.apply_tuning(rep)

    # stream ordering around library calls
    def _enter(self):
        torch = _torch()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch = _torch()
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def close(self):
        if getattr(self, "handle", None):
            lib().lap_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def usage(self):
        u, f = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().lap_ctx_usage(self.handle, ctypes.byref(u), ctypes.byref(f)))
        return u.value, f.value

    def set_timing(self, on=True):
        """False/0 off, True/1 events around every launch, 2 around finest-level launches only."""
        _check(lib().lap_ctx_set_timing(self.handle, int(on)))

    def reset_stats(self):
        _check(lib().lap_ctx_reset_stats(self.handle))

    def kernel_stats(self, cls: int, fine_only: bool = False):
        n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().lap_ctx_kernel_stats(self.handle, int(cls), 1 if fine_only else 0, ctypes.byref(n),
                                          ctypes.byref(ms), ctypes.byref(b)))
        return {"launches": n.value, "device_ms": ms.value, "alg_bytes": b.value}

    # ------------------------------------------------------------ tilings
    def autotune(self, m: int, n: int, reps: int = 5) -> dict:
        """Time every candidate tiling of the stencil kernels on an m x n level
        and keep the fastest for its size class; returns the report."""
        buf = ctypes.create_string_buffer(1 << 16)
        self._enter()
        st = lib().lap_autotune(self.handle, int(m), int(n), int(reps), buf, len(buf))
        self._leave()
        _check(st)
        return json.loads(buf.value.decode())

    def apply_tuning(self, report: dict):
        """Re-apply the choices of an autotune report (e.g. loaded from JSON)."""
        # the class follows from the tuned size (tables written with other class bounds stay valid)
        sc = size_class(int(report["m"]), int(report["n"])) if "m" in report else int(report["size_class"])
        for e in report["best"]:
            self.set_tiling(e["class"], 0 if e["dtype"] == "f64" else 1, sc, e["V"], e["ty"], e["target_waves"])

    def set_tiling(self, cls, dtype, size_class, V, ty, target_waves=0):
        _check(lib().lap_ctx_set_tiling(self.handle, int(cls), int(dtype), int(size_class), int(V), int(ty),
                                        int(target_waves)))

    def get_tiling(self, cls, dtype, size_class):
        v, t, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lap_ctx_get_tiling(self.handle, int(cls), int(dtype), int(size_class), ctypes.byref(v),
                                        ctypes.byref(t), ctypes.byref(w)))
        return v.value, t.value, w.value

    def set_subtree(self, max_nodes=-1):
        """Small-level subtree: -1 any level whose sub-V-cycle fits LDS, 0 off,
        else the largest top level (m*n nodes) that may run as one launch."""
        _check(lib().lap_ctx_set_subtree(self.handle, int(max_nodes)))

    def set_fusion(self, on=True):
        """Fused smoothing passes (two sweeps per pass, restriction and
        prolongation folded in); off = one launch per sweep."""
        _check(lib().lap_ctx_set_fusion(self.handle, 1 if on else 0))

    def get_fusion(self):
        v = ctypes.c_int32()
        _check(lib().lap_ctx_get_fusion(self.handle, ctypes.byref(v)))
        return bool(v.value)

    def get_subtree(self):
        v, b = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().lap_ctx_get_subtree(self.handle, ctypes.byref(v), ctypes.byref(b)))
        return v.value, b.value

    def grid(self, psi0, f=None, dx=1.0, dy=1.0, alloc=LAP_ALLOC_ALL) -> "Grid":
        return Grid(self, psi0, f, dx, dy, alloc)

    def solve_batch(self, grids, **kw):
        o = opts(**kw)
        arr = (ctypes.c_void_p * len(grids))(*[g.handle.value for g in grids])
        infos = (LapInfo * len(grids))()
        self._enter()
        st = lib().lap_solve_batch(self.handle, arr, len(grids), ctypes.byref(o), infos)
        self._leave()
        _check(st, allow=(N.LAP_ENOTCONV, N.LAP_EDIVERGED))
        return [i.as_dict() for i in infos]

    def batch_step(self, grids, precision="mixed", steps=1):
        """One continuous-batching tick of `steps` outer steps; returns (done flags, infos)."""
        n = len(grids)
        arr = (ctypes.c_void_p * n)(*[g.handle.value for g in grids])
        done = (ctypes.c_int32 * n)()
        infos = (LapInfo * n)()
        self._enter()
        st = lib().lap_batch_step(self.handle, arr, n, PRECISIONS[precision] if isinstance(precision, str)
                                  else int(precision), int(steps), done, infos)
        self._leave()
        _check(st, allow=(N.LAP_ENOTCONV, N.LAP_EDIVERGED))
        return [bool(d) for d in done], [i.as_dict() for i in infos]


def size_class(m: int, n: int) -> int:
    return int(lib().lap_size_class(int(m), int(n)))


def footprint(m: int, n: int, alloc=LAP_ALLOC_ALL) -> int:
    return int(lib().lap_grid_footprint(int(m), int(n), int(alloc)))


class Grid:
    """A device-resident problem (boundary, source, solution, hierarchies)."""

    def __init__(self, ctx: Context, psi0, f=None, dx=1.0, dy=1.0, alloc=LAP_ALLOC_ALL):
        torch = _torch()
        self.ctx = ctx
        psi0 = torch.as_tensor(psi0, dtype=torch.float64, device=ctx.device).contiguous()
        if psi0.dim() != 2:
            raise ValueError("psi0 must be a 2-D (n, m) array")
        self.n, self.m = psi0.shape
        self.dx, self.dy = float(dx), float(dy)
        src = None
        if f is not None:
            src = torch.as_tensor(f, dtype=torch.float64, device=ctx.device).contiguous()
            if tuple(src.shape) != (self.n, self.m):
                raise ValueError("f must have the shape of psi0")
        h = ctypes.c_void_p()
        ctx._enter()
        st = lib().lap_grid_create_ex(ctx.handle, self.m, self.n, self.dx, self.dy, _ptr(psi0), _ptr(src),
                                      int(alloc), ctypes.byref(h))
        ctx._leave()
        _check(st)
        self.handle = h
        self.last_info = None

    def destroy(self):
        if self.handle:
            lib().lap_grid_destroy(self.handle)
            self.handle = None

    def levels(self):
        nl = ctypes.c_int32()
        _check(lib().lap_grid_levels(self.handle, ctypes.byref(nl)))
        out = []
        for l in range(nl.value):
            a, b = ctypes.c_int32(), ctypes.c_int32()
            _check(lib().lap_grid_level_shape(self.handle, l, ctypes.byref(a), ctypes.byref(b)))
            out.append((a.value, b.value))
        return out

    def solve(self, method="mg", precision="fp64", omega=1.0, tol=1e-10, max_iter=100, raise_on_fail=False,
              **kw) -> dict:
        o = opts(method=method, precision=precision, omega=omega, tol=tol, max_iter=max_iter, **kw)
        info = LapInfo()
        self.ctx._enter()
        st = lib().lap_solve_ex(self.handle, ctypes.byref(o), ctypes.byref(info))
        self.ctx._leave()
        if raise_on_fail:
            _check(st)
        else:
            _check(st, allow=(N.LAP_ENOTCONV, N.LAP_EDIVERGED))
        d = info.as_dict()
        d["status"] = st
        self.last_info = d
        return d

    def read(self):
        torch = _torch()
        out = torch.empty((self.n, self.m), dtype=torch.float64, device=self.ctx.device)
        self.ctx._enter()
        st = lib().lap_grid_read(self.handle, _ptr(out))
        self.ctx._leave()
        _check(st)
        return out

    def write(self, psi):
        torch = _torch()
        psi = torch.as_tensor(psi, dtype=torch.float64, device=self.ctx.device).contiguous()
        self.ctx._enter()
        st = lib().lap_grid_write(self.handle, _ptr(psi))
        self.ctx._leave()
        _check(st)

    def residual(self):
        """(||r||_2, max|r|) of the current solution, FP64."""
        l2, li = ctypes.c_double(), ctypes.c_double()
        self.ctx._enter()
        st = lib().lap_residual_ex(self.handle, ctypes.byref(l2), ctypes.byref(li))
        self.ctx._leave()
        _check(st)
        return l2.value, li.value

    def set_tol(self, tol: float):
        _check(lib().lap_grid_set_tol(self.handle, float(tol)))

    def set_omega(self, omega: float):
        """Smoother relaxation of the grid's batched steps (lap_batch_step)."""
        _check(lib().lap_grid_set_omega(self.handle, float(omega)))

    def reset(self):
        _check(lib().lap_grid_reset(self.handle))


# ----------------------------------------------------------------- op level
def pitch(m: int) -> int:
    return (m + 63) // 64 * 64


def pitched(a, dtype=None):
    """Copy an (n, m) tensor into a zero-padded (n, pitch(m)) device tensor
    (the layout of the lap_op_* calls); returns the padded tensor."""
    torch = _torch()
    a = torch.as_tensor(a, device="cuda")
    dtype = dtype or a.dtype
    n, m = a.shape
    out = torch.zeros((n, pitch(m)), dtype=dtype, device=a.device)
    out[:, :m] = a.to(dtype)
    return out


def _dt(t):
    torch = _torch()
    return 0 if t.dtype == torch.float64 else 1


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def op_rb_sweep(m, n, dx, dy, omega, u_in, f, u_out, ec=None):
    """One red-black sweep u_out <- sweep(u_in [+ P ec]) on pitched tensors."""
    ld = u_out.shape[1]
    ldc = ec.shape[1] if ec is not None else 0
    _check(lib().lap_op_rb_sweep(_dt(u_out), m, n, ld, float(dx), float(dy), float(omega), _ptr(u_in), _ptr(f),
                                 _ptr(ec), ldc, _ptr(u_out), _stream()))


def op_residual(m, n, dx, dy, u, f=None, r=None, want_norms=True):
    torch = _torch()
    ld = u.shape[1]
    norms = torch.zeros(2, dtype=torch.float64, device=u.device) if want_norms else None
    work = torch.empty(int(lib().lap_op_work_bytes(m, n)), dtype=torch.uint8, device=u.device)
    _check(lib().lap_op_residual(_dt(u), m, n, ld, float(dx), float(dy), _ptr(u), _ptr(f), _ptr(r), _ptr(norms),
                                 _ptr(work), _stream()))
    return norms


def op_residual_static(m, n, dx, dy, u, f=None, r=None, want_norms=True):
    """op_residual without a work buffer: the norm partials go to the
    library's fixed per-GPU array (lap_op_residual_static)."""
    torch = _torch()
    ld = u.shape[1]
    norms = torch.zeros(2, dtype=torch.float64, device=u.device) if want_norms else None
    _check(lib().lap_op_residual_static(_dt(u), m, n, ld, float(dx), float(dy), _ptr(u), _ptr(f), _ptr(r),
                                        _ptr(norms), _stream()))
    return norms


def op_restrict(m, n, dx, dy, u, f, bc):
    ld = u.shape[1] if u is not None else f.shape[1]
    _check(lib().lap_op_restrict(_dt(bc), m, n, ld, float(dx), float(dy), _ptr(u), _ptr(f), _ptr(bc), bc.shape[1],
                                 _stream()))


def op_adi_half(m, n, dx, dy, omega, direction, form, u, f=None):
    torch = _torch()
    work = torch.empty(int(lib().lap_op_work_bytes(m, n)), dtype=torch.uint8, device=u.device)
    _check(lib().lap_op_adi_half(0, m, n, u.shape[1], float(dx), float(dy), float(omega), int(direction), int(form),
                                 _ptr(u), _ptr(f), _ptr(work), _stream()))
    torch.cuda.current_stream().synchronize()


def op_stream_copy(src, dst, nbytes=None, blocks=2048):
    """Plain device copy (the bandwidth reference kernel)."""
    nbytes = int(nbytes if nbytes is not None else src.numel() * src.element_size())
    _check(lib().lap_op_stream_copy(_ptr(src), _ptr(dst), nbytes, int(blocks), _stream()))
