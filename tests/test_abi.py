"""CPU checks of the C-ABI library: it loads without a GPU, exports every
entry point include/lap.h declares, and the host-only calls behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lap.h")
LIB = os.path.join(ROOT, "paper_2208_02427_amd", "liblap.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lap_[a-z0-9_]+)\s*\(", txt)))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("liblap.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported():
    lib = _lib()
    names = declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_2208_02427_amd import _native
    assert set(declared()) == set(_native.SIGNATURES)


def test_host_only_calls():
    _lib()
    from paper_2208_02427_amd import _native as N
    lib = N.load()
    o = N.LapOpts()
    lib.lap_opts_default(ctypes.byref(o))
    assert (o.method, o.precision, o.nu1, o.nu2, o.max_iter) == (N.LAP_MG, N.LAP_FP64, 2, 2, 100)
    assert o.tol == 1e-10 and o.omega == 1.0
    assert lib.lap_version().startswith(b"liblap")
    # footprints grow with the hierarchies asked for and with the grid
    f64 = lib.lap_grid_footprint(4097, 4097, N.LAP_ALLOC_FP64)
    mix = lib.lap_grid_footprint(4097, 4097, N.LAP_ALLOC_MIXED)
    allf = lib.lap_grid_footprint(4097, 4097, N.LAP_ALLOC_ALL)
    assert 0 < mix < allf and 0 < f64 < allf
    assert lib.lap_grid_footprint(8193, 8193, N.LAP_ALLOC_ALL) > 3.5 * allf
    assert lib.lap_grid_footprint(2, 9, N.LAP_ALLOC_ALL) == 0
    assert lib.lap_op_work_bytes(65, 33) >= 33 * 64 * 8
    # every level of a (2^j + 1)-sided hierarchy from 65 to 8193 has a tiling class of its own
    assert [lib.lap_size_class(2 ** j + 1, 2 ** j + 1) for j in range(6, 14)] == list(range(8))
    assert lib.lap_size_class(5, 5) == 0 and lib.lap_size_class(16385, 16385) == 7
    # argument errors are reported without touching a device
    h = ctypes.c_void_p()
    assert lib.lap_ctx_create(None, 1 << 30, None, ctypes.byref(h)) == N.LAP_EINVAL
    assert b"arena" in lib.lap_last_error()
    assert lib.lap_ctx_create(ctypes.c_void_p(256), 1 << 10, None, ctypes.byref(h)) == N.LAP_EINVAL
    assert lib.lap_op_rb_sweep(0, 2, 5, 64, 0.1, 0.1, 1.0, None, None, None, 0, None, None) == N.LAP_EINVAL
    assert lib.lap_op_rb_sweep(0, 5, 5, 70, 0.1, 0.1, 1.0, None, None, None, 0, ctypes.c_void_p(256), None) \
        == N.LAP_EINVAL
    assert lib.lap_op_rb_sweep(0, 5, 5, 64, 0.1, 0.1, 2.0, None, None, None, 0, ctypes.c_void_p(256), None) \
        == N.LAP_EINVAL


def test_product_path_does_not_import_oracle():
    """The binding and the library never reference the oracle package."""
    pkg = os.path.join(ROOT, "paper_2208_02427_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"\boracle\b\s*(import|\.)|from\s+oracle|import\s+oracle", txt), fn
