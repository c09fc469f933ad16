"""Autotuner and tilings: every tiling of a kernel produces bitwise identical
fields (pointwise kernels; the window / chunk split only changes which
wavefront computes a node), and the autotuner returns a valid choice."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import need_gpu, say, to_dev

pytestmark = pytest.mark.gpu

TILINGS = [(1, 16, 0), (2, 32, 0), (4, 128, 0), (2, 0, 8192), (4, 0, 16384), (1, 0, 256)]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solution_bitwise_identical_across_tilings(precision):
    torch, lap = need_gpu()
    p = W.square_problem(257, seed=2, bumps=True, bump_seed=3)
    outs = []
    for (V, ty, tgt) in TILINGS:
        say("tiling", precision, V, ty, tgt)
        ctx = lap.Context(arena_bytes=256 << 20)
        for sc in range(8):
            for cls in range(15):
                for dt in (0, 1):
                    ctx.set_tiling(cls, dt, sc, V, ty, tgt)
        g = ctx.grid(to_dev(torch, p.psi0), to_dev(torch, p.f), p.dx, p.dy)
        info = g.solve("mg", precision=precision, tol=0.0, max_iter=3)
        outs.append(g.read().cpu().numpy())
        g.destroy()
        ctx.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_autotune_report_and_effect():
    torch, lap = need_gpu()
    say("autotune 257")
    ctx = lap.Context(arena_bytes=256 << 20)
    rep = ctx.autotune(257, 257, reps=2)
    assert rep["size_class"] == lap.size_class(257, 257) == 2
    kinds = {(e["kernel"], e["dtype"]) for e in rep["best"]}
    assert ("sweep", "f64") in kinds and ("defect", "f64") in kinds and ("restrict", "f32") in kinds
    for e in rep["best"]:
        assert (e["V"], e["ty"], e["target_waves"]) == ctx.get_tiling(e["class"], 0 if e["dtype"] == "f64" else 1, 2)
        assert e["ms"] > 0
    ctx2 = lap.Context(arena_bytes=64 << 20)
    ctx2.apply_tuning(rep)
    e = rep["best"][0]
    assert ctx2.get_tiling(e["class"], 0 if e["dtype"] == "f64" else 1, 2) == (e["V"], e["ty"], e["target_waves"])
    with pytest.raises(lap.LapError):
        ctx.set_tiling(0, 0, 1, 3, 16, 0)
    with pytest.raises(lap.LapError):
        ctx.set_tiling(0, 0, 1, 2, 15, 0)
    with pytest.raises(lap.LapError):
        ctx.set_tiling(0, 0, 8, 2, 16, 0)
