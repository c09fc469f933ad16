"""Shared helpers of the GPU tests (not collected by pytest)."""
import sys

import numpy as np
import pytest

import workloads as W


def say(*a):
    """Name the case on stdout before a GPU step (survives a crash of the run)."""
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2208_02427_amd as lap
    lap.lib()          # fails loudly if liblap.so is missing
    return torch, lap


def to_dev(torch, a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def rand_problem(m, n, seed, dx=None, dy=None, source=True, interior=True):
    rng = np.random.default_rng(seed)
    dx = dx if dx is not None else 1.0 / (m - 1)
    dy = dy if dy is not None else 1.3 / (n - 1)
    psi = W.random_boundary(m, n, rng)
    if interior:
        psi[1:-1, 1:-1] = rng.random((n - 2, m - 2))
    f = rng.standard_normal((n, m)) * 10.0 if source else None
    return psi, f, dx, dy


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))))
