"""Rows that wrap (GPU, through the C ABI): the 16-bit D2V9 step moves two nodes per thread
and treats the pair at each end of a row apart (the shifted pull of a pair and, in the
in-place step, its shifted store wrap around the row there). A grid only 2, 4 or 6 nodes
wide, where every pair or most pairs wrap, repeated periodically along x, must give
bit for bit the same populations as the repeated grid itself, where almost every pair is
an interior one: same node arithmetic, only the addressing differs. With obstacles,
fields, both forcing schemes, both storage formats and both step modes.
"""
import numpy as np
import pytest
import torch

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W

pytestmark = pytest.mark.gpu


def _tile(a, nx, ny, reps):
    """Repeat a node field (N,) or (C, N) reps times along x."""
    if a is None:
        return None
    if a.ndim == 1:
        return np.tile(a.reshape(ny, nx), (1, reps)).reshape(-1)
    return np.stack([_tile(c, nx, ny, reps) for c in a])


def _run(nx, ny, wl, storage, k, inplace, forcing, steps):
    sim = lbm.Simulation("D2V9", nx, ny, 1, tau=0.7, E=(2e-4, -1e-4, 0), B=(0, 0, 3e-3), storage=storage,
                         dev_scale_log2=k, mask=wl.mask, forcing=forcing, inplace=inplace)
    sim.init(wl.rho, wl.u)
    sim.step(steps)
    f = sim.export_f64().cpu().numpy().reshape(9, ny, nx)
    sim.close()
    return f


@pytest.mark.parametrize("inplace", [False, True], ids=["two-buffer", "in-place"])
@pytest.mark.parametrize("storage,k", [("f16", 12), ("bf16", 0)])
@pytest.mark.parametrize("nx,reps", [(2, 65), (4, 33), (6, 43)])
@pytest.mark.parametrize("forcing,phi", [("source", 0.0), ("shift", 0.2)])
def test_wrapping_rows_match_the_repeated_grid(nx, reps, storage, k, inplace, forcing, phi):
    ny, steps = 5, 7
    small = W.random_fields("D2V9", nx, ny, 1, seed=nx + 10 * reps, solid_fraction=phi, umax=0.02)
    big = W.Workload("tiled", "D2V9", nx * reps, ny, 1, tau=0.7, steps=0, rho=_tile(small.rho, nx, ny, reps),
                     u=_tile(small.u, nx, ny, reps), mask=_tile(small.mask, nx, ny, reps))
    fs = _run(nx, ny, small, storage, k, inplace, forcing, steps)
    fb = _run(nx * reps, ny, big, storage, k, inplace, forcing, steps)
    assert np.array_equal(np.tile(fs, (1, 1, reps)), fb)
    assert np.isfinite(fs).all() and np.abs(fs).max() > 0
