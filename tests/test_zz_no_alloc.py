"""lbm_current_noalloc (the totals of lbm_current with the reduction in the library's static
device scratch instead of the workspace) against lbm_current on the same handle: the same
bits, on two calls in a row, the second on a smaller grid, then again on the first handle
(each call overwrites what it reads of the shared scratch)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W

pytestmark = pytest.mark.gpu


def _sim(wl, **kw):
    sim = lbm.Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=wl.E, B=wl.B, mask=wl.mask, s=wl.s, **kw)
    sim.init(wl.rho, wl.u)
    return sim


def _noalloc(sim):
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    rc = sim.lib.lbm_current_noalloc(sim.h, ctypes.c_void_p(out.data_ptr()))
    assert rc == lbm.LBM_OK, sim.lib.lbm_last_error(sim.h)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_current_noalloc_matches_current():
    big = W.random_fields("D2V9", 1030, 37, 1, seed=11, solid_fraction=0.2, umax=0.02)
    big.E = (2e-5, -1e-5, 0.0)
    small = W.random_fields("D3V19", 9, 7, 5, seed=12, solid_fraction=0.1, soft=True, umax=0.02)
    small.E, small.B = (1e-5, 0.0, 2e-5), (0.0, 1e-3, 0.0)
    a, b = _sim(big), _sim(small)
    a.step(7)
    b.step(5)
    for sim, label in ((a, "1030x37 D2V9"), (b, "9x7x5 D3V19"), (a, "1030x37 D2V9 again")):
        want = sim.current()
        got = _noalloc(sim)
        print(f"{label}: lbm_current {want}, lbm_current_noalloc {got}")
        assert np.array_equal(got, want), (label, got, want)
    # the in-place step in its odd layout, and a state that changed since the last call
    c = _sim(big, inplace=True)
    c.step(3)
    assert np.array_equal(_noalloc(c), c.current())
    a.step(1)
    assert np.array_equal(_noalloc(a), a.current())
    for s in (a, b, c):
        s.close()


def test_current_noalloc_rejects():
    wl = W.random_fields("D2V9", 16, 8, 1, seed=1)
    sim = lbm.Simulation("D2V9", 16, 8, 1, tau=0.8)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    assert sim.lib.lbm_current_noalloc(sim.h, ctypes.c_void_p(out.data_ptr())) == lbm.LBM_ESTATE
    sim.init(wl.rho, wl.u)
    assert sim.lib.lbm_current_noalloc(sim.h, None) == lbm.LBM_EINVAL
    assert sim.lib.lbm_current_noalloc(None, ctypes.c_void_p(out.data_ptr())) == lbm.LBM_EINVAL
    sim.close()
