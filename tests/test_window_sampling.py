"""The sampled-window parity method: the oracle recomputes a block of nodes on a
periodic sub-window that holds its whole dependence cone. Checked here, on the CPU,
against full-grid oracle runs (the window result must be identical)."""
import numpy as np
import pytest

from paper_1710_09472_amd import workloads as W
from parity_helpers import oracle_fields, oracle_window_fields


@pytest.mark.parametrize("lattice,shape,centre,core,steps", [
    ("D2V9", (64, 48, 1), (60, 3, 0), 8, 10),
    ("D2V9", (80, 4, 1), (0, 0, 0), 8, 12),
    ("D3V19", (30, 26, 24), (29, 0, 12), 4, 6),
])
def test_window_equals_full_grid(lattice, shape, centre, core, steps):
    wl = W.random_fields(lattice, *shape, seed=21, solid_fraction=0.15, soft=True, umax=0.02)
    wl.tau, wl.E, wl.B = 0.7, (1e-4, -2e-5, 1e-5 if lattice == "D3V19" else 0), (0, 0, 2e-3)
    rho, u, _, _ = oracle_fields(wl, steps)
    idx, rho_w, u_w = oracle_window_fields(wl, steps, core, centre)
    np.testing.assert_array_equal(rho_w, rho[idx])
    np.testing.assert_array_equal(u_w, u[:, idx])
