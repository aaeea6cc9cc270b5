"""Edge cases of the GPU path, through the C ABI.

* Single-node grids (every neighbour is the node itself), against the oracle.
* Zero steps leave the state bit for bit; zero-length rho <-> mu conversions are no-ops.
* Grids at the library's size limit (Q * stride just below 2^31 elements, 8.6 GB per
  FP32 state): exact mass and the momentum recurrence P' = P + M E + P x B over 20
  steps, and sampled blocks against the oracle on their dependence cones, including the
  last nodes of the grid.
"""
import numpy as np
import pytest
import torch

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_fields, gpu_sim, oracle_fields, oracle_window_fields, rel_errors

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lattice,forcing", [("D2V9", "source"), ("D3V19", "source"), ("D2V9", "shift"),
                                             ("D3V19", "shift")])
def test_single_node_grid(lattice, forcing):
    wl = W.random_fields(lattice, 1, 1, 1, seed=3, umax=0.05)
    wl.tau, wl.forcing = 0.7, forcing
    wl.E = (1e-3, -5e-4, 2e-4 if lattice == "D3V19" else 0.0)
    wl.B = (1e-3, -2e-3, 3e-3) if lattice == "D3V19" else (0, 0, 3e-3)
    sim = gpu_sim(wl)
    sim.step(20)
    rho, u = gpu_fields(sim)
    rho_o, u_o, _, _ = oracle_fields(wl, 20)
    er, eu = rel_errors(rho, u, rho_o, u_o)
    assert er < 1e-5 and eu < 1e-5, (er, eu)


def test_zero_steps_and_zero_length():
    wl = W.random_fields("D2V9", 300, 5, seed=4, solid_fraction=0.1)
    sim = gpu_sim(wl)
    before = sim.get_state().clone()
    sim.step(0)
    assert torch.equal(sim.get_state(), before)
    empty = torch.empty(0, dtype=torch.float64, device="cuda")
    assert lbm.density_from_mu(empty).numel() == 0 and lbm.mu_from_density(empty).numel() == 0


# (lattice, nx, ny, nz): Q * (N + 1024) just below 2^31 (N a multiple of 256)
LIMIT = [("D2V9", 16384, 14560, 1), ("D3V19", 512, 512, 431)]


@pytest.mark.parametrize("lattice,nx,ny,nz", LIMIT)
def test_grid_at_size_limit(lattice, nx, ny, nz):
    N = nx * ny * nz
    Q = 9 if lattice == "D2V9" else 19
    sizes = lbm.buffer_sizes(lbm.make_params(lattice, nx, ny, nz))
    assert Q * sizes["stride"] < 2 ** 31 and Q * (sizes["stride"] + 256) >= 2 ** 31 - 2 ** 20
    D = 2 if lattice == "D2V9" else 3
    E = np.array([2e-6, -1e-6, 5e-7 if D == 3 else 0.0])
    B = np.array([0, 0, 1e-3]) if D == 2 else np.array([5e-4, -1e-3, 1e-3])
    rng = np.random.default_rng(6)
    wl = W.Workload("limit", lattice, nx, ny, nz, tau=0.7, steps=20, E=tuple(E), B=tuple(B),
                    rho=1.0 + 0.01 * rng.standard_normal(N))
    sim = gpu_sim(wl)
    t0 = sim.current()
    M, P = t0[0], np.array(t0[1:])
    sim.step(wl.steps)
    t1 = sim.current()
    for _ in range(wl.steps):
        P = P + M * E + np.cross(P, B)
    assert abs(t1[0] / M - 1) < 1e-6
    np.testing.assert_allclose(np.array(t1[1:1 + D]), P[:D], rtol=2e-4, atol=1e-4 * np.abs(P).max())
    rho, u = gpu_fields(sim)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    last = (nx - 1, ny - 1, nz - 1)
    for centre in ((0, 0, 0), last, (nx // 2, ny - 3, nz // 2)):
        glob, rho_o, u_o = oracle_window_fields(wl, wl.steps, 8, centre)
        er, eu = rel_errors(rho[glob], u[:, glob], rho_o, u_o)
        assert er < 1e-5 and eu < 1e-5, (centre, er, eu)
