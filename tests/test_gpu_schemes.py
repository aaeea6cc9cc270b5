"""GPU parity of the velocity-shift forcing and the free-slip walls (Sec. 7, 9.3, 9.4)
against the FP64 oracle, through the C ABI.

Bar: FP32 1e-5 relative on rho and u over fluid nodes (as for the source forcing), with
obstacles, walls on y (2D) and y, z (3D), ragged tails, E and B; the paper's own Ohm
setups at full size (2D 512x256 for 1000 steps, element-wise; 3D 128^3 for 30 steps,
element-wise); exact plug-flow momentum in a slip channel at full size; the adjoint
refuses these schemes. FP16/BF16 errors are printed and bounded.
"""
import numpy as np
import pytest

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_fields, gpu_sim, oracle_fields, permutation_to_oracle, rel_errors

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = [
    # name, lattice, shape, seed, obstacle fraction, soft, E, B, forcing, slip
    ("d2-shift-slip", "D2V9", (300, 9, 1), 1, 0.1, False, (2e-4, -1e-4, 0), (0, 0, 4e-3), "shift", 1),
    ("d2-source-slip", "D2V9", (257, 7, 1), 2, 0.1, True, (2e-4, 5e-5, 0), (0, 0, 3e-3), "source", 1),
    ("d2-shift-bb", "D2V9", (64, 11, 1), 3, 0.15, True, (1e-4, 0, 0), (0, 0, 0), "shift", 0),
    ("d3-shift-slip-yz", "D3V19", (260, 6, 7), 4, 0.08, True, (1e-4, 3e-5, -2e-5), (2e-3, -1e-3, 3e-3), "shift", 3),
    ("d3-source-slip-y", "D3V19", (33, 7, 5), 5, 0.1, False, (1e-4, 0, 0), (0, 0, 2e-3), "source", 1),
    ("d3-shift-tiny", "D3V19", (5, 3, 3), 6, 0.0, False, (1e-4, 0, 0), (0, 0, 1e-3), "shift", 3),
]


def _case(lattice, shape, seed, phi, soft, E, B, forcing, slip):
    wl = W.random_fields(lattice, *shape, seed=seed, solid_fraction=phi, soft=soft, umax=0.02)
    wl.tau, wl.E, wl.B, wl.forcing, wl.slip = 0.7, E, B, forcing, slip
    if wl.s is not None:
        wl.s = 0.3 * wl.s
    return wl


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_schemes_parity_fields_and_populations(case):
    wl = _case(*case[1:])
    steps = 25
    sim = gpu_sim(wl)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    rho_o, u_o, m, f_o = oracle_fields(wl, steps)
    solid = m._mask(wl.mask)
    solid = np.zeros(m.N, np.uint8) if solid is None else solid
    er, eu = rel_errors(rho, u, rho_o, u_o, solid)
    assert er < TOL and eu < TOL, (er, eu)
    fl = solid == 0
    f_gpu = sim.export_f64().cpu().numpy()
    perm = permutation_to_oracle(sim, m)
    fo = f_o.reshape(m.Q, m.N)
    np.testing.assert_allclose(f_gpu[perm][:, fl], fo[:, fl], rtol=0, atol=2e-6 * np.abs(fo).max())
    assert np.all(rho[~fl] == 0) and np.all(u[:, ~fl] == 0)
    tot, tot_o = sim.current(), m.totals(f_o, wl.mask)
    assert abs(tot[0] / tot_o[0] - 1) < 1e-6


@pytest.mark.parametrize("storage,k", [("f16", 14), ("bf16", 0)])
def test_schemes_16bit_error(storage, k):
    """16-bit storage with slip walls and the shift (solid-slot bounce-back path)."""
    wl = _case(*CASES[3][1:])
    steps = 25
    rho_o, u_o, m, _ = oracle_fields(wl, steps)
    sim = gpu_sim(wl, storage=storage, dev_scale_log2=k)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    er, eu = rel_errors(rho, u, rho_o, u_o, m._mask(wl.mask))
    print(f"{storage}: rho {er:.2e} u {eu:.2e}")
    assert er < (2e-5 if storage == "f16" else 2e-3) and eu < (2e-3 if storage == "f16" else 2e-2), (er, eu)


def test_ohm_paper_2d_full_parity():
    """The paper's 2D Ohm sample (512x256, 64 disks r = 3, slip y, shift, tau 0.9) at a
    field large enough to read in FP32 (E_x = 1e-5), 1000 steps, element-wise."""
    wl = W.ohm_paper_2d(Ex=1e-5)
    steps = 1000
    sim = gpu_sim(wl)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    rho_o, u_o, m, _ = oracle_fields(wl, steps)
    er, eu = rel_errors(rho, u, rho_o, u_o, m._mask(wl.mask))
    print(f"ohm_paper_2d 1000 steps: rho {er:.2e} u {eu:.2e}")
    assert er < TOL and eu < TOL, (er, eu)


def test_ohm_paper_3d_full_parity():
    """The paper's 3D Ohm sample (128^3, 450 balls r = 3, slip y and z, shift, tau 0.9),
    E_x = 1e-5, 30 steps, element-wise over all 2.1M nodes."""
    wl = W.ohm_paper_3d(Ex=1e-5)
    steps = 30
    sim = gpu_sim(wl)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    rho_o, u_o, m, _ = oracle_fields(wl, steps)
    er, eu = rel_errors(rho, u, rho_o, u_o, m._mask(wl.mask))
    print(f"ohm_paper_3d 30 steps: rho {er:.2e} u {eu:.2e}")
    assert er < TOL and eu < TOL, (er, eu)


@pytest.mark.parametrize("lattice,shape,slip", [("D2V9", (4096, 258, 1), 1), ("D3V19", (256, 66, 34), 3)])
def test_slip_plug_flow_full_size(lattice, shape, slip):
    """Uniform fluid between free-slip walls under E_x with the shift: no wall friction,
    so P_x(t) = t M E_x exactly (in FP64 totals of FP32 states) and u stays uniform."""
    wl = W.Workload("plug", lattice, *shape, tau=0.8, steps=400, E=(1e-6, 0, 0),
                    rho=np.ones(shape[0] * shape[1] * shape[2]), forcing="shift", slip=slip)
    sim = gpu_sim(wl)
    M = sim.current()[0]
    sim.step(wl.steps)
    tot = sim.current()
    assert abs(tot[0] / M - 1) < 1e-6
    want = wl.steps * M * wl.E[0]
    assert abs(tot[1] / want - 1) < 2e-5, (tot[1], want)
    rho, u = gpu_fields(sim)
    fl = rho > 0
    assert np.ptp(u[0][fl]) < 1e-4 * np.abs(u[0][fl]).max()
