"""GPU parity under the Bose-Einstein weight (the other semiclassical statistic of the
paper, Sec. 2; parameters theta = 1, mu = -0.1 and theta = 0.5, mu = -2: the paper gives
none). The kernels are the same as for the electron weight; only the constants of
Sec. 3/8/9.1 change. Bar: FP32 1e-5 relative on rho and u against the FP64 oracle.
"""
import numpy as np
import pytest

from oracle.oracle import OracleModel
from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_fields, permutation_to_oracle, rel_errors

pytestmark = pytest.mark.gpu

CASES = [
    ("d2-be", "D2V9", (300, 9, 1), 1.0, -0.1, (2e-4, -1e-4, 0), (0, 0, 3e-3), "source", 0),
    ("d2-be-shift-slip", "D2V9", (130, 8, 1), 0.5, -2.0, (1e-4, 0, 0), (0, 0, 2e-3), "shift", 1),
    ("d3-be", "D3V19", (260, 6, 5), 1.0, -0.1, (1e-4, 3e-5, -2e-5), (1e-3, -2e-3, 3e-3), "source", 0),
    ("d3-be-shift-slip", "D3V19", (40, 7, 6), 0.5, -2.0, (1e-4, 0, 0), (0, 0, 1e-3), "shift", 3),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_bose_einstein_parity(case):
    _, lattice, shape, theta, mu, E, B, forcing, slip = case
    wl = W.random_fields(lattice, *shape, seed=21, solid_fraction=0.1, umax=0.02)
    steps = 25
    sim = lbm.Simulation(lattice, *shape, tau=0.7, E=E, B=B, stats="be", theta=theta, mu=mu, mask=wl.mask,
                         forcing=forcing, slip=slip)
    sim.init(wl.rho, wl.u)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    m = OracleModel(lattice, *shape, tau=0.7, E=E, B=B, stats="be", theta=theta, mu=mu, forcing=forcing, slip=slip)
    f = m.run(m.init_state(wl.rho, wl.u, wl.mask), steps, wl.mask)
    rho_o, u_o = m.moments(f, wl.mask)
    solid = m._mask(wl.mask)
    er, eu = rel_errors(rho, u, rho_o, u_o, solid)
    assert er < 1e-5 and eu < 1e-5, (er, eu)
    fl = solid == 0
    fo = f.reshape(m.Q, m.N)
    f_gpu = sim.export_f64().cpu().numpy()
    perm = permutation_to_oracle(sim, m)
    np.testing.assert_allclose(f_gpu[perm][:, fl], fo[:, fl], rtol=0, atol=2e-6 * np.abs(fo).max())
