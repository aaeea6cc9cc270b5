"""rho <-> mu of the semiclassical weights on the GPU (Sec. 9.1-9.2) against the oracle
(mpmath quadrature of I_0 at 40 digits).

Bars: rho(mu) 1e-13 relative; mu of the oracle's rho returns the mu it came from to 1e-12
relative (absolute 1e-13 theta near mu = 0);
round trip over 10^6 values 1e-12; the paper's densities at mu = 1 (rho_2D = pi,
rho_3D = 4.18886...); NaN where no mu exists (BE 3D above the condensation density).
"""
import mpmath as mp
import numpy as np
import pytest
import torch

from oracle import constants as K
from paper_1710_09472_amd import lbm

pytestmark = pytest.mark.gpu

CASES = [
    ("fd-2d", "D2V9", "fd", 1.0 / 270.0, np.concatenate([np.linspace(-20, 300, 9), [0.0, 1e-3]]) / 270.0),
    ("fd-3d", "D3V19", "fd", 1.0 / 270.0, np.concatenate([np.linspace(-20, 300, 9), [0.0, 1e-3]]) / 270.0),
    ("fd-3d-warm", "D3V19", "fd", 0.3, np.array([-2.0, -0.1, 0.0, 0.25, 1.5])),
    ("be-2d", "D2V9", "be", 1.0, np.array([-8.0, -1.0, -0.1, -1e-3])),
    ("be-3d", "D3V19", "be", 1.0, np.array([-8.0, -1.0, -0.1, -1e-3, -1e-6])),
    ("be-3d-cold", "D3V19", "be", 0.5, np.array([-3.0, -0.2, -1e-4])),
]


def _oracle_theta(theta):
    return "1/270" if abs(theta - 1.0 / 270.0) < 1e-18 else theta


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_density_and_inverse_against_oracle(case):
    _, lattice, stats, theta, mus = case
    D = 2 if lattice == "D2V9" else 3
    rho = lbm.density_from_mu(mus, lattice, stats, theta).cpu().numpy()
    th = _oracle_theta(theta)
    # the oracle's mu are the float64 values given to the GPU
    ref = np.array([float(K.density_from_mu(D, stats, th, mp.mpf(float(m)))) for m in mus])
    np.testing.assert_allclose(rho, ref, rtol=1e-13)
    # the inverse of the oracle's rho (rounded once to FP64) is the mu it came from, to
    # 1e-16 relative in rho, i.e. ~1e-16 |mu| (degenerate) or ~1e-16 theta (Boltzmann)
    back = lbm.mu_from_density(ref, lattice, stats, theta).cpu().numpy()
    np.testing.assert_allclose(back, mus, rtol=1e-12, atol=1e-13 * theta)


@pytest.mark.parametrize("lattice,stats,theta,lo,hi", [("D3V19", "fd", 1.0 / 270.0, -0.05, 1.2),
                                                      ("D2V9", "fd", 1.0 / 270.0, -0.05, 1.2),
                                                      ("D3V19", "be", 1.0, -5.0, -1e-4)])
def test_round_trip_million(lattice, stats, theta, lo, hi):
    mu = torch.linspace(lo, hi, 1_000_000, dtype=torch.float64, device="cuda")
    rho = lbm.density_from_mu(mu, lattice, stats, theta)
    back = lbm.mu_from_density(rho, lattice, stats, theta)
    torch.cuda.synchronize()
    err = ((back - mu).abs() / mu.abs().clamp(min=1.0)).max().item()
    assert err < 1e-12, err
    assert torch.all(rho[1:] > rho[:-1])  # rho increases with mu


def test_paper_densities_at_mu_1():
    """Sec. 9.4 prints rho_2D = 3.142, rho_3D = 4.189 at mu = 1; the 2D value is pi up to
    e^-270, the 3D one I_0 of the electron weight."""
    r2 = lbm.density_from_mu([1.0], "D2V9").item()
    r3 = lbm.density_from_mu([1.0], "D3V19").item()
    assert abs(r2 / np.pi - 1) < 1e-15
    assert abs(r3 / float(K.weight_integral(3, 0)) - 1) < 1e-14
    assert round(r2, 3) == 3.142 and round(r3, 3) == 4.189


def test_no_mu_where_none_exists():
    crit = (np.pi * 1.0) ** 1.5 * float(mp.zeta(1.5))  # BE 3D condensation density at theta = 1
    mu = lbm.mu_from_density([0.5 * crit, 1.001 * crit, -1.0, 0.0], "D3V19", "be", 1.0).cpu().numpy()
    assert np.isfinite(mu[0]) and mu[0] < 0 and np.isnan(mu[1:]).all()
    assert np.isnan(lbm.density_from_mu([0.1], "D3V19", "be", 1.0).item())  # BE needs mu < 0
