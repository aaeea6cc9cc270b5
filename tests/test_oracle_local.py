"""Pins of the oracle's per-node arithmetic: equilibrium, Lorentz source, collision.

The equilibrium is checked against its moments (Sec. 6), against the direct N = 2
derivation of Sec. 5.1 (a second route to the same function), against the unreduced
form of Sec. 9.1 and against the textbook D2Q9 equilibrium in the Hermite limit. The
source is checked against its moment constraints (Sec. 7) and against a numerical
derivative of the equilibrium. The collision is checked against its invariants.
"""
import numpy as np
import pytest

from oracle.oracle import OracleModel

RNG = np.random.default_rng(12345)


def _model(lattice, stats="fd", E=(0, 0, 0), B=(0, 0, 0), tau=0.8):
    return OracleModel(lattice, 3, 3, 1 if lattice == "D2V9" else 3, tau=tau, E=E, B=B, stats=stats)


def _moments(m, f):
    M0 = f.sum()
    M1 = (f[:, None] * m.xi).sum(0)
    M2 = np.einsum("a,ai,aj->ij", f, m.xi, m.xi)
    return M0, M1, M2


LATTICES = ["D2V9", "D3V19"]


@pytest.mark.parametrize("lattice", LATTICES)
def test_equilibrium_moments(lattice):
    """sum f^eq = rho, sum f^eq xi = rho u, sum f^eq xi xi = rho (thetabar delta + u u)
    (moments of Sec. 6, eq. (moments-non-expanded-edf-eq), with thetabar = I_2/I_0)."""
    m = _model(lattice)
    D = m.D
    thb = float(m.coef.thetabar)
    for _ in range(20):
        rho = RNG.uniform(0.5, 2.0)
        u = RNG.uniform(-0.1, 0.1, D)
        feq = m.equilibrium(rho, u)
        M0, M1, M2 = _moments(m, feq)
        assert abs(M0 - rho) < 1e-14 * rho
        np.testing.assert_allclose(M1[:D], rho * u, rtol=0, atol=1e-15)
        want = rho * (thb * np.eye(3) + np.outer(np.r_[u, [0] * (3 - D)], np.r_[u, [0] * (3 - D)]))
        np.testing.assert_allclose(M2[:D, :D], want[:D, :D], rtol=0, atol=2e-15)


@pytest.mark.parametrize("lattice", LATTICES)
def test_equilibrium_direct_route(lattice):
    """Sec. 5.1, eq. (feq-reduce-general-method-without-pol-eq): the N = 2 equilibrium
    written directly in I_0, I_2, I_4 (no polynomials), with w_a in place of omega."""
    m = _model(lattice)
    k = m.coef
    I0, I2, I4, D2 = float(k.I0), float(k.I2), float(k.I4), float(k.Delta2) ** 2
    D = m.D
    for _ in range(20):
        rho = RNG.uniform(0.5, 2.0)
        u = RNG.uniform(-0.1, 0.1, D)
        xu = m.xi[:, :D] @ u
        xi2 = (m.xi ** 2).sum(1)
        u2 = u @ u
        direct = rho / I0 * m.w * (1 + I0 / I2 * xu + I0 / I4 * 0.5 * xu ** 2 +
                                   0.5 * u2 * (I0 / I4 * (D2 - 1) / D * xi2 - I2 / I4 * D2))
        np.testing.assert_allclose(m.equilibrium(rho, u), direct, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("lattice", LATTICES)
def test_equilibrium_unreduced_form(lattice):
    """The unreduced discrete EDF of Sec. 9.1 (eq. (feq-exp-2nd-order-eq)) with
    thetabar = I_2/I_0 equals the reduced one the model uses."""
    m = _model(lattice)
    k = m.coef
    c0, c1, c2, cb, cp, th = (float(v) for v in (k.c0, k.c1, k.c2, k.c2bar, k.c2p, k.thetabar))
    D = m.D
    for _ in range(10):
        rho = RNG.uniform(0.5, 2.0)
        u = RNG.uniform(-0.1, 0.1, D)
        xu = m.xi[:, :D] @ u
        xi2 = (m.xi ** 2).sum(1)
        u2 = u @ u
        full = rho * m.w * (c0 ** 2 + c1 ** 2 * xu + 0.5 * c2 * (c2 * th + cp) * xi2 + 0.5 * c2 ** 2 * xu ** 2
                            + 0.5 * c2 * cb * (D * th + u2) * xi2
                            + 0.5 * (cb * xi2 + cp) * (D * (c2 * th + cp) + c2 * u2 + D * cb * (D * th + u2)))
        np.testing.assert_allclose(m.equilibrium(rho, u), full, rtol=1e-12, atol=1e-15)


def test_equilibrium_hermite_textbook():
    """Hermite weight: the model reduces to the textbook D2Q9 equilibrium
    w rho (1 + 3 e.v + 9/2 (e.v)^2 - 3/2 v^2) in lattice velocity v = c_s u."""
    m = _model("D2V9", stats="hermite")
    np.testing.assert_allclose(m.w[np.argsort((m.e ** 2).sum(1), kind="stable")][[0, 1, 5]],
                               [4 / 9, 1 / 9, 1 / 36], rtol=1e-14)
    for _ in range(10):
        rho = RNG.uniform(0.5, 2.0)
        v = RNG.uniform(-0.05, 0.05, 2)
        u = v / m.cs
        ev = m.e[:, :2] @ v
        text = m.w * rho * (1 + 3 * ev + 4.5 * ev ** 2 - 1.5 * (v @ v))
        np.testing.assert_allclose(m.equilibrium(rho, u), text, rtol=1e-13)


@pytest.mark.parametrize("lattice", LATTICES)
@pytest.mark.parametrize("field", ["E", "B", "EB"])
def test_source_moment_constraints(lattice, field):
    """Sec. 7, eqs. (force-eq1)-(force-eq3) with the sign reading S = +a.grad_u f^eq:
    sum S = 0, sum S xi = rho (E + u x B), sum S xi xi = rho (u E + E u) (the magnetic
    part of the second moment vanishes)."""
    D = 2 if lattice == "D2V9" else 3
    E = RNG.uniform(-1e-2, 1e-2, 3) if "E" in field else np.zeros(3)
    B = RNG.uniform(-1e-2, 1e-2, 3) if "B" in field else np.zeros(3)
    if D == 2:
        E[2] = 0
        B[:2] = 0
    m = _model(lattice, E=E, B=B)
    for _ in range(10):
        rho = RNG.uniform(0.5, 2.0)
        u = np.zeros(3)
        u[:D] = RNG.uniform(-0.1, 0.1, D)
        S = m.source(rho, u[:D])
        M0, M1, M2 = _moments(m, S)
        assert abs(M0) < 1e-16
        np.testing.assert_allclose(M1[:D], (rho * (E + np.cross(u, B)))[:D], rtol=0, atol=1e-16)
        want = rho * (np.outer(u, E) + np.outer(E, u))
        np.testing.assert_allclose(M2[:D, :D], want[:D, :D], rtol=0, atol=1e-16)


@pytest.mark.parametrize("lattice", LATTICES)
def test_source_is_directional_derivative(lattice):
    """S_a = a_a . grad_u f^eq_a (Sec. 7): compare with a central difference of the
    oracle's own equilibrium along a_a = E + xi_a x B. f^eq is quadratic in u, so the
    central difference is exact up to rounding."""
    D = 2 if lattice == "D2V9" else 3
    E = np.array([3e-3, -2e-3, 1e-3]) if D == 3 else np.array([3e-3, -2e-3, 0])
    B = np.array([1e-3, 2e-3, -4e-3]) if D == 3 else np.array([0, 0, -4e-3])
    m = _model(lattice, E=E, B=B)
    rho = 1.3
    u = np.zeros(3)
    u[:D] = [0.03, -0.02, 0.01][:D]
    S = m.source(rho, u[:D])
    h = 1e-3
    for a in range(m.Q):
        acc = E + np.cross(m.xi[a], B)
        fp = m.equilibrium(rho, (u + h * acc)[:D])[a]
        fm = m.equilibrium(rho, (u - h * acc)[:D])[a]
        assert abs((fp - fm) / (2 * h) - S[a]) < 1e-12, a


@pytest.mark.parametrize("lattice", LATTICES)
def test_collision_invariants(lattice):
    """Discrete BGK with source conserves mass and gains momentum rho (E + u x B)."""
    D = 2 if lattice == "D2V9" else 3
    E = np.array([1e-3, -2e-3, 5e-4]) if D == 3 else np.array([1e-3, -2e-3, 0])
    B = np.array([2e-3, -1e-3, 3e-3]) if D == 3 else np.array([0, 0, 3e-3])
    m = _model(lattice, E=E, B=B, tau=0.7)
    for _ in range(10):
        f = m.w * RNG.uniform(0.8, 1.2, m.Q) / float(m.coef.I0)
        rho, u = m.node_moments(f)
        uu = np.zeros(3)
        uu[:D] = u
        g = m.collide_node(f)
        d0, d1, _ = _moments(m, g - f)
        assert abs(d0) < 1e-15
        np.testing.assert_allclose(d1[:D], (rho * (E + np.cross(uu, B)))[:D], rtol=0, atol=1e-15)


@pytest.mark.parametrize("lattice", LATTICES)
def test_collision_relaxation_and_partial_bounce_back(lattice):
    """Without force: f* - f^eq = (1 - 1/tau)(f - f^eq) exactly; at equilibrium the
    collision is the identity; partial bounce-back with s mixes in the reversed
    pre-collision populations and keeps the mass."""
    m = _model(lattice, tau=0.9)
    f = m.w * RNG.uniform(0.8, 1.2, m.Q) / float(m.coef.I0)
    rho, u = m.node_moments(f)
    feq = m.equilibrium(rho, u)
    g = m.collide_node(f)
    np.testing.assert_allclose(g - feq, (1 - 1 / 0.9) * (f - feq), rtol=0, atol=1e-16)
    np.testing.assert_allclose(m.collide_node(feq), feq, rtol=0, atol=1e-16)
    s = 0.3
    gs = m.collide_node(f, s)
    np.testing.assert_allclose(gs, (1 - s) * g + s * f[m.opp], rtol=0, atol=1e-16)
    assert abs(gs.sum() - f.sum()) < 1e-15
