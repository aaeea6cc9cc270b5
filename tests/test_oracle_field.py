"""Pins of the oracle's whole-grid step: streaming, walls, conservation and the exact
momentum recurrence of a periodic box.

Streaming is checked against numpy's periodic shift (np.roll) on states where the
collision is the identity; walls against the halfway bounce-back rule written with
array masks; the whole step against closed forms of the total momentum.
"""
import numpy as np
import pytest

from oracle.oracle import OracleModel
from paper_1710_09472_amd import workloads as W

RNG = np.random.default_rng(2024)


def _grid_shape(m):
    return (m.nz, m.ny, m.nx)


def _local_eq_state(m, seed, mask=None):
    wl = W.random_fields(m.lattice, m.nx, m.ny, m.nz, seed=seed)
    return m.init_state(wl.rho, wl.u, mask)


@pytest.mark.parametrize("lattice,shape", [("D2V9", (7, 5, 1)), ("D3V19", (5, 4, 3))])
def test_streaming_matches_roll(lattice, shape):
    """With f = f^eq(rho(x), u(x)) and no force the collision is the identity, so one
    step is pure streaming: f_a(x + e_a) = f_a(x), periodic."""
    m = OracleModel(lattice, *shape, tau=0.77)
    f0 = _local_eq_state(m, 1)
    f1 = m.step(f0)
    g0 = f0.reshape((m.Q,) + _grid_shape(m))
    g1 = f1.reshape((m.Q,) + _grid_shape(m))
    for a in range(m.Q):
        ex, ey, ez = m.e[a]
        want = np.roll(g0[a], shift=(ez, ey, ex), axis=(0, 1, 2))
        np.testing.assert_allclose(g1[a], want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lattice,shape", [("D2V9", (7, 6, 1)), ("D3V19", (5, 4, 4))])
def test_bounce_back_rule(lattice, shape):
    """Halfway bounce-back: a population whose destination x + e_a is solid arrives at
    x in the opposite direction; every other one moves to x + e_a. Solid nodes hold 0."""
    m = OracleModel(lattice, *shape, tau=0.77)
    mask = (RNG.uniform(size=m.N) < 0.25).astype(np.uint8)
    f0 = _local_eq_state(m, 2, mask)
    f1 = m.step(f0, mask)
    G = _grid_shape(m)
    g0 = f0.reshape((m.Q,) + G)
    g1 = f1.reshape((m.Q,) + G)
    solid = mask.reshape(G).astype(bool)
    for a in range(m.Q):
        ex, ey, ez = m.e[a]
        moved = np.roll(g0[a] * ~solid, shift=(ez, ey, ex), axis=(0, 1, 2))
        # population a at x comes from x - e_a if that is fluid
        src_solid = np.roll(solid, shift=(ez, ey, ex), axis=(0, 1, 2))
        # ... or, if x - e_a is solid, from x's own opposite population
        bounced = g0[m.opp[a]]
        want = np.where(src_solid, bounced, moved)
        want[solid] = 0.0
        np.testing.assert_allclose(g1[a], want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("lattice,shape", [("D2V9", (9, 7, 1)), ("D3V19", (6, 5, 4))])
def test_translation_equivariance(lattice, shape):
    m = OracleModel(lattice, *shape, tau=0.65, E=(1e-3, 2e-4, 1e-4 if lattice == "D3V19" else 0),
                    B=(0, 0, 5e-3))
    wl = W.random_fields(lattice, *shape, seed=3, solid_fraction=0.2, soft=True)
    f0 = m.init_state(wl.rho, wl.u, wl.mask)
    out = m.run(f0, 5, wl.mask, wl.s)
    sh = (1, 2, 3)[: 3]
    G = _grid_shape(m)
    roll = lambda a, comp: np.roll(a.reshape(((comp,) if comp else ()) + G), shift=(sh[2] % m.nz, sh[1], sh[0]),
                                   axis=(-3, -2, -1)).reshape(-1)
    f0s = roll(f0, m.Q)
    outs = m.run(f0s, 5, roll(wl.mask, 0), roll(wl.s, 0))
    np.testing.assert_allclose(outs, roll(out, m.Q), rtol=0, atol=1e-15)


@pytest.mark.parametrize("lattice,shape", [("D2V9", (12, 10, 1)), ("D3V19", (8, 6, 5))])
def test_mass_conservation_walls_and_partial_bb(lattice, shape):
    m = OracleModel(lattice, *shape, tau=0.6, E=(2e-3, 1e-3, 0), B=(0, 0, 2e-3))
    wl = W.random_fields(lattice, *shape, seed=4, solid_fraction=0.2, soft=True)
    f = m.init_state(wl.rho, wl.u, wl.mask)
    M0 = m.totals(f, wl.mask)[0]
    f = m.run(f, 200, wl.mask, wl.s)
    assert abs(m.totals(f, wl.mask)[0] / M0 - 1) < 1e-13


@pytest.mark.parametrize("lattice,shape", [("D2V9", (16, 12, 1)), ("D3V19", (8, 6, 5))])
def test_momentum_recurrence_periodic(lattice, shape):
    """Periodic box, no solids: collision adds rho (E + u x B) per node and streaming
    keeps totals, so P_(t+1) = P_t + M E + P_t x B exactly (M = total mass)."""
    D = 2 if lattice == "D2V9" else 3
    E = np.array([1e-4, -3e-5, 2e-5 if D == 3 else 0.0])
    B = np.array([2e-3, -1e-3, 3e-3]) if D == 3 else np.array([0, 0, 3e-3])
    m = OracleModel(lattice, *shape, tau=0.7, E=E, B=B)
    wl = W.random_fields(lattice, *shape, seed=5, umax=0.01)
    f = m.init_state(wl.rho, wl.u)
    t = m.totals(f)
    M, P = t[0], t[1:].copy()
    T = 1000
    f = m.run(f, T)
    for _ in range(T):
        P = P + M * E + np.cross(P, B)
    got = m.totals(f)[1:]
    assert abs(m.totals(f)[0] / M - 1) < 1e-12  # FP64 rounding over 1000 steps
    np.testing.assert_allclose(got[:D], P[:D], rtol=1e-11, atol=1e-13 * np.abs(P).max())


@pytest.mark.parametrize("lattice,shape", [("D2V9", (10, 8, 1)), ("D3V19", (6, 5, 4))])
def test_uniform_partial_bounce_back_recurrence(lattice, shape):
    """Uniform s on a periodic box: P_(t+1) = (1 - 2s) P_t + (1 - s) M E, so
    P_T = (1-2s)^T P_0 + (1 - s) M E (1 - (1-2s)^T) / (2s)."""
    s = 0.15
    E = np.array([2e-4, -1e-4, 5e-5 if lattice == "D3V19" else 0.0])
    m = OracleModel(lattice, *shape, tau=0.75, E=E)
    wl = W.random_fields(lattice, *shape, seed=6, umax=0.01)
    f = m.init_state(wl.rho, wl.u)
    t = m.totals(f)
    M, P0 = t[0], t[1:]
    T = 60
    f = m.run(f, T, s=np.full(m.N, s))
    q = (1 - 2 * s) ** T
    want = q * P0 + (1 - s) * M * E * (1 - q) / (2 * s)
    np.testing.assert_allclose(m.totals(f)[1:], want, rtol=1e-12, atol=1e-15)
