"""Oracle constants: weight integrals, polynomial coefficients and quadrature weights.

TEST INFRASTRUCTURE ONLY. This module is part of the CPU oracle of the semiclassical
lattice Boltzmann method (Coelho & Doria, "Lattice Boltzmann method for semiclassical
fluids"). Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may import it; the GPU product path never does.

Everything here is computed in arbitrary precision with mpmath (40 significant digits)
and returned as Python floats (or mpf when asked), directly from the paper's
definitions:

* weight functions: Fermi-Dirac electron weight, eq. (weight-func-isotherm-eq) of
  Sec. 9.1; the Bose-Einstein weight of the same form, eq. (be-fd-dist-eq) of Sec. 2
  with u = 0 and the xi^2/theta scaling of Sec. 9.1; Hermite weight,
  eq. (hermite-weight-eq) of Sec. 2;
* density from chemical potential, rho = I_0(theta, mu), and its inverse by root
  finding (Sec. 9.1-9.2: rho = (pi theta)^(D/2) g_(D/2)(e^(mu/theta)));
* weight integrals I_2N: eq. (i2n-cont2) of Sec. 3 (radial form);
* polynomial coefficients c_K, c'_K, cbar_K, Delta_2K, J_2K: the coefficient list
  of Sec. 3 (K <= 2 for the second-order model of Sec. 9; the whole list to K = 4,
  d_4, d'_4 and dbar_4 included, for the fourth-order thermal model);
* pseudo-temperature thetabar = I_2/I_0: Sec. 9.1;
* reference speed c_s and weights w_alpha of D2V9, D3V15, D3V19, D3V27: Sec. 8 and
  Table 1 (lattices-tab); D1V7: App. A (quadrature equations to order 9, their printed
  solution, and the printed closed-form root of the c_s equation).

No blocking, caching trick or reformulation is applied beyond what those formulas say.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import mpmath as mp

mp.mp.dps = 40

#: Lattices whose weights Table 1 gives in closed form in terms of I_0, I_2, I_4 (, I_6).
LATTICE_DIM = {"D2V9": 2, "D3V15": 3, "D3V19": 3, "D3V27": 3}

#: D1V7 (App. A): e = 0, +1, -1, +2, -2, +3, -3 in the paper's order.
D1V7_E = (0, 1, -1, 2, -2, 3, -3)


def _omega(stats: str, theta, mu, D: int):
    """Radial weight function omega(xi).

    * "fd": eq. (weight-func-isotherm-eq), Sec. 9.1: 1 / (exp((xi^2 - mu)/theta) + 1);
      with theta = 1/270, mu = 1 this is 1/(e^-270 e^(270 xi^2) + 1).
    * "be": the Bose-Einstein form, 1 / (exp((xi^2 - mu)/theta) - 1), mu < 0 (z < 1).
    * "hermite": eq. (hermite-weight-eq), Sec. 2: (2 pi)^(-D/2) exp(-xi^2/2).
    """
    theta = mp.mpf(theta)
    mu = mp.mpf(mu)
    if stats == "fd":
        return lambda x: 1 / (mp.exp((x * x - mu) / theta) + 1)
    if stats == "be":
        if mu >= 0:
            raise ValueError("the Bose-Einstein weight needs mu < 0")
        return lambda x: 1 / mp.expm1((x * x - mu) / theta)
    if stats == "hermite":
        pref = (2 * mp.pi) ** (-mp.mpf(D) / 2)
        return lambda x: pref * mp.exp(-x * x / 2)
    raise ValueError(f"unknown statistics {stats!r}")


def _fermi_edge_points(theta, mu):
    """Break points for the quadrature: the FD weight drops from 1 to 0 within a few
    theta of xi^2 = mu, so the interval is split every 5 theta across the edge
    (xi^2 = mu - 100 theta ... mu + 200 theta)."""
    theta = mp.mpf(theta)
    mu = mp.mpf(mu)
    pts = [mp.mpf(0)]
    for k in range(-100, 201, 5):
        x2 = mu + k * theta
        if x2 > 0:
            pts.append(mp.sqrt(x2))
    return sorted(set(pts))


@functools.lru_cache(maxsize=None)
def weight_integral(D: int, twoN: int, stats: str = "fd", theta="1/270", mu=1.0) -> mp.mpf:
    """I_{2N} of eq. (i2n-cont2), Sec. 3:

        I_2N = pi^(D/2) / (2^(N-1) Gamma(N + D/2)) * int_0^inf omega(xi) xi^(2N+D-1) dxi.

    ``twoN`` is the even order 2N. ``theta`` may be given as a float or as the string
    "1/270" for the exact rational used by the paper's electron model.
    """
    if twoN % 2:
        return mp.mpf(0)  # odd moments vanish by symmetry (Sec. 3)
    N = twoN // 2
    th = mp.mpf(1) / 270 if theta == "1/270" else mp.mpf(theta)
    w = _omega(stats, th, mu, D)
    pref = mp.pi ** (mp.mpf(D) / 2) / (mp.mpf(2) ** (N - 1) * mp.gamma(N + mp.mpf(D) / 2))
    f = lambda x: w(x) * x ** (2 * N + D - 1)
    if stats == "fd":
        pts = _fermi_edge_points(th, mu)
        val = mp.quad(f, pts) + mp.quad(f, [pts[-1], mp.inf])
    elif stats == "be":
        # the BE weight varies on the scales sqrt(|mu|) (near 0) and sqrt(theta)
        sc = sorted({mp.sqrt(abs(mp.mpf(mu))), mp.sqrt(th)})
        pts = [mp.mpf(0)] + [c * k for c in sc for k in (mp.mpf(1) / 4, 1, 4)] + [mp.sqrt(th) * 16]
        pts = sorted(set(pts))
        val = mp.quad(f, pts) + mp.quad(f, [pts[-1], mp.inf])
    else:
        val = mp.quad(f, [0, 1, 3, 6, 12, mp.inf])
    return pref * val


@dataclass(frozen=True)
class Coefficients:
    """Second-order polynomial coefficients and derived quantities (Sec. 3, Sec. 9.1)."""

    D: int
    I0: mp.mpf
    I2: mp.mpf
    I4: mp.mpf
    I6: mp.mpf
    c0: mp.mpf
    c1: mp.mpf
    c2: mp.mpf
    c2bar: mp.mpf
    c2p: mp.mpf
    J2: mp.mpf
    Delta2: mp.mpf
    thetabar: mp.mpf
    cs: mp.mpf


@functools.lru_cache(maxsize=None)
def coefficients(D: int, stats: str = "fd", theta="1/270", mu=1.0) -> Coefficients:
    """Coefficient list of Sec. 3 for K <= 2 and the reference speed of Sec. 8.

    c_K = I_2K^(-1/2); J_2 = I_2^2/(I_4 I_0); Delta_2 = sqrt(2/((D+2) - J_2 D));
    cbar_2 = c_2 (Delta_2 - 1)/D; c'_2 = -c_2 (I_2/I_0) Delta_2;
    thetabar = I_2/I_0 (Sec. 9.1); c_s = sqrt(I_2/(3 I_4)) (Sec. 8, Table 1).
    """
    I0 = weight_integral(D, 0, stats, theta, mu)
    I2 = weight_integral(D, 2, stats, theta, mu)
    I4 = weight_integral(D, 4, stats, theta, mu)
    I6 = weight_integral(D, 6, stats, theta, mu)
    c0 = 1 / mp.sqrt(I0)
    c1 = 1 / mp.sqrt(I2)
    c2 = 1 / mp.sqrt(I4)
    J2 = I2 ** 2 / (I4 * I0)
    Delta2 = mp.sqrt(2 / ((D + 2) - J2 * D))
    c2bar = c2 * (-1 + Delta2) / D
    c2p = -c2 * (I2 / I0) * Delta2
    thetabar = I2 / I0
    cs = mp.sqrt(I2 / (3 * I4))
    return Coefficients(D, I0, I2, I4, I6, c0, c1, c2, c2bar, c2p, J2, Delta2, thetabar, cs)


def lattice_weights(lattice: str, stats: str = "fd", theta="1/270", mu=1.0) -> dict:
    """Quadrature weights by shell |e|^2 (0 rest, 1 axis, 2 face diagonal, 3 body
    diagonal) and c_s, from Sec. 8 (D2V9, D3V15) and Table 1 (D3V19, D3V27).

    Returns {"w": {norm2: w}, "cs": c_s} with mpf values.
    """
    D = LATTICE_DIM[lattice]
    k = coefficients(D, stats, theta, mu)
    I0, I2, I4, I6, J2 = k.I0, k.I2, k.I4, k.I6, k.J2
    if lattice == "D2V9":
        w = {0: I0 * (1 - 5 * J2 / 9), 1: I0 * J2 / 9, 2: I0 * J2 / 36}
    elif lattice == "D3V15":
        w = {0: I0 * (1 - 7 * J2 / 9), 1: I0 * J2 / 9, 3: I0 * J2 / 72}
    elif lattice == "D3V19":
        w = {0: I0 * (1 - 2 * J2 / 3), 1: I0 * J2 / 18, 2: I0 * J2 / 36}
    elif lattice == "D3V27":
        w = {
            0: I0 - 2 * I2 ** 2 / (3 * I4) - I6 * I2 ** 3 / (27 * I4 ** 3),
            1: (3 * I2 ** 2 * I4 ** 2 + I6 * I2 ** 3) / (54 * I4 ** 3),
            2: (3 * I4 ** 2 * I2 ** 2 - I6 * I2 ** 3) / (108 * I4 ** 3),
            3: I2 ** 3 * I6 / (216 * I4 ** 3),
        }
    else:
        raise ValueError(lattice)
    return {"w": w, "cs": k.cs}


def lattice_vectors(lattice: str):
    """Integer lattice vectors e_alpha (Sec. 8, Table 1): all vectors of the listed
    fully symmetric shells. Returned as a list of tuples of length D; the order is the
    oracle's own (rest, then axis, then diagonal shells)."""
    import itertools

    D = LATTICE_DIM[lattice]
    shells = {"D2V9": (0, 1, 2), "D3V15": (0, 1, 3), "D3V19": (0, 1, 2), "D3V27": (0, 1, 2, 3)}[lattice]
    vecs = []
    for n2 in shells:
        for v in itertools.product((-1, 0, 1), repeat=D):
            if sum(c * c for c in v) == n2:
                vecs.append(tuple(v))
    return vecs


def density_from_mu(D: int, stats: str = "fd", theta="1/270", mu=1.0) -> mp.mpf:
    """rho(mu) at fixed theta: the zeroth weight integral, rho = I_0 (Sec. 9.1, the
    relation rho = (pi theta)^(D/2) g_(D/2)(e^(mu/theta)) that sets initial conditions)."""
    return weight_integral(D, 0, stats, theta, mu)


def mu_from_density(D: int, rho, stats: str = "fd", theta="1/270") -> mp.mpf:
    """The inverse of density_from_mu (rho increases with mu) by the Illinois method on a
    bracket, applied to log rho. The bracket starts at the degenerate estimate (D rho Gamma(D/2) /
    (2 pi^(D/2)))^(2/D) for FD (Sommerfeld's leading term) and at the Boltzmann estimate
    theta ln(rho / (pi theta)^(D/2)) for BE, and widens until it changes sign; for BE it
    stays below mu = 0 (no mu exists above the density there, the 3D condensation)."""
    th = mp.mpf(1) / 270 if theta == "1/270" else mp.mpf(theta)
    rho = mp.mpf(rho)
    # in log rho, which is near linear in mu both where rho ~ e^(mu/theta) and where
    # rho ~ mu^(D/2), so the bracketed iteration converges quickly
    g = lambda m: mp.log(weight_integral(D, 0, stats, th, m)) - mp.log(rho)
    if stats == "fd":
        x0 = (D * rho * mp.gamma(mp.mpf(D) / 2) / (2 * mp.pi ** (mp.mpf(D) / 2))) ** (mp.mpf(2) / D)
        a, b, k = x0 - th, x0 + th, 0
        while g(a) > 0:
            k += 1
            a = x0 - th * 2 ** k
        k = 0
        while g(b) < 0:
            k += 1
            b = x0 + th * 2 ** k
    else:
        b = -th * mp.mpf(10) ** -30
        if g(b) <= 0:
            raise ValueError("no mu < 0 gives this density (Bose-Einstein condensation)")
        a = min(th * mp.log(rho / (mp.pi * th) ** (mp.mpf(D) / 2)), -th / 10)
        while g(a) > 0:
            a *= 2
    return mp.findroot(g, (a, b), solver="illinois", tol=mp.mpf(10) ** -32, maxsteps=400, verify=False)


@dataclass(frozen=True)
class Coefficients4:
    """The coefficient list of Sec. 3 up to K = 4 (14 coefficients) and the I_2N used."""

    D: int
    I: dict          # {2N: I_2N}, N = 0..5
    c: dict          # c_K, K = 0..4
    cp: dict         # c'_K, K = 2..4
    cbar: dict       # cbar_K, K = 2..4
    d4: mp.mpf
    d4p: mp.mpf
    d4bar: mp.mpf


@functools.lru_cache(maxsize=None)
def coefficients4(D: int, stats: str = "fd", theta="1/270", mu=1.0) -> Coefficients4:
    """Coefficient list of Sec. 3 to K = 4:

        c_K = I_2K^(-1/2)                                     (K = 0..4)
        c'_K = -c_K (I_(2K-2) / I_(2K-4)) Delta_(2K-2)          (K = 2..4)
        cbar_K = c_K (-1 + Delta_(2K-2)) / (D + 2K - 4)         (K = 2..4)
        Delta_2K = sqrt(2 / ((D + 2K) - J_2K (D + 2K - 2))),  J_2K = I_2K^2 / (I_(2K+2) I_(2K-2))
        d_4^2 = 8 delta_4^2 I_4 / (delta_2 [delta_2 delta_6 (D + 4) - delta_4^2 D])
        d'_4 = -(d_4 / D) [I_0/I_2 + I_4 delta_2 / (I_2 delta_4)] + 2 c_4 I_6 Delta_6 / (D I_4)
        dbar_4 = d_4 delta_2 / (D (D+2) delta_4) + c_4 [D - 2 (D+2) Delta_6] / (D (D+2) (D+4))
        delta_L = 2 I_(L+2) I_(L-2) / Delta_L^2   (Delta_L = Delta_2K for L = 2K).
    The positive root is taken for d_4. Reading: Delta_L with an even index L stands for the
    Delta_2K of the same index, the only one defined."""
    I = {2 * n: weight_integral(D, 2 * n, stats, theta, mu) for n in range(6)}
    c = {K: 1 / mp.sqrt(I[2 * K]) for K in range(5)}
    J = lambda K: I[2 * K] ** 2 / (I[2 * K + 2] * I[2 * K - 2])
    Dl = lambda K: mp.sqrt(2 / ((D + 2 * K) - J(K) * (D + 2 * K - 2)))  # Delta_2K
    cp = {K: -c[K] * I[2 * K - 2] / I[2 * K - 4] * Dl(K - 1) for K in (2, 3, 4)}
    cbar = {K: c[K] * (-1 + Dl(K - 1)) / (D + 2 * K - 4) for K in (2, 3, 4)}
    dl = lambda L: 2 * I[L + 2] * I[L - 2] / Dl(L // 2) ** 2
    d4 = mp.sqrt(8 * dl(4) ** 2 * I[4] / (dl(2) * (dl(2) * dl(6) * (D + 4) - dl(4) ** 2 * D)))
    d4p = -d4 / D * (I[0] / I[2] + I[4] * dl(2) / (I[2] * dl(4))) + 2 * c[4] * I[6] * Dl(3) / (D * I[4])
    d4bar = d4 * dl(2) / (D * (D + 2) * dl(4)) + c[4] * (D - 2 * (D + 2) * Dl(3)) / (D * (D + 2) * (D + 4))
    return Coefficients4(D, I, c, cp, cbar, d4, d4p, d4bar)


@functools.lru_cache(maxsize=None)
def d1v7(stats: str = "fd", theta="1/270", mu=1.0) -> dict:
    """D1V7 of App. A: c_s from the printed closed form (principal branches of the square
    and cube roots), one of the positive roots of 12 I_2 - 49 I_4 c_s^2 + 70 I_6 c_s^4
    - 35 I_8 c_s^6 = 0, and the printed solution of the quadrature equations for w_0..w_3
    (weights of |e| = 0..3). The I_2N are those of eq. (i2n-cont2) with D = 1. Where the
    closed form is not real (its imaginary part is more than rounding: then the principal
    branches have picked a complex root of the cubic) or a weight is not positive, there is
    no D1V7 lattice for this weight: ValueError.

    Returns {"cs", "w": {0: w_0, 1: w_1, 2: w_2, 3: w_3}, "I": {2N: I_2N}} (mpf)."""
    I = {2 * n: weight_integral(1, 2 * n, stats, theta, mu) for n in range(5)}
    I2, I4, I6, I8 = I[2], I[4], I[6], I[8]
    A = -4900 * I6 ** 2 + 5145 * I4 * I8
    B = 686000 * I6 ** 3 - 1080450 * I4 * I6 * I8 + 396900 * I2 * I8 ** 2
    R = mp.cbrt(B + mp.sqrt(mp.mpc(4 * A ** 3 + B ** 2)))
    c2 = 2 * I6 / (3 * I8) - 49 * mp.cbrt(2) * I4 / R + 140 * mp.cbrt(2) * I6 ** 2 / (3 * I8 * R) \
        + R / (105 * mp.cbrt(2) * I8)
    if not (mp.re(c2) > 0) or abs(mp.im(c2)) > mp.mpf(10) ** (-mp.mp.dps // 2) * abs(c2):
        raise ValueError(f"D1V7: the closed form for c_s^2 is not real ({c2}) for this weight")
    cs = mp.sqrt(mp.re(c2))
    y = cs ** 2
    w = {
        0: (360 * I[0] - 150 * I6 * y ** 3 + 420 * I4 * y ** 2 - 490 * I2 * y) / 360,
        1: (-13 * I4 * y ** 2 + 5 * I6 * y ** 3 + 12 * I2 * y) / 16,
        2: (30 * I4 * y ** 2 - 15 * I6 * y ** 3 - 9 * I2 * y) / 120,
        3: (15 * I6 * y ** 3 - 15 * I4 * y ** 2 + 4 * I2 * y) / 720,
    }
    if not all(v > 0 for v in w.values()):
        raise ValueError("D1V7: a quadrature weight is not positive for this weight")
    return {"cs": cs, "w": w, "I": I}
