"""Pins of the oracle's constants (weight integrals, coefficients, lattice weights).

Each check ties oracle/constants.py to something other than itself: the values the
paper prints, closed forms of the Fermi-Dirac integrals, the Hermite limit, the
quadrature equations and the orthonormality of the polynomials.
"""
import itertools
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import constants as K

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, txt = line.split()
            decimals = len(txt.split(".")[1])
            vals[key] = (mp.mpf(txt), mp.mpf(10) ** (-decimals))
    return vals


@pytest.mark.parametrize("D,lattice,fname", [(2, "D2V9", "paper_constants_2d.txt"),
                                             (3, "D3V19", "paper_constants_3d.txt")])
def test_printed_tables(D, lattice, fname):
    """Sec. 9.1.1 / 9.1.2 tables: agreement to within one unit of the last printed
    digit (24 decimals). One printed value (3D cbar_2) is truncated rather than rounded
    in its last digit, so the bound is one unit, not half a unit."""
    gold = _read_golden(fname)
    k = K.coefficients(D)
    lw = K.lattice_weights(lattice)
    ours = {"c0": k.c0, "c1": k.c1, "c2": k.c2, "c2bar": k.c2bar, "c2p": k.c2p,
            "thetabar": k.thetabar, "w0": lw["w"][0], "ws": lw["w"][1], "wl": lw["w"][2],
            "cs": lw["cs"]}
    for key, (val, ulp) in gold.items():
        assert abs(ours[key] - val) <= ulp, (key, ours[key], val)


def test_2d_integrals_closed_form():
    """For D = 2 the radial integral reduces to complete Fermi-Dirac integrals of
    integer order: I_2N = -pi theta^(N+1) Li_(N+1)(-e^(mu/theta)) / 2^N (substitute
    t = xi^2 in eq. (i2n-cont2)). Also the Sommerfeld forms of Sec. 9.1.1:
    I_0 = pi theta ln(1 + e^(mu/theta)) ~ pi mu."""
    theta = mp.mpf(1) / 270
    for twoN in (0, 2, 4, 6):
        N = twoN // 2
        closed = -mp.pi * theta ** (N + 1) * mp.polylog(N + 1, -mp.exp(1 / theta)) / 2 ** N
        got = K.weight_integral(2, twoN)
        assert abs(got / closed - 1) < mp.mpf("1e-30"), (twoN, got, closed)
    assert abs(K.weight_integral(2, 0) - mp.pi * theta * mp.log(1 + mp.exp(1 / theta))) < mp.mpf("1e-30")
    # Sommerfeld for D = 2 terminates: I_2 = (pi/4)(1 + pi^2 theta^2 / 3), I_4 = (pi/24)(1 + pi^2 theta^2)
    assert abs(K.weight_integral(2, 2) - mp.pi / 4 * (1 + mp.pi ** 2 * theta ** 2 / 3)) < mp.mpf("1e-30")
    assert abs(K.weight_integral(2, 4) - mp.pi / 24 * (1 + mp.pi ** 2 * theta ** 2)) < mp.mpf("1e-30")


def test_3d_integrals_sommerfeld():
    """D = 3: the Sommerfeld expansion (eq. (sommerfeld-approx-eq), Sec. 9.1) of the
    half-integer Fermi-Dirac integrals, good to ~1e-8 as the paper states."""
    theta = mp.mpf(1) / 270
    eta = 1 / theta
    for twoN in (0, 2, 4):
        N = twoN // 2
        nu = N + mp.mpf(3) / 2
        g = eta ** nu / mp.gamma(nu + 1) * (1 + nu * (nu - 1) * mp.pi ** 2 / 6 / eta ** 2
                                           + nu * (nu - 1) * (nu - 2) * (nu - 3) * 7 * mp.pi ** 4 / 360 / eta ** 4)
        # I_2N = pi^(3/2) theta^(N+3/2) g_(N+3/2)(z) / 2^N for the FD weight in 3D
        approx = mp.pi ** mp.mpf(1.5) * theta ** nu * g / 2 ** N
        got = K.weight_integral(3, twoN)
        assert abs(got / approx - 1) < 1e-8, (twoN, got, approx)


@pytest.mark.parametrize("D", [2, 3])
def test_hermite_limit(D):
    """Hermite weight: I_2N = 1 (eq. (i2n-hermite)); c_K = 1, cbar_K = 0, c'_K = -1;
    standard D2Q9 / D3Q19 weights and c_s = 1/sqrt(3) (Sec. 3, Sec. 8)."""
    for twoN in (0, 2, 4, 6):
        assert abs(K.weight_integral(D, twoN, "hermite") - 1) < 1e-30
    k = K.coefficients(D, "hermite")
    assert abs(k.c0 - 1) < 1e-30 and abs(k.c1 - 1) < 1e-30 and abs(k.c2 - 1) < 1e-30
    assert abs(k.c2bar) < 1e-30 and abs(k.c2p + 1) < 1e-30
    lat = "D2V9" if D == 2 else "D3V19"
    lw = K.lattice_weights(lat, "hermite")
    expect = {0: mp.mpf(4) / 9, 1: mp.mpf(1) / 9, 2: mp.mpf(1) / 36} if D == 2 else \
             {0: mp.mpf(1) / 3, 1: mp.mpf(1) / 18, 2: mp.mpf(1) / 36}
    for key in expect:
        assert abs(lw["w"][key] - expect[key]) < 1e-30
    assert abs(lw["cs"] - 1 / mp.sqrt(3)) < 1e-30


def _delta_tensor(idx):
    """delta_{i1...iM} of Sec. 2: sum over all pairings of products of Kronecker deltas."""
    if not idx:
        return 1
    if len(idx) % 2:
        return 0
    first, rest = idx[0], idx[1:]
    tot = 0
    for k in range(len(rest)):
        if rest[k] == first:
            tot += _delta_tensor(rest[:k] + rest[k + 1:])
    return tot


@pytest.mark.parametrize("lattice,stats", [("D2V9", "fd"), ("D3V19", "fd"), ("D3V15", "fd"),
                                           ("D3V27", "fd"), ("D2V9", "hermite"), ("D3V19", "hermite")])
def test_quadrature_equations(lattice, stats):
    """eq. (quadrature-eq-2), Sec. 8: sum_a w_a xi_a^(i1..iM) = I_M delta_(i1..iM) for
    M <= 5 (all four lattices have order 5 in Table 1). Checked by brute-force sums over
    the lattice vectors, with I_M computed directly from eq. (i2n-cont2)."""
    D = K.LATTICE_DIM[lattice]
    lw = K.lattice_weights(lattice, stats)
    cs = lw["cs"]
    vecs = K.lattice_vectors(lattice)
    w = [lw["w"][sum(c * c for c in v)] for v in vecs]
    assert abs(sum(w) - K.weight_integral(D, 0, stats)) < 1e-28
    for M in range(1, 6):
        IM = K.weight_integral(D, M, stats)
        for idx in itertools.product(range(D), repeat=M):
            s = mp.mpf(0)
            for wa, v in zip(w, vecs):
                p = wa
                for i in idx:
                    p *= mp.mpf(v[i]) / cs
                s += p
            assert abs(s - IM * _delta_tensor(list(idx))) < 1e-25, (M, idx, s)


def test_d3v15_negative_rest_weight():
    """Positivity (Sec. 8) fails for D3V15 under the electron weight, which is why the
    3D model uses D3V19."""
    w0 = K.lattice_weights("D3V15")["w"][0]
    assert w0 < 0 and abs(w0 + mp.mpf("0.3721374148573512")) < 1e-15
    for lat in ("D2V9", "D3V19", "D3V27"):
        assert all(v > 0 for v in K.lattice_weights(lat)["w"].values())


@pytest.mark.parametrize("D", [2, 3])
def test_identities(D):
    """c_2 thetabar + c'_2 + D cbar_2 thetabar = 0 (Sec. 9.1) and
    J_2 Delta_2^2 - (D+2)(Delta_2^2 - 1)/D = 1 (Sec. 7)."""
    k = K.coefficients(D)
    assert abs(k.c2 * k.thetabar + k.c2p + D * k.c2bar * k.thetabar) < 1e-30
    assert abs(k.J2 * k.Delta2 ** 2 - (D + 2) * (k.Delta2 ** 2 - 1) / D - 1) < 1e-30


@pytest.mark.parametrize("D", [2, 3])
def test_orthonormality(D):
    """eq. (omeg-feq), Sec. 3: int omega P_N P_M = delta_NM delta_(i|j) for N, M <= 2,
    with P_0 = c0, P_i = c1 xi_i, P_ij = c2 xi_i xi_j + (cbar2 xi^2 + c'2) delta_ij.
    The integrals are done numerically in polar/spherical coordinates from the radial
    weight, independent of the coefficient formulas."""
    mp.mp.dps = 25
    try:
        k = K.coefficients(D)
        th = mp.mpf(1) / 270
        om = lambda r: 1 / (mp.exp((r * r - 1) / th) + 1)
        pts = K._fermi_edge_points(th, 1)
        # radial moments R_m = int_0^inf omega r^(m + D - 1) dr
        R = {m: mp.quad(lambda r: om(r) * r ** (m + D - 1), pts) + mp.quad(lambda r: om(r) * r ** (m + D - 1), [pts[-1], mp.inf])
             for m in (0, 2, 4)}
        # angular averages of products of unit-vector components, by numeric integration
        cache = {}

        def ang(powers):
            if powers not in cache:
                cache[powers] = ang_raw(powers)
            return cache[powers]

        # Angular part: Gauss-Legendre in cos(theta) and a uniform grid in phi, both
        # exact for the trigonometric polynomials of degree <= 8 that occur here.
        phi = 2 * np.pi * np.arange(32) / 32
        if D == 2:
            def ang_raw(powers):
                v = np.cos(phi) ** powers[0] * np.sin(phi) ** powers[1]
                return mp.mpf(float(v.sum() * 2 * np.pi / 32))
        else:
            ct, wt = np.polynomial.legendre.leggauss(12)
            st = np.sqrt(1 - ct * ct)

            def ang_raw(powers):
                v = (st[:, None] * np.cos(phi)[None, :]) ** powers[0] * \
                    (st[:, None] * np.sin(phi)[None, :]) ** powers[1] * ct[:, None] ** powers[2]
                return mp.mpf(float((wt[:, None] * v).sum() * 2 * np.pi / 32))

        def integral(poly_terms):
            # poly_terms: list of (coef, radial power m, angular powers tuple)
            tot = mp.mpf(0)
            for c, m, pw in poly_terms:
                if c == 0:
                    continue
                tot += c * R[m] * ang(pw)
            return tot

        def unit(i):
            p = [0] * D
            p[i] += 1
            return p

        def P2(i, j):
            # c2 xi_i xi_j + (cbar2 xi^2 + c'2) delta_ij as (coef, radial power, angular powers)
            pw = [0] * D
            pw[i] += 1
            pw[j] += 1
            terms = [(k.c2, 2, tuple(pw))]
            if i == j:
                terms += [(k.c2bar, 2, (0,) * D), (k.c2p, 0, (0,) * D)]
            return terms

        def mul(A, B):
            out = []
            for ca, ma, pa in A:
                for cb, mb, pb in B:
                    out.append((ca * cb, ma + mb, tuple(x + y for x, y in zip(pa, pb))))
            return out

        P0 = [(k.c0, 0, (0,) * D)]
        assert abs(integral(mul(P0, P0)) - 1) < 1e-13
        for i in range(D):
            Pi = [(k.c1, 1, tuple(unit(i)))]
            for j in range(D):
                Pj = [(k.c1, 1, tuple(unit(j)))]
                prod = mul(Pi, Pj)
                assert abs(integral(prod) - (1 if i == j else 0)) < 1e-13
        pairs = [(i, j) for i in range(D) for j in range(i, D)]
        for (i, j) in pairs:
            assert abs(integral(mul(P2(i, j), P0))) < 1e-13
            for (l, m) in pairs:
                want = (1 if (i == l and j == m) else 0) + (1 if (i == m and j == l) else 0)
                got = integral(mul(P2(i, j), P2(l, m)))
                assert abs(got - want) < 1e-13, ((i, j), (l, m), got, want)
    finally:
        mp.mp.dps = 40


# Bose-Einstein parameters for the tests (the paper gives none): fugacity e^(mu/theta).
BE_PARAMS = [(1.0, -0.1), (0.5, -2.0)]


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("stats,theta,mu", [("fd", "1/270", 1.0), ("fd", 0.3, 0.4)] +
                         [("be", t, m) for t, m in BE_PARAMS])
def test_integrals_polylog_closed_form(D, stats, theta, mu):
    """Sec. 2: rho = (2 pi theta')^(D/2) g_(D/2)(z) with g_nu(z) = -Li_nu(-z) (FD) or
    Li_nu(z) (BE); in the xi^2/theta scaling of Sec. 9.1 (theta' = theta/2) the weight
    integrals are I_2N = (theta/2)^N (pi theta)^(D/2) g_(D/2+N)(e^(mu/theta)). mpmath's
    polylog is a route independent of the quadrature."""
    th = mp.mpf(1) / 270 if theta == "1/270" else mp.mpf(theta)
    z = mp.exp(mp.mpf(mu) / th)
    for N in range(3):
        s = mp.mpf(D) / 2 + N
        g = -mp.polylog(s, -z) if stats == "fd" else mp.polylog(s, z)
        want = (th / 2) ** N * (mp.pi * th) ** (mp.mpf(D) / 2) * mp.re(g)
        got = K.weight_integral(D, 2 * N, stats, theta, mu)
        assert abs(got / want - 1) < mp.mpf(10) ** -28, (N, got, want)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("stats", ["fd", "be"])
def test_nondegenerate_limit(D, stats):
    """For z = e^(mu/theta) -> 0 both semiclassical weights tend to the Maxwell-Boltzmann
    Gaussian, whose moments give J_2 = I_2^2/(I_4 I_0) = 1 exactly; the correction is
    O(z) (z = e^-40 here)."""
    k = K.coefficients(D, stats, 1.0, -40.0)
    assert abs(k.J2 - 1) < 1e-16


@pytest.mark.parametrize("lattice", ["D2V9", "D3V19"])
@pytest.mark.parametrize("theta,mu", BE_PARAMS)
def test_bose_einstein_weights_positive(lattice, theta, mu):
    """The quadratures of Sec. 8 need positive weights (true here: J_2 < 1 for BE)."""
    lw = K.lattice_weights(lattice, "be", theta, mu)
    assert all(float(v) > 0 for v in lw["w"].values())
    assert K.coefficients(K.LATTICE_DIM[lattice], "be", theta, mu).J2 < 1


def test_density_mu_2d_closed_forms_and_inverse():
    """Sec. 9.1: in 2D g_1 is elementary, rho = pi theta ln(1 + e^(mu/theta)) (FD, and
    rho ~ pi mu for mu/theta >> 1) and rho = -pi theta ln(1 - e^(mu/theta)) (BE);
    mu_from_density inverts density_from_mu (2D and 3D)."""
    th = mp.mpf(1) / 270
    for mu in (-0.02, 0.3, 1.0):
        r = K.density_from_mu(2, "fd", "1/270", mu)
        assert abs(r / (mp.pi * th * mp.log(1 + mp.exp(mu / th))) - 1) < mp.mpf(10) ** -28
    assert abs(K.density_from_mu(2, "fd", "1/270", 1.0) / mp.pi - 1) < mp.mpf(10) ** -30
    for theta, mu in BE_PARAMS:
        r = K.density_from_mu(2, "be", theta, mu)
        assert abs(r / (-mp.pi * theta * mp.log(1 - mp.exp(mu / mp.mpf(theta)))) - 1) < mp.mpf(10) ** -28
    for D in (2, 3):
        for stats, theta, mu in (("fd", "1/270", 1.0), ("fd", "1/270", 0.05), ("be", 1.0, -0.1), ("be", 0.5, -2.0)):
            r = K.density_from_mu(D, stats, theta, mu)
            back = K.mu_from_density(D, r, stats, theta)
            assert abs(back - mu) < mp.mpf(10) ** -20 * max(1, abs(mu)), (D, stats, mu, back)
