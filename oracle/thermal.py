"""Oracle of the fourth-order (K = 4) thermal model on the D1V7 lattice.

TEST INFRASTRUCTURE ONLY. Part of the CPU oracle (see oracle/oracle.py): only the tests,
the package smoke check and the benchmark's CPU-baseline leg may import it; the GPU
product path never does. The step is plain numpy FP64; constants and the state function
g come from mpmath.

What is computed (Coelho & Doria, "Lattice Boltzmann method for semiclassical fluids"):

* The equilibrium expanded to fourth order in the polynomials orthonormal under the
  weight omega, f^eq = omega sum_(N<=4) (1/N!) A_N P_N with A_N = int f^FD P_N
  (eq. feq-complete-exp-eq, Sec. 3-5; K = 4 is the order that carries the energy
  equation, Sec. 6). It is the orthogonal projection, in the omega-weighted inner
  product, of f^FD / omega onto the polynomials of degree <= 4. In one dimension it is
  therefore omega p for the polynomial p whose weighted moments match those of the local
  distribution, int omega p xi^k = M_k for k = 0..4, with
      M_0 = rho, M_1 = rho u, M_2 = rho (thetabar + u^2), M_3 = rho (u^3 + 3 u thetabar),
      M_4 = rho (u^4 + 6 u^2 thetabar + 3 thetabar^2 g)
  (eqs. rho-def-eq, vel-def-eq, theta-bar-def-eq, gz-def-eq; the one-dimensional
  isotropic tensor of fourth order is 3) and int omega xi^2n = (2n-1)!! I_2n
  (eq. i2n-cont). (This definition replaces the printed fourth-order expansion, which is
  the same projection written out.)
* The third-order truncation (K = 3, the order that carries the full momentum equation,
  Sec. 6) is the same projection onto degree <= 3: p matches M_0..M_3; M_4 of f^eq is then
  whatever the weight's moments make it, so the energy equation is not the paper's.
* D1V7 (App. A), exact to order 9: f^eq_a = w_a p(xi_a), xi_a = e_a / c_s.
* thetabar and g of the local Fermi-Dirac distribution 1/(z^-1 exp((xi-u)^2/theta) + 1)
  in one dimension: rho = sqrt(pi theta) g_1/2(z), rho thetabar = (sqrt(pi)/2)
  theta^(3/2) g_3/2(z), 3 rho thetabar^2 g = (3 sqrt(pi)/4) theta^(5/2) g_5/2(z), with
  g_nu(z) = -Li_nu(-z) (the Fermi-Dirac integrals of Sec. 9.2, in one dimension). Hence
  thetabar = theta g_3/2 / (2 g_1/2), g = g_5/2 g_1/2 / g_3/2^2, and
  s = rho^2 / thetabar = 2 pi g_1/2^3 / g_3/2 fixes z: g is a function of s alone, defined
  for 0 < s < 12 (s -> 12 is the Fermi ground state, s -> 0 the Boltzmann limit, g -> 1).
* BGK relaxation with Delta t = 1 and periodic streaming on e_a.
* Reading: g is held at the weight's own value, g_0 = I_4 I_0 / I_2^2 (the value of the
  Fermi-Dirac state the weight is), as Sec. 9.1 holds thetabar constant in the isothermal
  model (g_mode "const", the default). With g following the local state (g_mode "state")
  the D1V7 model is linearly unstable in the degenerate regime (largest amplification
  1.07 per step at theta = 1/4, mu = 1, tau = 0.8, tested), stable in the Boltzmann limit;
  with g held it is stable, and its slow thermal mode decays as the paper's energy
  equation with the heat flux Q = -kappa grad thetabar - grad[kappa thetabar (g - 1)]
  (eq. pseudo-heat-flux-eq) predicts.
"""
from __future__ import annotations

import functools

import mpmath as mp
import numpy as np

from . import constants as C


def fd_integral(nu, x):
    """g_nu(e^x) = -Li_nu(-e^x) (mpmath; the imaginary part of rounding is dropped)."""
    return -mp.re(mp.polylog(nu, -mp.exp(x)))


def fd_state(x, theta):
    """(rho, thetabar, g) of the 1D Fermi-Dirac distribution with z = e^x at theta."""
    theta = mp.mpf(theta)
    g1, g3, g5 = fd_integral(mp.mpf(1) / 2, x), fd_integral(mp.mpf(3) / 2, x), fd_integral(mp.mpf(5) / 2, x)
    rho = mp.sqrt(mp.pi * theta) * g1
    return rho, theta * g3 / (2 * g1), g5 * g1 / g3 ** 2


def s_of_x(x):
    """s = rho^2 / thetabar = 2 pi g_1/2(z)^3 / g_3/2(z), z = e^x."""
    g1, g3 = fd_integral(mp.mpf(1) / 2, x), fd_integral(mp.mpf(3) / 2, x)
    return 2 * mp.pi * g1 ** 3 / g3


def g_of_s(s):
    """g of the 1D Fermi-Dirac distribution with rho^2 / thetabar = s (0 < s < 12): the
    root x = ln z of s_of_x(x) = s (bracketed Illinois iteration on ln s, which is
    increasing in x), then g = g_5/2 g_1/2 / g_3/2^2."""
    s = mp.mpf(s)
    if not (0 < s < 12):
        raise ValueError("no Fermi-Dirac state has rho^2 / thetabar outside (0, 12)")
    f = lambda x: mp.log(s_of_x(x)) - mp.log(s)
    a, b = mp.mpf(-2), mp.mpf(2)
    while f(a) > 0:
        a -= 4
    while f(b) < 0:
        b = 2 * b + 2
    x = mp.findroot(f, (a, b), solver="illinois", tol=mp.mpf(10) ** -28, maxsteps=300, verify=False)
    g1, g3, g5 = fd_integral(mp.mpf(1) / 2, x), fd_integral(mp.mpf(3) / 2, x), fd_integral(mp.mpf(5) / 2, x)
    return g5 * g1 / g3 ** 2


class GTable:
    """g as a function of s on the states with ln z in [x_lo, x_hi]: Chebyshev interpolants
    of ln s(x) and g(x) through their values at n Chebyshev points in x (both analytic, so
    the interpolants converge geometrically; the tests hold g to 1e-13 against g_of_s).
    For a given s, x solves ln s(x) = ln s by Newton's method on the interpolant (ln s is
    increasing in x)."""

    def __init__(self, x_lo: float, x_hi: float, n: int = 28):
        self.lo, self.hi = float(x_lo), float(x_hi)
        k = np.arange(n)
        t = np.cos(np.pi * (k + 0.5) / n)
        x = 0.5 * (self.hi + self.lo) + 0.5 * (self.hi - self.lo) * t
        ls, gv = [], []
        with mp.workdps(24):
            for v in x:
                g1, g3, g5 = (fd_integral(mp.mpf(nu) / 2, mp.mpf(v)) for nu in (1, 3, 5))
                ls.append(float(mp.log(2 * mp.pi * g1 ** 3 / g3)))
                gv.append(float(g5 * g1 / g3 ** 2))
        cheb = np.polynomial.chebyshev
        self.cl = cheb.chebfit(t, np.array(ls), n - 1)
        self.cg = cheb.chebfit(t, np.array(gv), n - 1)
        self.dcl = cheb.chebder(self.cl)
        self.s_lo = float(np.exp(cheb.chebval(-1.0, self.cl)))
        self.s_hi = float(np.exp(cheb.chebval(1.0, self.cl)))

    def __call__(self, s):
        cheb = np.polynomial.chebyshev
        s = np.asarray(s, dtype=np.float64)
        if np.any(s < self.s_lo) or np.any(s > self.s_hi):
            raise ValueError(f"s outside the table [{self.s_lo}, {self.s_hi}]")
        target = np.log(s)
        t = np.zeros_like(s)
        for _ in range(60):
            r = cheb.chebval(t, self.cl) - target
            t = np.clip(t - r / cheb.chebval(t, self.dcl), -1.0, 1.0)
            if np.all(np.abs(r) < 1e-15):
                break
        return cheb.chebval(t, self.cg)


@functools.lru_cache(maxsize=None)
def _table(x_lo, x_hi):
    return GTable(x_lo, x_hi)


class ThermalOracle:
    """1D periodic grid of N nodes, D1V7, fourth-order equilibrium, BGK.

    The weight is the Fermi-Dirac one of the given theta, mu (Sec. 9.1 form); its own
    state (rho = I_0, u = 0, thetabar = I_2/I_0) has f^eq = w exactly. States are
    (rho, u, thetabar) per node; populations f[a, n] in the order of D1V7_E."""

    def __init__(self, N: int, tau: float, theta=0.25, mu=1.0, g_mode="const", x_range=(-1.5, 2.0),
                 stats="fd", K=4):
        if K not in (3, 4):
            raise ValueError("K is 3 or 4")
        self.K = int(K)
        k = C.d1v7(stats, theta, mu)
        self.N, self.tau = int(N), float(tau)
        self.cs = float(k["cs"])
        self.e = np.array(C.D1V7_E)
        self.w = np.array([float(k["w"][abs(a)]) for a in C.D1V7_E])
        self.xi = self.e / self.cs
        I = k["I"]
        dfact = {0: 1, 2: 1, 4: 3, 6: 15, 8: 105}  # (2n-1)!!
        mom = {j: (float(I[j]) * dfact[j] if j % 2 == 0 else 0.0) for j in range(9)}
        self.H = np.array([[mom[i + j] for j in range(self.K + 1)] for i in range(self.K + 1)])
        self.rho_ref = float(I[0])
        self.thetabar_ref = float(I[2] / I[0])
        self.s_ref = self.rho_ref ** 2 / self.thetabar_ref
        self.g_ref = float(I[4] * I[0] / I[2] ** 2)
        if g_mode not in ("const", "state") or (g_mode == "state" and stats != "fd"):
            raise ValueError(g_mode)
        self.g_mode = g_mode
        # "state": states with ln z within x_range of the weight's own ln z = mu / theta
        self.x_range = (float(mu) / float(theta) + x_range[0], float(mu) / float(theta) + x_range[1])

    def g(self, rho, thetabar):
        if self.g_mode == "const":
            return np.full(np.shape(rho), self.g_ref)
        return _table(*self.x_range)(rho ** 2 / thetabar)

    def moments_target(self, rho, u, tb, g):
        M = [rho, rho * u, rho * (tb + u * u), rho * (u ** 3 + 3 * u * tb),
             rho * (u ** 4 + 6 * u * u * tb + 3 * tb * tb * g)]
        return np.stack(M[:self.K + 1])

    def equilibrium(self, rho, u, tb, g):
        """f^eq[a, n] = w_a p_n(xi_a), H c_n = M_n (p of degree K)."""
        c = np.linalg.solve(self.H, self.moments_target(rho, u, tb, g))
        V = np.stack([self.xi ** k for k in range(self.K + 1)], axis=1)  # [a, k]
        return self.w[:, None] * (V @ c)

    def macro(self, f):
        rho = f.sum(0)
        u = (f * self.xi[:, None]).sum(0) / rho
        tb = (f * self.xi[:, None] ** 2).sum(0) / rho - u * u
        return rho, u, tb

    def init_state(self, rho, u, tb):
        rho, u, tb = (np.asarray(a, dtype=np.float64) for a in (rho, u, tb))
        return self.equilibrium(rho, u, tb, self.g(rho, tb))

    def step(self, f):
        rho, u, tb = self.macro(f)
        feq = self.equilibrium(rho, u, tb, self.g(rho, tb))
        post = f - (f - feq) / self.tau
        return np.stack([np.roll(post[a], self.e[a]) for a in range(7)])

    def run(self, f, steps: int):
        for _ in range(steps):
            f = self.step(f)
        return f

    def totals(self, f):
        """(sum rho, sum rho u, sum of the second moment sum_a f xi^2) over the grid."""
        return f.sum(), (f * self.xi[:, None]).sum(), (f * self.xi[:, None] ** 2).sum()
