"""Python front end of the CPU oracle (plain FP64 C in ``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, the package smoke check and the benchmark's
CPU-baseline leg may import this module. It shares no code with the GPU library and
never imports it. Constants come from :mod:`oracle.constants` (mpmath, from the
paper's formulas); arrays are numpy float64.

State layout: ``f[a, z, y, x]`` flattened as ``f[a*N + n]``, n = x + nx*(y + ny*z),
full populations. The velocity order is the oracle's own (``OracleModel.e``); compare
with other implementations through the vectors, never through the index.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

from . import constants as K

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "lbm_oracle.c"
_LIB = _HERE / "liblbm_oracle.so"

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the shared-library path."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-o", str(tmp),
             str(_SRC), "-lm"],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        build()
        lib = ctypes.CDLL(str(_LIB))
        lib.orc_model_size.restype = ctypes.c_int
        lib.orc_init_model.restype = ctypes.c_int
        lib.orc_run.restype = ctypes.c_int
        lib.orc_get_threads.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def set_threads(n: int) -> None:
    _lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_lib().orc_get_threads())


def _ptr(a, typ=_dp):
    return None if a is None else a.ctypes.data_as(typ)


class OracleModel:
    """One lattice/grid/parameter set of the FP64 oracle.

    ``lattice``: "D2V9" or "D3V19" (the lattices of the paper's electron model,
    Sec. 9.1); ``stats``: "fd" (electron weight, theta = 1/270, mu = 1) or "hermite".
    E and B are accelerations in xi-units per time step.
    """

    def __init__(self, lattice: str, nx: int, ny: int, nz: int = 1, tau: float = 0.8,
                 E=(0.0, 0.0, 0.0), B=(0.0, 0.0, 0.0), stats: str = "fd", theta="1/270",
                 mu: float = 1.0, forcing: str = "source", slip: int = 0):
        self.lattice = lattice
        self.D = K.LATTICE_DIM[lattice]
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        if self.D == 2 and self.nz != 1:
            raise ValueError("2D lattice needs nz = 1")
        self.N = self.nx * self.ny * self.nz
        self.tau = float(tau)
        self.E = tuple(float(v) for v in E)
        self.B = tuple(float(v) for v in B)
        self.coef = K.coefficients(self.D, stats, theta, mu)
        lw = K.lattice_weights(lattice, stats, theta, mu)
        self.w_by_norm2 = {k: float(v) for k, v in lw["w"].items()}
        self.cs = float(lw["cs"])
        self.e = np.array([tuple(v) + (0,) * (3 - self.D) for v in K.lattice_vectors(lattice)],
                          dtype=np.int32)
        self.Q = len(self.e)
        self.w = np.array([self.w_by_norm2[int((v * v).sum())] for v in self.e])
        self.xi = self.e / self.cs
        self.opp = np.array([int(np.nonzero((self.e == -v).all(axis=1))[0][0]) for v in self.e])
        lib = _lib()
        self._m = ctypes.create_string_buffer(lib.orc_model_size())
        coef = np.array([float(self.coef.c0), float(self.coef.c1), float(self.coef.c2),
                         float(self.coef.c2bar), float(self.coef.c2p), self.cs])
        wn = np.array([self.w_by_norm2.get(k, 0.0) for k in range(4)])
        ev = np.ascontiguousarray(self.e, dtype=np.int32)
        rc = lib.orc_init_model(self._m, self.D, self.Q, ev.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                self.nx, self.ny, self.nz, ctypes.c_double(self.tau),
                                _ptr(np.array(self.E)), _ptr(np.array(self.B)), _ptr(coef), _ptr(wn))
        if rc != 0:
            raise RuntimeError("oracle model init failed")
        self._keep = (coef, wn, ev)
        # forcing: "source" (xi-dependent term of Sec. 7) or "shift" (f^eq at u + tau a);
        # slip: free-slip wall planes, bit 0 y in {0, ny-1}, bit 1 z in {0, nz-1}
        self.forcing, self.slip = forcing, int(slip)
        if lib.orc_set_scheme(self._m, {"source": 0, "shift": 1}[forcing], self.slip) != 0:
            raise ValueError("forcing must be 'source' or 'shift'; slip 0..1 (2D) or 0..3 (3D)")
        self.wall = np.zeros(self.N, dtype=np.uint8)
        zz, yy, _ = np.meshgrid(np.arange(self.nz), np.arange(self.ny), np.arange(self.nx), indexing="ij")
        if self.slip & 1:
            self.wall[((yy == 0) | (yy == self.ny - 1)).reshape(-1)] = 1
        if self.slip & 2:
            self.wall[((zz == 0) | (zz == self.nz - 1)).reshape(-1)] = 1

    # ---------------------------------------------------------------- per node
    def node_moments(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = ctypes.c_double()
        u = np.zeros(3)
        _lib().orc_node_moments(self._m, _ptr(f), ctypes.byref(rho), _ptr(u))
        return rho.value, u[: self.D].copy()

    def equilibrium(self, rho, u):
        uu = np.zeros(3)
        uu[: self.D] = u
        out = np.zeros(self.Q)
        _lib().orc_equilibrium(self._m, ctypes.c_double(rho), _ptr(uu), _ptr(out))
        return out

    def source(self, rho, u):
        uu = np.zeros(3)
        uu[: self.D] = u
        out = np.zeros(self.Q)
        _lib().orc_source(self._m, ctypes.c_double(rho), _ptr(uu), _ptr(out))
        return out

    def collide_node(self, f, s=0.0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.Q)
        _lib().orc_collide_node(self._m, _ptr(f), ctypes.c_double(s), _ptr(out))
        return out

    # ---------------------------------------------------------------- fields
    def _mask(self, mask):
        """Solid flags: the obstacles of `mask` and the free-slip wall planes."""
        if mask is None:
            return self.wall.copy() if self.slip else None
        m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
        assert m.size == self.N
        return (m | self.wall) if self.slip else m

    def _s(self, s):
        if s is None:
            return None
        a = np.ascontiguousarray(s, dtype=np.float64).reshape(-1)
        assert a.size == self.N
        return a

    def init_state(self, rho, u=None, mask=None):
        """f = f^eq(rho(x), u(x)); rho shape (N,) or grid, u shape (D, N) or None."""
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        assert rho.size == self.N
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.D, self.N)
        m = self._mask(mask)
        f = np.zeros(self.Q * self.N)
        _lib().orc_init_state(self._m, _ptr(m, _u8p), _ptr(rho), _ptr(uu), _ptr(f))
        return f

    def step(self, f, mask=None, s=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.empty_like(f)
        m, ss = self._mask(mask), self._s(s)
        _lib().orc_step(self._m, _ptr(m, _u8p), _ptr(ss), _ptr(f), _ptr(out))
        return out

    def run(self, f, nsteps, mask=None, s=None):
        f = np.array(f, dtype=np.float64, copy=True)
        m, ss = self._mask(mask), self._s(s)
        rc = _lib().orc_run(self._m, _ptr(m, _u8p), _ptr(ss), _ptr(f), int(nsteps))
        if rc != 0:
            raise MemoryError("oracle run: allocation failed")
        return f

    def moments(self, f, mask=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.zeros(self.N)
        u = np.zeros(self.D * self.N)
        _lib().orc_moments(self._m, _ptr(self._mask(mask), _u8p), _ptr(f), _ptr(rho), _ptr(u))
        return rho, u.reshape(self.D, self.N)

    def totals(self, f, mask=None):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(4)
        _lib().orc_totals(self._m, _ptr(self._mask(mask), _u8p), _ptr(f), _ptr(out))
        return out

    # ---------------------------------------------------------------- adjoint
    def seed_current(self, axis=0, norm=None, mask=None):
        lam = np.zeros(self.Q * self.N)
        _lib().orc_seed_current(self._m, _ptr(self._mask(mask), _u8p), int(axis),
                                ctypes.c_double(float(self.N if norm is None else norm)), _ptr(lam))
        return lam

    def adjoint_step(self, f_t, lam_in, mask=None, s=None, grad_s=None, grad=None):
        """One reverse step. Returns lam_out; accumulates into grad_s (N,) and
        grad (4,) = (dJ/dEx, dJ/dEy, dJ/dEz, dJ/dtau) when given. Both forcings,
        obstacles and free-slip planes (the transpose of the step's streaming)."""
        f_t = np.ascontiguousarray(f_t, dtype=np.float64)
        lam_in = np.ascontiguousarray(lam_in, dtype=np.float64)
        out = np.empty_like(lam_in)
        g = np.zeros(4) if grad is None else grad
        _lib().orc_adjoint_step(self._m, _ptr(self._mask(mask), _u8p), _ptr(self._s(s)), _ptr(f_t),
                                _ptr(lam_in), _ptr(out), _ptr(grad_s), _ptr(g))
        return out

    def objective_current(self, f, axis=0, mask=None, norm=None):
        """J = (1/norm) sum over fluid nodes of sum_a f_a xi_a[axis] (norm = N)."""
        t = self.totals(f, mask)
        return t[1 + axis] / float(self.N if norm is None else norm)

    def gradient(self, f0, nsteps, mask=None, s=None, axis=0):
        """J(F_T) and its gradient with respect to s (field), E and tau, by storing
        every forward state and running the adjoint backwards (small grids only).
        Returns (J, grad_s (N,), grad (4,))."""
        states = [np.array(f0, dtype=np.float64, copy=True)]
        for _ in range(nsteps):
            states.append(self.step(states[-1], mask, s))
        J = self.objective_current(states[-1], axis, mask)
        lam = self.seed_current(axis, mask=mask)
        gs = np.zeros(self.N)
        g = np.zeros(4)
        for t in range(nsteps - 1, -1, -1):
            lam = self.adjoint_step(states[t], lam, mask, s, gs, g)
        return J, gs, g
