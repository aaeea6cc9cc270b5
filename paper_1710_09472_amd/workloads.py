"""Seeded synthetic inputs for the semiclassical LBM workloads.

This module builds geometry masks, soft-porosity fields and initial density/velocity
fields. It holds none of the method's arithmetic (no equilibrium, moment, force or
streaming formula), so both the GPU path and the CPU oracle can be fed from it.
Every array is numpy (float64 unless stated), in node order n = x + nx*(y + ny*z).

Workloads (all sizes in lattice nodes):

* ``poiseuille_2d``  D2V9 64x32, solid rows y = 0 and y = 31, periodic x, rho = 1,
  u = 0, E = (1e-6, 0), tau = 0.8, 2000 steps (the paper's Poiseuille test, Sec. 9.3,
  at a size a CPU finishes in seconds).
* ``riemann_2d``  D2V9 4096x4, periodic y, solid columns x = 0 and x = 4095, rho = 1.2
  for x < 2048 else 0.8, u = 0, tau = 0.6, 1500 steps (shock tube, Sec. 9.2).
* ``throughput_2d``  D2V9 4096x4096 fully periodic, rho = 1 + 0.01 N(0,1) (seed 1),
  u = 0, tau = 0.6.
* ``hall_duct_3d``  D3V19 256x128x128, solid planes y in {0,127} and z in {0,127},
  periodic x, E = (1e-6, 0, 0), B = (0, 0, 1e-3), tau = 0.7, 5000 steps.
* ``porous_ohm_2d``  D2V9 2048x2048 periodic with random non-overlapping disks of
  radius 8 (solid fraction 0.30, seed 2), E_x in {1..8} x 1e-7, tau = 0.9, 20000 steps
  (the Ohm's-law test of Sec. 9.4 at a larger size).
* ``soft_porous_3d``  D3V19 128^3 periodic with a soft partial-bounce-back field s in
  [0, 1] of mean 0.2 (seed 3), E = (1e-6, 0, 0), tau = 0.75, 600 steps.

The paper's own setups (Sec. 9.3, 9.4), with its velocity-shift forcing:

* ``ohm_paper_2d``  D2V9 512x256, free-slip walls y = 0, 255, periodic x, 64
  non-overlapping disks of radius 3 (seed 4, porosity 0.986), E_x = 1e-7, tau = 0.9.
* ``ohm_paper_3d``  D3V19 128^3, free-slip walls y and z, periodic x, 450 non-overlapping
  balls of radius 3 (seed 5, porosity 0.974), E_x = 1e-7, tau = 0.9.
* ``poiseuille_paper_2d``  D2V9 256x256, bounce-back rows y = 0, 255, periodic x,
  E_x = 1e-8, tau given (the paper sweeps five values), 10^6 steps.
* ``poiseuille_paper_3d``  D3V19 256x256x1, the same channel, periodic in x and z.

These use density 1 where the paper starts from mu = 1 (rho = I_0): the update is
homogeneous of degree one in f, so the velocity field does not depend on that scale.

The fourth-order thermal model (D1V7):

* ``thermal_1d``  D1V7, n nodes (default 2^24) periodic, Fermi-Dirac weight theta = 1/4,
  mu = 1 (moderately degenerate, z = e^4), rho = 1 + 0.01 N(0,1), u = 0.01 N(0,1),
  thetabar = thetabar_ref (1 + 0.01 N(0,1)) (seed 6, independent draws), tau = 0.8.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    lattice: str
    nx: int
    ny: int
    nz: int
    tau: float
    steps: int
    E: tuple = (0.0, 0.0, 0.0)
    B: tuple = (0.0, 0.0, 0.0)
    rho: np.ndarray | None = None     # (N,) float64
    u: np.ndarray | None = None       # (D, N) float64 or None (= 0)
    mask: np.ndarray | None = None    # (N,) uint8, 1 = solid, or None
    s: np.ndarray | None = None       # (N,) float64 in [0, 1], or None
    notes: dict = field(default_factory=dict)
    forcing: str = "source"           # "source" (xi-dependent term) or "shift" (velocity shift)
    slip: int = 0                     # free-slip wall planes: 1 y, 2 z (bits)
    thetabar: np.ndarray | None = None  # (N,) float64, D1V7 thermal model (None: the weight's)
    theta: float = 1.0 / 270.0        # weight parameters (electron model by default)
    mu: float = 1.0

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def D(self) -> int:
        return {"D1": 1, "D2": 2}.get(self.lattice[:2], 3)


def _grid(nx, ny, nz=1):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1), y.reshape(-1), z.reshape(-1)


def channel_mask_2d(nx: int, ny: int) -> np.ndarray:
    """Solid rows y = 0 and y = ny - 1."""
    _, y, _ = _grid(nx, ny)
    return ((y == 0) | (y == ny - 1)).astype(np.uint8)


def duct_mask_3d(nx: int, ny: int, nz: int) -> np.ndarray:
    """Solid planes y in {0, ny-1} and z in {0, nz-1}; x stays periodic."""
    _, y, z = _grid(nx, ny, nz)
    return ((y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)).astype(np.uint8)


def end_walls_mask_2d(nx: int, ny: int) -> np.ndarray:
    """Solid columns x = 0 and x = nx - 1 (closed shock tube)."""
    x, _, _ = _grid(nx, ny)
    return ((x == 0) | (x == nx - 1)).astype(np.uint8)


def disk_mask_2d(nx: int, ny: int, radius: int, solid_fraction: float, seed: int,
                 max_tries: int = 10_000_000) -> tuple[np.ndarray, int]:
    """Random non-overlapping disks on the periodic nx x ny torus.

    Random sequential addition: centres are drawn uniformly (numpy default_rng(seed));
    a centre is accepted if its periodic distance to every accepted centre is at least
    2*radius + 1; a node (i, j) is solid if (i - cx)^2 + (j - cy)^2 <= radius^2 with
    periodic wrap. Drawing stops as soon as the solid fraction reaches
    ``solid_fraction``. Returns (mask, number of disks).
    """
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), dtype=bool)
    r = int(radius)
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    inside = dx * dx + dy * dy <= r * r
    ox, oy = dx[inside], dy[inside]
    cell = 2 * r + 1
    # bucket grid for the overlap test
    gx, gy = max(1, nx // cell), max(1, ny // cell)
    buckets: dict = {}
    centres = []
    target = solid_fraction * nx * ny
    nsolid = 0
    tries = 0
    while nsolid < target:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("disk packing did not reach the requested solid fraction")
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        cxi, cyi = int(np.floor(cx)) % nx, int(np.floor(cy)) % ny
        bx, by = cxi * gx // nx, cyi * gy // ny
        ok = True
        for ddx in (-1, 0, 1):
            for ddy in (-1, 0, 1):
                for (px, py) in buckets.get(((bx + ddx) % gx, (by + ddy) % gy), ()):
                    ex = abs(px - cxi)
                    ex = min(ex, nx - ex)
                    ey = abs(py - cyi)
                    ey = min(ey, ny - ey)
                    if ex * ex + ey * ey < cell * cell:
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        buckets.setdefault((bx, by), []).append((cxi, cyi))
        centres.append((cxi, cyi))
        xs = (cxi + ox) % nx
        ys = (cyi + oy) % ny
        new = ~solid[ys, xs]
        solid[ys, xs] = True
        nsolid += int(new.sum())
    return solid.reshape(-1).astype(np.uint8), len(centres)


def ball_obstacles(dims: tuple, radius: int, count: int, seed: int, margin_axes: tuple = (),
                   max_tries: int = 1_000_000) -> np.ndarray:
    """`count` non-overlapping discrete balls (disks in 2D) of `radius` on the grid
    dims = (nx, ny, nz), periodic along every axis not in `margin_axes`.

    Random sequential addition (numpy default_rng(seed)): integer centres drawn
    uniformly, along each axis in `margin_axes` (1 = y, 2 = z) restricted to
    [radius + 1, n - 2 - radius] so that no ball touches the boundary planes; a centre
    is accepted if its periodic distance to every accepted centre is at least
    2 radius + 1. A node is solid if its (periodic) squared distance to a centre is at
    most radius^2. Returns the uint8 mask (1 = solid).
    """
    nx, ny, nz = dims
    n = np.array([nx, ny, nz])
    rng = np.random.default_rng(seed)
    r = int(radius)
    d3 = 3 if nz > 1 else 2
    off = np.stack(np.meshgrid(*[np.arange(-r, r + 1)] * d3, indexing="ij"), -1).reshape(-1, d3)
    off = off[(off ** 2).sum(1) <= r * r]
    if d3 == 2:
        off = np.concatenate([off, np.zeros((len(off), 1), int)], 1)
    lo = np.zeros(3, int)
    hi = n.copy()
    for a in margin_axes:
        lo[a], hi[a] = r + 1, n[a] - 1 - r
    centres = []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("ball placement did not fit the requested count")
        c = np.array([rng.integers(lo[i], hi[i]) if n[i] > 1 else 0 for i in range(3)])
        if centres:
            dd = np.abs(np.array(centres) - c)
            dd = np.minimum(dd, n - dd)
            if ((dd ** 2).sum(1) < (2 * r + 1) ** 2).any():
                continue
        centres.append(c)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    for c in centres:
        p = (c + off) % n
        solid[p[:, 2], p[:, 1], p[:, 0]] = 1
    return solid.reshape(-1)


def soft_porosity_3d(n: int, mean: float, seed: int, sigma: float = 3.0) -> np.ndarray:
    """Soft solid fraction s in [0, 1] on a periodic n^3 grid.

    N(0,1) noise (default_rng(seed)) is smoothed with a periodic Gaussian filter of
    standard deviation ``sigma`` cells (FFT), then mapped through a logistic
    s = 1/(1 + exp(-(g - t)/w)) with w = 0.25 std(g) and the threshold t found by
    bisection so that mean(s) = ``mean``.
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n, n))
    k = np.fft.fftfreq(n)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx * kx + ky * ky + kz * kz))
    g = np.real(np.fft.ifftn(np.fft.fftn(g) * filt))
    w = 0.25 * g.std()
    lo, hi = g.min() - 20 * w, g.max() + 20 * w

    def m(t):
        return float(np.mean(1.0 / (1.0 + np.exp(-(g - t) / w))))

    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if m(mid) > mean:
            lo = mid
        else:
            hi = mid
    t = 0.5 * (lo + hi)
    s = 1.0 / (1.0 + np.exp(-(g - t) / w))
    return s.reshape(-1)


def poiseuille_2d(nx: int = 64, ny: int = 32) -> Workload:
    return Workload("poiseuille_2d", "D2V9", nx, ny, 1, tau=0.8, steps=2000, E=(1e-6, 0.0, 0.0),
                    rho=np.ones(nx * ny), mask=channel_mask_2d(nx, ny))


def riemann_2d(nx: int = 4096, ny: int = 4) -> Workload:
    x, _, _ = _grid(nx, ny)
    rho = np.where(x < nx // 2, 1.2, 0.8).astype(np.float64)
    return Workload("riemann_2d", "D2V9", nx, ny, 1, tau=0.6, steps=1500, rho=rho,
                    mask=end_walls_mask_2d(nx, ny))


def throughput_2d(nx: int = 4096, ny: int = 4096, seed: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.01 * rng.standard_normal(nx * ny)
    return Workload("throughput_2d", "D2V9", nx, ny, 1, tau=0.6, steps=1000, rho=rho)


def hall_duct_3d(nx: int = 256, ny: int = 128, nz: int = 128) -> Workload:
    return Workload("hall_duct_3d", "D3V19", nx, ny, nz, tau=0.7, steps=5000, E=(1e-6, 0.0, 0.0),
                    B=(0.0, 0.0, 1e-3), rho=np.ones(nx * ny * nz), mask=duct_mask_3d(nx, ny, nz))


def porous_ohm_2d(n: int = 2048, Ex: float = 1e-7, seed: int = 2, radius: int = 8,
                  solid_fraction: float = 0.30) -> Workload:
    mask, ndisks = disk_mask_2d(n, n, radius, solid_fraction, seed)
    return Workload("porous_ohm_2d", "D2V9", n, n, 1, tau=0.9, steps=20000, E=(Ex, 0.0, 0.0),
                    rho=np.ones(n * n), mask=mask, notes={"disks": ndisks})


def soft_porous_3d(n: int = 128, seed: int = 3, mean: float = 0.2) -> Workload:
    s = soft_porosity_3d(n, mean, seed)
    return Workload("soft_porous_3d", "D3V19", n, n, n, tau=0.75, steps=600, E=(1e-6, 0.0, 0.0),
                    rho=np.ones(n ** 3), s=s)


def ohm_paper_2d(Ex: float = 1e-7, seed: int = 4, steps: int = 20000) -> Workload:
    nx, ny = 512, 256
    mask = ball_obstacles((nx, ny, 1), 3, 64, seed, margin_axes=(1,))
    return Workload("ohm_paper_2d", "D2V9", nx, ny, 1, tau=0.9, steps=steps, E=(Ex, 0.0, 0.0),
                    rho=np.ones(nx * ny), mask=mask, forcing="shift", slip=1)


def ohm_paper_3d(Ex: float = 1e-7, seed: int = 5, steps: int = 20000) -> Workload:
    n = 128
    mask = ball_obstacles((n, n, n), 3, 450, seed, margin_axes=(1, 2))
    return Workload("ohm_paper_3d", "D3V19", n, n, n, tau=0.9, steps=steps, E=(Ex, 0.0, 0.0),
                    rho=np.ones(n ** 3), mask=mask, forcing="shift", slip=3)


def poiseuille_paper_2d(tau: float = 0.8, n: int = 256, steps: int = 1_000_000) -> Workload:
    return Workload("poiseuille_paper_2d", "D2V9", n, n, 1, tau=tau, steps=steps, E=(1e-8, 0.0, 0.0),
                    rho=np.ones(n * n), mask=channel_mask_2d(n, n), forcing="shift")


def poiseuille_paper_3d(tau: float = 0.8, n: int = 256, steps: int = 1_000_000) -> Workload:
    """The 3D run of Sec. 9.3: D3V19 n x n x 1, bounce-back rows y = 0, n - 1, periodic in x
    and z, velocity shift E_x = 1e-8."""
    mask = channel_mask_2d(n, n)
    return Workload("poiseuille_paper_3d", "D3V19", n, n, 1, tau=tau, steps=steps, E=(1e-8, 0.0, 0.0),
                    rho=np.ones(n * n), mask=mask, forcing="shift")


def thermal_1d(thetabar_ref: float, n: int = 1 << 24, seed: int = 6, tau: float = 0.8,
               theta: float = 0.25, mu: float = 1.0, amp: float = 0.01) -> Workload:
    """D1V7 thermal workload: white-noise density, velocity and thetabar perturbations of
    relative size amp around (1, 0, thetabar_ref); thetabar_ref is the weight's I_2/I_0,
    given by the caller."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal(n)
    u = amp * rng.standard_normal((1, n))
    tb = thetabar_ref * (1.0 + amp * rng.standard_normal(n))
    return Workload("thermal_1d", "D1V7", n, 1, 1, tau=tau, steps=0, rho=rho, u=u, thetabar=tb,
                    theta=theta, mu=mu)


def random_fields(lattice: str, nx: int, ny: int, nz: int = 1, seed: int = 0, drho: float = 0.05,
                  umax: float = 0.02, solid_fraction: float = 0.0, soft: bool = False) -> Workload:
    """Generic random test input: rho = 1 + drho U(-1,1), u = umax U(-1,1) per component,
    optional random solid nodes and a random s in [0, 1)."""
    rng = np.random.default_rng(seed)
    D = 2 if lattice.startswith("D2") else 3
    N = nx * ny * nz
    rho = 1.0 + drho * rng.uniform(-1, 1, N)
    u = umax * rng.uniform(-1, 1, (D, N))
    mask = (rng.uniform(0, 1, N) < solid_fraction).astype(np.uint8) if solid_fraction > 0 else None
    s = rng.uniform(0, 1, N) if soft else None
    return Workload(f"random_{lattice}", lattice, nx, ny, nz, tau=0.8, steps=0, rho=rho, u=u,
                    mask=mask, s=s)


def window(arr: np.ndarray, dims: tuple, lo: tuple, size: tuple, ncomp: int | None = None) -> np.ndarray:
    """Periodic sub-window of a node field (or of a [ncomp, N] field): the nodes
    lo[i] .. lo[i] + size[i] - 1 along each axis (x, y, z), wrapped."""
    nx, ny, nz = dims
    idx = [(np.arange(size[i]) + lo[i]) % dims[i] for i in range(3)]
    if ncomp is None:
        g = arr.reshape(nz, ny, nx)
        return g[np.ix_(idx[2], idx[1], idx[0])].reshape(-1).copy()
    g = arr.reshape(ncomp, nz, ny, nx)
    return g[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]].reshape(ncomp, -1).copy()
