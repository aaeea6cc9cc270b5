"""How finely FP32 storage of the deviations can pin the shock tube (Sec. 9.2, the 4096x4
strip with closed ends, 1500 steps): the FP64 oracle run again with its deviations
d_a = f_a - what_a rho0 rounded to FP32 (round to nearest even) after every step, FP64
arithmetic otherwise, against the plain FP64 run.

The rounding moves the shock front: the largest velocity error sits at the front, where the
solution jumps by ~0.03 of max|u| per cell, and is ~2e-4 of max|u|, while the L2 norm of the
velocity error stays below 1e-5 and the density plateaus are untouched. With a different
rounding of the same magnitude (one ulp up or down on a random quarter of the values, as
the FP32 arithmetic of a kernel rounds differently from FP64) the max-norm error is
6e-6 ... 1e-5. So on this workload the max-norm of u measures the front position, which
storage rounding alone can shift by ~1e-4 of max|u|; the GPU bound of the shock-tube parity
test (1e-5 in the max-norm of u) is therefore a statement about the kernel, not a guaranteed
property of FP32 deviation storage. Oracle and numpy only (no GPU)."""
import numpy as np
import pytest

from paper_1710_09472_amd import workloads as W

SHOCK_SPEED_2D = 0.782457  # isothermal Riemann solution, lattice units (reading of Sec. 9.2)


def _rounded_run(m, f, steps, mask, what, rng=None, frac=0.0):
    f = f.reshape(m.Q, m.N).copy()
    for _ in range(steps):
        d = (f - what).astype(np.float32)
        if rng is not None:
            sel = rng.random(d.shape) < frac
            up = np.where(rng.random(int(sel.sum())) < 0.5, -np.inf, np.inf).astype(np.float32)
            d[sel] = np.nextafter(d[sel], up)
        f = m.step((d.astype(np.float64) + what).reshape(-1), mask).reshape(m.Q, m.N)
    return f.reshape(-1)


@pytest.mark.slow
def test_shock_tube_fp32_storage_moves_the_front(oracle_lib):
    wl = W.riemann_2d()
    m = oracle_lib.OracleModel("D2V9", wl.nx, wl.ny, 1, tau=wl.tau)
    f0 = m.init_state(wl.rho, None, wl.mask)
    rho_o, u_o = m.moments(m.run(f0, wl.steps, wl.mask), wl.mask)
    what = (m.w / m.w.sum())[:, None]  # rho0 = 1
    fl = wl.mask == 0
    umax = np.abs(u_o[:, fl]).max()

    def errors(f):
        rho, u = m.moments(f, wl.mask)
        er = np.abs(rho[fl] - rho_o[fl]).max() / np.abs(rho_o[fl]).max()
        du = np.abs(u - u_o).max(0)
        eu = du[fl].max() / umax
        l2 = np.linalg.norm(u[:, fl] - u_o[:, fl]) / np.linalg.norm(u_o[:, fl])
        return er, eu, l2, int(np.argmax(du) % wl.nx)

    er, eu, l2, xu = errors(_rounded_run(m, f0, wl.steps, wl.mask, what))
    front = (wl.nx // 2 - 0.5) + SHOCK_SPEED_2D * wl.steps
    print(f"RNE FP32 storage: rho {er:.3e}, u max {eu:.3e} at x = {xu} (front {front:.1f}), u L2 {l2:.3e}")
    assert abs(xu - front) < 4           # the error is the displacement of the front
    assert 5e-5 < eu < 1e-3               # ... and at the front it is far above 1e-5 of max|u|
    assert l2 < 1e-5                      # while the velocity field as a whole stays within 1e-5
    worst = 0.0
    for seed in range(2):
        er_j, eu_j, l2_j, _ = errors(_rounded_run(m, f0, wl.steps, wl.mask, what, np.random.default_rng(seed), 0.25))
        print(f"rounding jitter (seed {seed}): rho {er_j:.3e}, u max {eu_j:.3e}, u L2 {l2_j:.3e}")
        worst = max(worst, eu_j)
        assert l2_j < 1e-5
    assert 1e-6 < worst < 5e-5
