"""The differentiation workload at full size: D3V19 128^3 periodic soft-porosity field
(mean solid fraction 0.2), E_x = 1e-6, tau = 0.75, 600 steps, checkpoints every 50.

The checkpointed adjoint gradient of the mean x-current with respect to E_x, tau and the
porosity field s is checked against central finite differences of the same FP32 GPU
forward run, to 1e-4 relative. The kernels see E, 1/tau and s in FP32, so each
difference quotient divides by the perturbation the kernels actually received: E
(relative step 1e-3) and omega = 1/tau (tau step 1e-3) as rounded to FP32, and for s a
seeded N(0,1) direction v with step 1e-4, compared as J(s+) - J(s-) against
<dJ/ds, s+ - s-> with s+- the FP32 fields. (The FP64 oracle checks the adjoint
element-wise on smaller grids; at this size its forward runs take minutes each.)
"""
import numpy as np
import pytest
import torch

from paper_1710_09472_amd import workloads as W
from paper_1710_09472_amd.adjoint import Problem, forward_with_checkpoints, mean_current

pytestmark = pytest.mark.gpu


def test_soft_porous_gradient_vs_fd():
    wl = W.soft_porous_3d()
    pb = Problem(wl.lattice, wl.nx, wl.ny, wl.nz, wl.steps, wl.rho, None, None, (0, 0, 0), checkpoint=50)
    E = torch.tensor(wl.E, dtype=torch.float64, device="cuda", requires_grad=True)
    tau = torch.tensor(wl.tau, dtype=torch.float64, device="cuda", requires_grad=True)
    s = torch.tensor(wl.s, dtype=torch.float32, device="cuda", requires_grad=True)
    J = mean_current(E, tau, s, pb)
    J.backward()

    def J_at(E_, tau_, s_):
        j, sim, _ = forward_with_checkpoints(pb, E_, tau_, s_)
        sim.close()
        return j

    s0 = s.detach()
    f32 = lambda x: float(np.float32(x))
    Ex = wl.E[0]
    h = 1e-3
    Ep, Em = Ex * (1 + h), Ex * (1 - h)
    fdE = (J_at((Ep, 0, 0), wl.tau, s0) - J_at((Em, 0, 0), wl.tau, s0)) / (f32(Ep) - f32(Em))
    tp, tm = wl.tau + h, wl.tau - h
    # the kernels use omega = fl32(1/tau): difference with respect to the tau they imply
    tp_eff, tm_eff = 1.0 / f32(1.0 / tp), 1.0 / f32(1.0 / tm)
    fdT = (J_at(wl.E, tp, s0) - J_at(wl.E, tm, s0)) / (tp_eff - tm_eff)
    v = torch.tensor(np.random.default_rng(4).standard_normal(wl.N), dtype=torch.float32, device="cuda")
    sp, sm = s0 + 1e-4 * v, s0 - 1e-4 * v
    dJs = J_at(wl.E, wl.tau, sp) - J_at(wl.E, wl.tau, sm)
    gE, gT = E.grad[0].item(), tau.grad.item()
    gS = float((s.grad.double() * (sp.double() - sm.double())).sum())
    print(f"J = {J.item():.10e}; dJ/dEx adj {gE:.8e} fd {fdE:.8e}; dJ/dtau adj {gT:.8e} fd {fdT:.8e}; "
          f"dJ along s adj {gS:.8e} fd {dJs:.8e}")
    assert abs(gE - fdE) <= 1e-4 * abs(fdE)
    assert abs(gT - fdT) <= 1e-4 * abs(fdT)
    assert abs(gS - dJs) <= 1e-4 * abs(dJs)
