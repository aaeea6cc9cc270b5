"""Gradients of the mean current through the library's hand-written adjoint step.

``MeanCurrent`` is a ``torch.autograd.Function``: J(E, tau, s) is the mean x-current per
node after T time steps,

    J = (1/N) sum over fluid nodes x of sum_a f_a(x, T) xi_a,x   (xi-units),

and its backward pass runs the discrete adjoint (``lbm_adjoint_step``) with
checkpoint-and-recompute: the forward pass keeps the state every K steps; the backward
pass restores each checkpoint, recomputes the K states of that segment with
``lbm_step_from`` and walks them in reverse. With ``keep_states`` the forward pass writes
every state into its own buffer (``lbm_step_from`` from one to the next, no copies) and
the backward pass recomputes nothing: T + 1 states of memory (the 128^3 D3V19 workload's
600 steps: 96 GB, within one MI355X's 288 GB) for a reverse pass of adjoint steps only. Gradients: dJ/dE (3), dJ/dtau and the
field dJ/ds of the partial bounce-back fraction. All arithmetic runs in the library's
kernels; this module only orders the calls and owns the buffers (torch tensors). Both
forcing schemes (``Problem.forcing``) and the free-slip wall planes (``Problem.slip``)
are covered; J and the seed exclude the wall planes, which are solid. With 16-bit forward
states (``Problem.storage``) the gradients are those of the stored model with its encoding
taken as the identity; with stochastic rounding the recomputed segments repeat the forward
run's bits through the step index (``lbm_set_step_index``).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from .lbm import Simulation


@dataclass
class Problem:
    lattice: str
    nx: int
    ny: int
    nz: int
    steps: int
    rho: np.ndarray                 # (N,) initial density
    u: np.ndarray | None = None     # (D, N) initial velocity, xi-units
    mask: np.ndarray | None = None  # (N,) uint8
    B: tuple = (0.0, 0.0, 0.0)
    checkpoint: int = 50
    keep_states: bool = False       # keep all T + 1 states: no recompute in the reverse pass
    axis: int = 0
    forcing: str = "source"         # "source" (Sec. 7) or "shift" (eq. (u-update-force-term-eq))
    slip: int = 0                   # free-slip wall planes (Sec. 9.4): bit 0 y, bit 1 z
    inplace: bool = False           # one state buffer (checkpoints still in two-buffer layout)
    storage: str = "f32"            # forward states in "f32", "f16" (x 2^dev_scale_log2) or "bf16"
    dev_scale_log2: int = 0
    rounding: str = "nearest"       # of 16-bit stored values: "nearest" or "stochastic"

    @property
    def N(self):
        return self.nx * self.ny * self.nz


def _make_sim(pb: Problem, E, tau, s):
    return Simulation(pb.lattice, pb.nx, pb.ny, pb.nz, tau=float(tau), E=[float(v) for v in E], B=pb.B,
                      mask=pb.mask, s=s, forcing=pb.forcing, slip=pb.slip, inplace=pb.inplace,
                      storage=pb.storage, dev_scale_log2=pb.dev_scale_log2, rounding=pb.rounding)


def forward_with_checkpoints(pb: Problem, E, tau, s):
    """Run T steps; return (J, sim, checkpoints) where checkpoints[i] is the state at
    step i*K (the state whose pull gives f(i*K)), or, with keep_states, at step i for
    every i = 0..T."""
    sim = _make_sim(pb, E, tau, s)
    sim.init(pb.rho, pb.u)
    if pb.keep_states:
        states = [sim.get_state()]
        sim.set_step_index(0)
        for _ in range(pb.steps):
            nxt = sim.new_state(zero=False)  # written by the step where any pull reads
            sim.step_from(states[-1], nxt)
            states.append(nxt)
        sim.set_state(states[-1])  # the totals of f(T)
        tot = sim.current()
        return tot[1 + pb.axis] / pb.N, sim, states
    cps = []
    for t0 in range(0, pb.steps, pb.checkpoint):
        cps.append(sim.get_state())
        sim.step(min(pb.checkpoint, pb.steps - t0))
    tot = sim.current()
    return tot[1 + pb.axis] / pb.N, sim, cps


def adjoint_gradients(pb: Problem, sim: Simulation, cps):
    """Reverse pass. Returns (grad_E (3,), grad_tau, grad_s (N,) or None) as device
    tensors, for dJ/d(...) with J as in the module docstring."""
    dev = sim.device
    K = pb.checkpoint
    lam = [sim.adjoint_seed(pb.axis, pb.N), sim.new_adjoint()]
    gsc = torch.zeros(4, dtype=torch.float64, device=dev)
    gs = torch.zeros(pb.N, dtype=torch.float32, device=dev) if sim.s is not None else None
    cur = 0
    if pb.keep_states:  # every state kept by the forward pass: adjoint steps only
        for t in range(pb.steps - 1, -1, -1):
            sim.adjoint_step(cps[t], lam[cur], lam[cur ^ 1], gs, gsc if t == 0 else None)
            cur ^= 1
        return gsc[:3].clone(), gsc[3].clone(), gs, lam[cur]
    seg_bufs = [sim.new_state() for _ in range(K)]
    nseg = len(cps)
    for i in range(nseg - 1, -1, -1):
        t0 = i * K
        n = min(K, pb.steps - t0)
        seg_bufs[0].copy_(cps[i])
        sim.set_step_index(t0)  # the recomputed steps repeat the forward run's bits
        for k in range(1, n):
            sim.step_from(seg_bufs[k - 1], seg_bufs[k])
        for k in range(n - 1, -1, -1):
            # dJ/dE, dJ/dtau stay as per-block partials until the last step of the pass
            sim.adjoint_step(seg_bufs[k], lam[cur], lam[cur ^ 1], gs, gsc if (i == 0 and k == 0) else None)
            cur ^= 1
    return gsc[:3].clone(), gsc[3].clone(), gs, lam[cur]


class MeanCurrent(torch.autograd.Function):
    """J = mean_current(E (3,), tau (), s (N,) or None, problem)."""

    @staticmethod
    def forward(ctx, E, tau, s, pb: Problem):
        Eh = E.detach().double().cpu().numpy()
        th = float(tau.detach().cpu())
        sh = None if s is None else s.detach().float()
        J, sim, cps = forward_with_checkpoints(pb, Eh, th, sh)
        ctx.pb, ctx.sim, ctx.cps = pb, sim, cps
        ctx.has_s = s is not None
        return torch.tensor(J, dtype=torch.float64, device=E.device)

    @staticmethod
    def backward(ctx, gJ):
        gE, gtau, gs, _ = adjoint_gradients(ctx.pb, ctx.sim, ctx.cps)
        ctx.sim.close()
        gJ = gJ.to(torch.float64)
        out_s = (gs.double() * gJ) if ctx.has_s else None
        return (gE * gJ), (gtau * gJ), out_s, None


def mean_current(E, tau, s, problem: Problem):
    return MeanCurrent.apply(E, tau, s, problem)
