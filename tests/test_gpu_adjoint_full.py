"""The differentiation workload at full size: D3V19 128^3 periodic soft-porosity field
(mean solid fraction 0.2), E_x = 1e-6, tau = 0.75, 600 steps, checkpoints every 50.

The checkpointed adjoint gradient of the mean x-current (``mean_current``, the library's
hand-written adjoint behind torch.autograd) against central differences of the FP64
oracle at the same full size, with the configured steps: E_x relative 1e-4, tau absolute
1e-4, and s along a seeded N(0, 1) direction v with step 1e-4 (compared as <dJ/ds, v>).
The oracle values are stored by ``tests/golden/make_soft_porous_fd.py``, which calls only
the oracle (about half an hour of host time); the stored hash of the inputs ties them to
the workload generator's current output. Bar: 1e-4 relative, each gradient on its own
scale.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

from paper_1710_09472_amd import workloads as W
from paper_1710_09472_amd.adjoint import Problem, mean_current

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "soft_porous_fd.json")


def _input_hash(wl) -> str:
    # the same recipe as the generator's
    h = hashlib.sha256()
    for a in (wl.rho, wl.s):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    h.update(repr((wl.lattice, wl.nx, wl.ny, wl.nz, wl.tau, wl.E, wl.steps)).encode())
    return h.hexdigest()


def test_soft_porous_gradient_vs_oracle_fd():
    gold = json.load(open(GOLDEN))
    wl = W.soft_porous_3d()
    assert gold["workload"]["input_sha256"] == _input_hash(wl), "workload changed since the oracle reference"
    h = gold["h"]
    assert h["E_relative"] == 1e-4 and h["tau_absolute"] == 1e-4 and h["s_direction"] == 1e-4
    pb = Problem(wl.lattice, wl.nx, wl.ny, wl.nz, wl.steps, wl.rho, None, None, (0, 0, 0), checkpoint=50)
    E = torch.tensor(wl.E, dtype=torch.float64, device="cuda", requires_grad=True)
    tau = torch.tensor(wl.tau, dtype=torch.float64, device="cuda", requires_grad=True)
    s = torch.tensor(wl.s, dtype=torch.float32, device="cuda", requires_grad=True)
    J = mean_current(E, tau, s, pb)
    J.backward()
    v = np.random.default_rng(h["direction_seed"]).standard_normal(wl.N)
    gE, gT = E.grad[0].item(), tau.grad.item()
    gS = float(s.grad.double().cpu().numpy() @ v)
    eJ = abs(J.item() / gold["J"] - 1)
    eE = abs(gE / gold["dJ_dEx"] - 1)
    eT = abs(gT / gold["dJ_dtau"] - 1)
    eS = abs(gS / gold["dJ_ds_dot_v"] - 1)
    print(f"J gpu {J.item():.10e} oracle {gold['J']:.10e} ({eJ:.2e}); "
          f"dJ/dEx adj {gE:.8e} oracle fd {gold['dJ_dEx']:.8e} ({eE:.2e}); "
          f"dJ/dtau adj {gT:.8e} oracle fd {gold['dJ_dtau']:.8e} ({eT:.2e}); "
          f"<dJ/ds, v> adj {gS:.8e} oracle fd {gold['dJ_ds_dot_v']:.8e} ({eS:.2e})")
    assert eJ < 1e-5
    assert eE < 1e-4
    assert eT < 1e-4
    assert eS < 1e-4
