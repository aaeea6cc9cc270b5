"""Write the FP64 oracle's central differences of the mean x-current for the
differentiation workload at its full size (``soft_porous_fd.json``).

Workload: D3V19 128^3 periodic, soft partial-bounce-back field s of mean 0.2 (seed 3),
E_x = 1e-6, tau = 0.75, rho = 1, u = 0, 600 steps. Objective: J = (1/N) sum over nodes of
sum_a f_a(x, T) xi_a,x at T = 600 (pre-collision, xi-units). Differences (central):

* E_x with a relative step h = 1e-4:      (J(E_x (1 + h)) - J(E_x (1 - h))) / (2 h E_x)
* tau with an absolute step h = 1e-4:     (J(tau + h) - J(tau - h)) / (2 h)
* s along v = N(0, 1) per node (numpy default_rng(4)), h = 1e-4:
                                          (J(s + h v) - J(s - h v)) / (2 h) = <dJ/ds, v>

Only ``oracle/`` computes anything here; the inputs come from the package's seeded
workload generator, which holds none of the method's arithmetic. A hash of the inputs is
stored, so that a test can check that the workload has not changed since.

Usage: python tests/golden/make_soft_porous_fd.py [--threads N]   (about 30 minutes on 6
cores of a 2.7 GHz Xeon)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import OracleModel, get_threads, set_threads  # noqa: E402
from paper_1710_09472_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "soft_porous_fd.json")
H = 1e-4
DIRECTION_SEED = 4


def input_hash(wl) -> str:
    h = hashlib.sha256()
    for a in (wl.rho, wl.s):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    h.update(repr((wl.lattice, wl.nx, wl.ny, wl.nz, wl.tau, wl.E, wl.steps)).encode())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    if args.threads:
        set_threads(args.threads)
    wl = W.soft_porous_3d()
    v = np.random.default_rng(DIRECTION_SEED).standard_normal(wl.N)
    t_start = time.time()

    def J(Ex=wl.E[0], tau=wl.tau, s=wl.s, label=""):
        t0 = time.time()
        m = OracleModel(wl.lattice, wl.nx, wl.ny, wl.nz, tau=tau, E=(Ex, 0.0, 0.0))
        f = m.init_state(wl.rho)
        f = m.run(f, wl.steps, None, s)
        j = m.objective_current(f, 0)
        print(f"{label:>8s}: J = {j:.17e}  ({time.time() - t0:.0f} s)", flush=True)
        return j

    Ex, tau = wl.E[0], wl.tau
    J0 = J(label="nominal")
    Jep, Jem = J(Ex=Ex * (1 + H), label="E+"), J(Ex=Ex * (1 - H), label="E-")
    Jtp, Jtm = J(tau=tau + H, label="tau+"), J(tau=tau - H, label="tau-")
    Jsp, Jsm = J(s=wl.s + H * v, label="s+"), J(s=wl.s - H * v, label="s-")
    out = {
        "what": "FP64 oracle central differences of the mean x-current, soft_porous_3d at full size",
        "workload": {"lattice": wl.lattice, "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "tau": tau, "E": list(wl.E),
                     "steps": wl.steps, "s_mean": float(wl.s.mean()), "input_sha256": input_hash(wl)},
        "h": {"E_relative": H, "tau_absolute": H, "s_direction": H, "direction_seed": DIRECTION_SEED},
        "J": J0,
        "J_pm": {"E": [Jep, Jem], "tau": [Jtp, Jtm], "s": [Jsp, Jsm]},
        "dJ_dEx": (Jep - Jem) / (2 * H * Ex),
        "dJ_dtau": (Jtp - Jtm) / (2 * H),
        "dJ_ds_dot_v": (Jsp - Jsm) / (2 * H),
        "oracle_threads": get_threads(),
        "seconds": round(time.time() - t_start, 1),
    }
    with open(OUT + ".tmp", "w") as fh:
        json.dump(out, fh, indent=1)
    os.replace(OUT + ".tmp", OUT)
    print(json.dumps({k: out[k] for k in ("dJ_dEx", "dJ_dtau", "dJ_ds_dot_v")}), flush=True)


if __name__ == "__main__":
    main()
