#!/usr/bin/env python3
"""Throughput benchmark of the semiclassical LBM step on one MI355X.

Workload: the 4096 x 4096 fully periodic D2V9 grid with the Fermi-Dirac electron
weight (theta = 1/270, mu = 1), rho = 1 + 0.01 N(0,1) (seed 1), u = 0, tau = 0.6.
A timed step is one fused collide-and-stream update of every node (pull streaming,
moments, equilibrium, Lorentz source, BGK relaxation, store) in FP32 arithmetic with
FP32 deviation storage, inputs resident in HBM.

Prints one JSON line: MLUPS (value), ms per step, the roofline of the step kernel
(algorithmic bytes per launch / measured average launch time, against 8 TB/s HBM3E),
the FP16- and BF16-storage steps, the adjoint step relative to the forward step, and
the FP64 CPU oracle timed on this host on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "MLUPS & % HBM peak: FD-LBM step FP32 vs FP16-storage, fwd+adjoint, at stated err"
HBM_PEAK_GBS = 8000.0
PROFILE_DIR = ROOT / "profiles"


def bytes_per_node(Q: int, elem: int) -> int:
    """Algorithmic HBM bytes of one node update: Q populations read and Q written."""
    return 2 * Q * elem


def timed_steps(sim, steps: int, warmup: int):
    """Warm up, then time `steps` launches with HIP events on the library's stream
    (torch's current stream) and with the host clock; both bracketed by synchronize."""
    import torch

    sim.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(sim.stream)
    sim.step(steps)
    ev1.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) * 1e-3


def adjoint_ratio(wl, steps: int, warmup: int):
    """Average time of one adjoint step (reverse pull, transposed collision and force,
    FP64 block partials for dJ/dE and dJ/dtau) relative to one forward step."""
    import torch
    from paper_1710_09472_amd.lbm import Simulation

    sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=(1e-6, 0, 0))
    sim.init(wl.rho)
    state = sim.get_state()
    lam = [sim.adjoint_seed(), sim.new_adjoint()]
    gsc = torch.zeros(4, dtype=torch.float64, device="cuda")
    for i in range(warmup):
        sim.adjoint_step(state, lam[i % 2], lam[(i + 1) % 2], None, gsc)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    for i in range(steps):
        sim.adjoint_step(state, lam[i % 2], lam[(i + 1) % 2], None, gsc)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    t_adj = e0.elapsed_time(e1) * 1e-3 / steps
    _, t_fwd = timed_steps(sim, steps, warmup)
    sim.close()
    return t_adj, t_fwd / steps


def adjoint_pipeline():
    """The differentiation workload (D3V19 128^3 soft porosity, 600 steps, checkpoints every
    50): forward run with checkpoints, then the reverse pass (segment recompute + adjoint
    steps). Returns ms per forward step, ms per reverse step and their ratio."""
    import torch
    from paper_1710_09472_amd import workloads as W
    from paper_1710_09472_amd.adjoint import Problem, adjoint_gradients, forward_with_checkpoints

    wl = W.soft_porous_3d()
    pb = Problem(wl.lattice, wl.nx, wl.ny, wl.nz, wl.steps, wl.rho, None, None, (0, 0, 0), checkpoint=50)
    s = torch.tensor(wl.s, dtype=torch.float32, device="cuda")
    J, sim, cps = forward_with_checkpoints(pb, wl.E, wl.tau, s)  # warm-up
    adjoint_gradients(pb, sim, cps)
    sim.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, sim, cps = forward_with_checkpoints(pb, wl.E, wl.tau, s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gE, gT, gs, _ = adjoint_gradients(pb, sim, cps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.close()
    fwd, bwd = (t1 - t0) / wl.steps, (t2 - t1) / wl.steps
    return {"workload": "soft_porous_3d: D3V19 128^3, mean s 0.2, E_x 1e-6, tau 0.75, 600 steps, K=50",
            "forward_ms_per_step": round(fwd * 1e3, 5), "reverse_ms_per_step": round(bwd * 1e3, 5),
            "ratio_to_forward": round(bwd / fwd, 3), "dJ_dEx": float(gE[0]), "dJ_dtau": float(gT)}


def traffic_from_profile(kernel_tag: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy-kernel calibration), read from the committed summary, if the
    kernel source has not changed since it was taken; else None."""
    f = PROFILE_DIR / f"{kernel_tag}_pmc.txt"
    if not f.exists():
        return None
    txt = f.read_text()
    m = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    h = re.search(r"^kernel_source_sha256:\s*([0-9a-f]+)", txt, re.M)
    if not m or not h:
        return None
    import hashlib

    src = (ROOT / "paper_1710_09472_amd" / "csrc" / "lbm_kernels.hip").read_bytes()
    if hashlib.sha256(src).hexdigest() != h.group(1):
        return None
    return float(m.group(1))


def cpu_baseline(wl, target_s: float = 12.0):
    """The FP64 oracle on this host's cores, on a 4096 x 256 strip of the same grid
    (same rho field rows, periodic), scaled to MLUPS."""
    import numpy as np

    from oracle.oracle import OracleModel, get_threads

    ny = 256
    sub_rho = wl.rho.reshape(wl.ny, wl.nx)[:ny].reshape(-1)
    m = OracleModel("D2V9", wl.nx, ny, 1, tau=wl.tau)
    f = m.init_state(sub_rho)
    f = m.run(f, 1)  # first call: thread start-up and page faults, not timed
    t0 = time.perf_counter()
    f = m.run(f, 5)
    one = (time.perf_counter() - t0) / 5
    steps = max(1, int(target_s / max(one, 1e-4)))
    t0 = time.perf_counter()
    f = m.run(f, steps)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    mlups = wl.nx * ny * steps / dt / 1e6
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": get_threads(), "kind": "oracle",
            "sample": f"D2V9 {wl.nx}x{ny} strip of the 4096x4096 grid, FP64, {steps} steps in {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the FP32 step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB three times with a plain device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the method runs on a "
              "single device here; multi-GPU domain decomposition is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_09472_amd import workloads as W
    from paper_1710_09472_amd.lbm import Simulation

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    wl = W.throughput_2d()
    N = wl.N
    sim = Simulation(wl.lattice, wl.nx, wl.ny, 1, tau=wl.tau)
    sim.init(wl.rho)
    wall, ev = timed_steps(sim, args.steps, args.warmup)
    t_launch = ev / args.steps
    mlups = N * args.steps / wall / 1e6
    alg = bytes_per_node(sim.Q, 4) * N
    achieved = alg / t_launch / 1e9
    traffic = traffic_from_profile("k_step_D2V9_f32_4096x4096")
    tot = sim.current()
    sim.close()
    del sim

    extras = {}
    if not args.no_extras:
        for st, k in (("f16", 12), ("bf16", 0)):
            s16 = Simulation(wl.lattice, wl.nx, wl.ny, 1, tau=wl.tau, storage=st, dev_scale_log2=k)
            s16.init(wl.rho)
            w16, e16 = timed_steps(s16, args.steps, args.warmup)
            t16 = e16 / args.steps
            extras[st] = {"MLUPS": round(N * args.steps / w16 / 1e6, 1), "ms_per_step": round(w16 / args.steps * 1e3, 5),
                          "achieved_GBs": round(bytes_per_node(s16.Q, 2) * N / t16 / 1e9, 1),
                          "dev_scale_log2": k}
            s16.close()
        t_adj, t_fwd = adjoint_ratio(wl, max(20, args.steps // 4), 5)
        extras["adjoint"] = {"step_only_4096sq": {"ms_per_step": round(t_adj * 1e3, 5),
                                                  "forward_ms_per_step": round(t_fwd * 1e3, 5),
                                                  "ratio_to_forward": round(t_adj / t_fwd, 3)},
                             "checkpointed_128cube": adjoint_pipeline()}

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "throughput_2d: D2V9 4096x4096 periodic, Fermi-Dirac weight theta=1/270 mu=1, "
                               "rho=1+0.01N(0,1) seed 1, u=0, tau=0.6, FP32 deviation storage",
                   "lattice": "D2V9", "nx": wl.nx, "ny": wl.ny, "storage": "f32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "k_step<D2V9,F32>", "bytes_per_launch": alg,
                     "avg_launch_ms": round(t_launch * 1e3, 5)},
        "storage16": extras.get("f16") and {"f16": extras["f16"], "bf16": extras["bf16"]},
        "adjoint": extras.get("adjoint"),
        "mass_after_run": tot[0],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
