#!/usr/bin/env python3
"""Throughput benchmark of the semiclassical LBM step on one MI355X.

Default workload: the 4096 x 4096 fully periodic D2V9 grid with the Fermi-Dirac electron
weight (theta = 1/270, mu = 1), rho = 1 + 0.01 N(0,1) (seed 1), u = 0, tau = 0.6.
A timed step is one fused collide-and-stream update of every node (pull streaming,
moments, equilibrium, Lorentz source, BGK relaxation, store) in FP32 arithmetic with
FP32 deviation storage, inputs resident in HBM.

Prints one JSON line: MLUPS (value), ms per step, the roofline of the step kernel
(algorithmic bytes per launch / measured average launch time, against 8 TB/s HBM3E),
the FP16- and BF16-storage steps, the adjoint step relative to the forward step, the
in-place step (one state buffer, FP32 and FP16) with its two phases, and the FP64 CPU
oracle timed on this host on a bounded sample of the same workload.

--workload selects one of the other full-size workloads (the 256x128x128 D3V19 Hall
duct, the 2048^2 D2V9 disk packing, the 128^3 D3V19 soft-porosity box) and --storage
its storage format; those runs time the step alone (no FP16/BF16 or adjoint extras).
--inplace times the in-place step (one state buffer) instead of the two-buffer step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                       [--storage f32|f16|bf16] [--inplace] [--no-cpu-baseline] [--no-extras]
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


# dev_scale_log2 of the FP16 runs: max|deviation| x 2^k near 2^12 for each workload
F16_SCALE = {"throughput_2d": 12, "hall_duct_3d": 28, "porous_ohm_2d": 25, "soft_porous_3d": 28,
             "ohm_paper_2d": 30, "ohm_paper_3d": 30, "poiseuille_paper_2d": 30, "thermal_1d": 17}


WORKLOAD_DESC = {
    "throughput_2d": "throughput_2d: D2V9 4096x4096 periodic, Fermi-Dirac weight theta=1/270 mu=1, "
                     "rho=1+0.01N(0,1) seed 1, u=0, tau=0.6",
    "hall_duct_3d": "hall_duct_3d: D3V19 256x128x128, solid planes y,z in {0,127}, periodic x, "
                    "E=(1e-6,0,0), B=(0,0,1e-3), tau=0.7",
    "porous_ohm_2d": "porous_ohm_2d: D2V9 2048x2048 periodic, radius-8 disks to solid fraction 0.30 (seed 2), "
                     "E_x=1e-7, tau=0.9",
    "soft_porous_3d": "soft_porous_3d: D3V19 128^3 periodic, partial bounce-back field s of mean 0.2 (seed 3), "
                      "E_x=1e-6, tau=0.75",
    "ohm_paper_2d": "ohm_paper_2d: D2V9 512x256, free-slip walls y, 64 disks r=3 (seed 4, porosity 0.986), "
                    "velocity-shift forcing E_x=1e-7, tau=0.9",
    "ohm_paper_3d": "ohm_paper_3d: D3V19 128^3, free-slip walls y and z, 450 balls r=3 (seed 5, porosity 0.974), "
                    "velocity-shift forcing E_x=1e-7, tau=0.9",
    "poiseuille_paper_2d": "poiseuille_paper_2d: D2V9 256x256, bounce-back rows y=0,255, velocity-shift forcing "
                           "E_x=1e-8, tau=0.8",
    "thermal_1d": "thermal_1d: D1V7 2^24 nodes periodic, fourth-order thermal model, Fermi-Dirac weight "
                  "theta=1/4 mu=1, rho=1+0.01N(0,1), u=0.01N(0,1), thetabar=thetabar_ref(1+0.01N(0,1)) seed 6, "
                  "tau=0.8",
}


def make_workload(name: str):
    from paper_1710_09472_amd import workloads as W

    if name == "thermal_1d":
        from paper_1710_09472_amd import lbm

        k = lbm.compute_constants("D1V7", "fd", 0.25, 1.0)
        return W.thermal_1d(k["I2"] / k["I0"])
    return {"throughput_2d": W.throughput_2d, "hall_duct_3d": W.hall_duct_3d,
            "porous_ohm_2d": W.porous_ohm_2d, "soft_porous_3d": W.soft_porous_3d,
            "ohm_paper_2d": W.ohm_paper_2d, "ohm_paper_3d": W.ohm_paper_3d,
            "poiseuille_paper_2d": W.poiseuille_paper_2d}[name]()


def wl_q(wl) -> int:
    """Populations per node of a workload's lattice."""
    return {"D2V9": 9, "D3V19": 19, "D1V7": 7}[wl.lattice]


def bytes_per_node(Q: int, elem: int) -> int:
    """Algorithmic HBM bytes of one node update: Q populations read and Q written."""
    return 2 * Q * elem


def solid_nodes(wl):
    """Solid flags of a workload: its obstacles and its free-slip wall planes (or None)."""
    import numpy as np

    if wl.mask is None and not wl.slip:
        return None
    solid = np.zeros((wl.nz, wl.ny, wl.nx), np.uint8) if wl.mask is None else \
        wl.mask.reshape(wl.nz, wl.ny, wl.nx).copy()
    if wl.slip & 1:
        solid[:, [0, wl.ny - 1], :] = 1
    if wl.slip & 2:
        solid[[0, wl.nz - 1], :, :] = 1
    return solid.reshape(-1)


def algorithmic_bytes(wl, Q: int, elem: int) -> int:
    """Minimum HBM bytes of one step: the populations of every fluid node read and
    written once, plus one byte of solid flag per node where there are solids and the
    FP32 porosity field where there is one."""
    solid = solid_nodes(wl)
    fluid = wl.N if solid is None else int((solid == 0).sum())
    b = fluid * bytes_per_node(Q, elem)
    if solid is not None:
        b += wl.N
    if wl.s is not None:
        b += 4 * wl.N
    return b


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


def inplace_phases(sim, steps: int):
    """Average durations of the two in-place kernels (the pull phase from the two-buffer
    layout, then the local phase back), from HIP events around every launch. The handle
    must be at even parity (an even number of steps since init)."""
    import torch

    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record(sim.stream)
    for i in range(steps):
        sim.step(1)
        evs[i + 1].record(sim.stream)
    torch.cuda.synchronize()
    d = [evs[i].elapsed_time(evs[i + 1]) * 1e-3 for i in range(steps)]
    return sum(d[0::2]) / len(d[0::2]), sum(d[1::2]) / len(d[1::2])


def inplace_extra(wl, storage: str, k: int, steps: int, warmup: int):
    """Throughput of the in-place (one-buffer) step on the workload's grid."""
    from paper_1710_09472_amd.lbm import Simulation

    sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=wl.E, B=wl.B, storage=storage,
                     dev_scale_log2=k, mask=wl.mask, s=wl.s, forcing=wl.forcing, slip=wl.slip, inplace=True)
    sim.init(wl.rho, wl.u)
    w, e = timed_steps(sim, steps, warmup + (warmup % 2))
    pull, local = inplace_phases(sim, 40)
    elem = 4 if storage == "f32" else 2
    alg = algorithmic_bytes(wl, sim.Q, elem)
    sim.close()
    return {"MLUPS": round(wl.N * steps / w / 1e6, 1), "ms_per_step": round(w / steps * 1e3, 5),
            "achieved_GBs": round(alg / (e / steps) / 1e9, 1),
            "pull_phase_ms": round(pull * 1e3, 5), "local_phase_ms": round(local * 1e3, 5),
            "state_buffers": 1}


def thermal_extra(steps: int, warmup: int):
    """Throughput of the fourth-order thermal step (D1V7, the 2^24-node thermal_1d
    workload; FP32 and FP16 storage, two buffers and in place) and its HBM fraction from
    HIP events on the library's stream."""
    from paper_1710_09472_amd.lbm import Simulation

    wl = make_workload("thermal_1d")
    sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, theta=wl.theta, mu=wl.mu)
    sim.init(wl.rho, wl.u, wl.thetabar)
    w, e = timed_steps(sim, steps, warmup)
    alg = algorithmic_bytes(wl, sim.Q, 4)
    sim.close()
    gbs = alg / (e / steps) / 1e9
    one = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, theta=wl.theta, mu=wl.mu, inplace=True)
    one.init(wl.rho, wl.u, wl.thetabar)
    w1, e1 = timed_steps(one, steps, warmup + (warmup % 2))
    one.close()
    out = {"workload": "thermal_1d: D1V7 2^24 nodes, K = 4, FP32", "MLUPS": round(wl.N * steps / w / 1e6, 1),
           "ms_per_step": round(w / steps * 1e3, 5), "achieved_GBs": round(gbs, 1),
           "hbm_frac": round(gbs / 8000.0, 4),
           "inplace": {"MLUPS": round(wl.N * steps / w1 / 1e6, 1), "ms_per_step": round(w1 / steps * 1e3, 5),
                       "achieved_GBs": round(alg / (e1 / steps) / 1e9, 1), "state_buffers": 1}}
    # FP16 storage (x 2^17), two state buffers and in place
    alg16 = algorithmic_bytes(wl, 7, 2)
    for inplace in (False, True):
        s16 = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, theta=wl.theta, mu=wl.mu, storage="f16",
                         dev_scale_log2=F16_SCALE["thermal_1d"], inplace=inplace)
        s16.init(wl.rho, wl.u, wl.thetabar)
        w16, e16 = timed_steps(s16, steps, warmup + (warmup % 2))
        s16.close()
        g16 = alg16 / (e16 / steps) / 1e9
        out["f16_inplace" if inplace else "f16"] = {"MLUPS": round(wl.N * steps / w16 / 1e6, 1),
                                                   "ms_per_step": round(w16 / steps * 1e3, 5),
                                                   "achieved_GBs": round(g16, 1), "hbm_frac": round(g16 / 8000.0, 4),
                                                   "dev_scale_log2": F16_SCALE["thermal_1d"]}
    return out


def adjoint_ratio(wl, steps: int, warmup: int, forcing: str = "source"):
    """Average time of one adjoint step (reverse pull, transposed collision and force,
    FP64 per-wave partials of dJ/dE and dJ/dtau held across steps and reduced on the
    last one) relative to one forward step of the same forcing."""
    import torch
    from paper_1710_09472_amd.lbm import Simulation

    sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=(1e-6, 0, 0), forcing=forcing)
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
        sim.adjoint_step(state, lam[i % 2], lam[(i + 1) % 2], None, gsc if i == steps - 1 else None)
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
    out = {"workload": "soft_porous_3d: D3V19 128^3, mean s 0.2, E_x 1e-6, tau 0.75, 600 steps, K=50",
           "forward_ms_per_step": round(fwd * 1e3, 5), "reverse_ms_per_step": round(bwd * 1e3, 5),
           "ratio_to_forward": round(bwd / fwd, 3), "dJ_dEx": float(gE[0]), "dJ_dtau": float(gT)}
    del cps
    # every state kept (601 x 159 MB = 96 GB of the 288 GB): the reverse pass recomputes nothing
    pk = Problem(wl.lattice, wl.nx, wl.ny, wl.nz, wl.steps, wl.rho, None, None, (0, 0, 0), keep_states=True)
    for timed in (False, True):  # the first run fills torch's allocator cache
        torch.cuda.synchronize()
        k0 = time.perf_counter()
        Jk, simk, states = forward_with_checkpoints(pk, wl.E, wl.tau, s)
        torch.cuda.synchronize()
        k1 = time.perf_counter()
        gEk, gTk, gsk, _ = adjoint_gradients(pk, simk, states)
        torch.cuda.synchronize()
        k2 = time.perf_counter()
        simk.close()
        del states
    fk, bk = (k1 - k0) / wl.steps, (k2 - k1) / wl.steps
    out["kept_states"] = {"forward_ms_per_step": round(fk * 1e3, 5), "reverse_ms_per_step": round(bk * 1e3, 5),
                          "ratio_to_forward": round(bk / fk, 3), "state_memory_GB": round((wl.steps + 1) * simk.sizes["state"] / 1e9, 1),
                          "same_gradients": bool(torch.equal(gEk, gE) and torch.equal(gTk, gT) and torch.equal(gsk, gs))}
    # the stated error: against the FP64 oracle's central differences at the same size and
    # steps, stored in the repository (tests/golden/soft_porous_fd.json)
    gold_path = ROOT / "tests" / "golden" / "soft_porous_fd.json"
    if gold_path.exists():
        import numpy as np

        gold = json.loads(gold_path.read_text())
        v = np.random.default_rng(gold["h"]["direction_seed"]).standard_normal(wl.N)
        gS = float(gs.double().cpu().numpy() @ v)
        out["err_vs_oracle_fd"] = {"dJ_dEx": float(f"{abs(out['dJ_dEx'] / gold['dJ_dEx'] - 1):.3g}"),
                                   "dJ_dtau": float(f"{abs(out['dJ_dtau'] / gold['dJ_dtau'] - 1):.3g}"),
                                   "dJ_ds_along_v": float(f"{abs(gS / gold['dJ_ds_dot_v'] - 1):.3g}"),
                                   "h": 1e-4}
    return out


def kernel_code_hash(thermal: bool = False) -> str:
    """sha256 of a step kernel's sources (the device header and the kernel files: the
    isothermal step's or the thermal step's) without // comments and blank lines: it
    changes with the code, not with its comments."""
    import hashlib

    lines = []
    names = ("lbm_thermal.hip",) if thermal else ("lbm_step_kernels.h", "lbm_kernels.hip")
    for name in ("lbm_device.h",) + names:
        for line in (ROOT / "paper_1710_09472_amd" / "csrc" / name).read_text().splitlines():
            line = re.sub(r"//.*$", "", line).rstrip()
            if line.strip():
                lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def traffic_from_profile(kernel_tag: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE + WRITE_SIZE,
    scaled by a copy-kernel calibration), read from the committed summary, if the
    kernel code has not changed since it was taken; else None."""
    f = PROFILE_DIR / f"{kernel_tag}_pmc.txt"
    if not f.exists():
        return None
    txt = f.read_text()
    m = re.search(r"^hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    h = re.search(r"^kernel_code_sha256:\s*([0-9a-f]+)", txt, re.M)
    if not m or not h or kernel_code_hash(kernel_tag.startswith("k_thermal")) != h.group(1):
        return None
    return float(m.group(1))


def cpu_baseline_thermal(wl, target_s: float = 12.0):
    """The FP64 thermal oracle (numpy) on the first 2^20 nodes of the 1D workload
    (periodic), scaled to MLUPS; numpy uses one thread for these element-wise passes."""
    from oracle.thermal import ThermalOracle

    n = min(wl.N, 1 << 20)
    m = ThermalOracle(n, wl.tau, theta=wl.theta, mu=wl.mu)
    f = m.init_state(wl.rho[:n], wl.u[0, :n], wl.thetabar[:n])
    f = m.step(f)
    t0 = time.perf_counter()
    f = m.step(f)
    one = time.perf_counter() - t0
    steps = max(1, int(target_s / max(one, 1e-4)))
    t0 = time.perf_counter()
    f = m.run(f, steps)
    dt = time.perf_counter() - t0
    model = ""
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": round(n * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"D1V7 first {n} nodes of the {wl.N}-node grid (periodic), FP64 numpy, {steps} steps in "
                      f"{dt:.1f} s", "cpu_model": model}


def _window_plan(dims, steps: int, core: int, centre):
    """Periodic sub-window holding the whole dependence cone of a core x core block after
    `steps` steps: axes longer than the window are cut to core + 2 (steps + 1) nodes around
    the block; shorter axes are kept whole. Returns (lo, size, block offset in the window)."""
    lo, size, off = [], [], []
    for i in range(3):
        width = core + 2 * (steps + 1)
        if dims[i] == 1 or width >= dims[i]:
            lo.append(0), size.append(dims[i]), off.append(centre[i] if dims[i] > 1 else 0)
        else:
            lo.append(centre[i] - (steps + 1)), size.append(width), off.append(steps + 1)
    return lo, size, off


def oracle_blocks(wl, steps: int, core: int, centres):
    """The FP64 oracle's rho and u after `steps` steps from the workload's initial state on
    core x core blocks, each recomputed exactly on the periodic sub-window of its dependence
    cone (the node update only reads the neighbours, so within `steps` steps the block does
    not see the rest of the grid). Periodic workloads without solids or porosity only.
    Returns (global node indices, rho, u (D, n))."""
    import numpy as np

    from oracle.oracle import OracleModel
    from paper_1710_09472_amd import workloads as W

    assert wl.mask is None and wl.s is None and not wl.slip
    dims = (wl.nx, wl.ny, wl.nz)
    idx, ref_rho, ref_u = [], [], []
    for c in centres:
        lo, size, off = _window_plan(dims, steps, core, c)
        m = OracleModel(wl.lattice, *size, tau=wl.tau, E=wl.E, B=wl.B, forcing=wl.forcing)
        rho_w = W.window(wl.rho, dims, lo, size)
        u_w = None if wl.u is None else W.window(wl.u, dims, lo, size, ncomp=wl.D)
        rho_o, u_o = m.moments(m.run(m.init_state(rho_w, u_w), steps))
        cs = [min(core, size[i]) for i in range(3)]
        loc = [(np.arange(cs[i]) + off[i]) % size[i] for i in range(3)]
        glob = [(loc[i] + lo[i]) % dims[i] for i in range(3)]
        li = (loc[0][None, None, :] + size[0] * (loc[1][None, :, None] + size[1] * loc[2][:, None, None])).reshape(-1)
        gi = (glob[0][None, None, :] + dims[0] * (glob[1][None, :, None] + dims[1] * glob[2][:, None, None])).reshape(-1)
        idx.append(gi), ref_rho.append(rho_o[li]), ref_u.append(u_o[:, li])
    return np.concatenate(idx), np.concatenate(ref_rho), np.concatenate(ref_u, axis=1)


def oracle_errors(wl, storages, steps: int = 100, core: int = 16,
                  centres=((0, 0, 0), (2048, 2048, 0))):
    """Max-norm errors of rho and u of the GPU step against the FP64 oracle (oracle_blocks)
    after `steps` steps: max|gpu - oracle| over the blocks divided by the largest |rho|, and
    the largest velocity component, of the oracle's blocks. storages: [(name, k)]."""
    import numpy as np
    import torch

    from paper_1710_09472_amd.lbm import Simulation

    t0 = time.perf_counter()
    idx, ref_rho, ref_u = oracle_blocks(wl, steps, core, centres)
    t_oracle = time.perf_counter() - t0
    out = {}
    for st, k in storages:
        sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=wl.E, B=wl.B, storage=st, dev_scale_log2=k,
                         forcing=wl.forcing)
        sim.init(wl.rho, wl.u)
        sim.step(steps)
        rho, u = sim.moments()
        torch.cuda.synchronize()
        rho, u = rho.double().cpu().numpy()[idx], u.double().cpu().numpy()[:, idx]
        sim.close()
        er = float(np.abs(rho - ref_rho).max() / np.abs(ref_rho).max())
        eu = float(np.abs(u - ref_u).max() / np.abs(ref_u).max())
        out[st] = {"rho": float(f"{er:.3g}"), "u": float(f"{eu:.3g}")}
        if st == "f16":
            out[st]["dev_scale_log2"] = k
    out["sample"] = (f"{len(centres)} blocks of {core}x{core} nodes at {[c[:2] for c in centres]} after {steps} steps, "
                     f"oracle on their dependence-cone windows ({t_oracle:.1f} s); max-norm error / max|ref|")
    return out


def cpu_baseline(wl, target_s: float = 12.0):
    """The FP64 oracle on this host's cores on a slab of the same workload (the first
    256 rows of a 2D grid, the first planes of a 3D grid, about half a million nodes,
    periodic, with the same solids and porosity), scaled to MLUPS."""
    import numpy as np

    from oracle.oracle import OracleModel, get_threads, set_threads

    if wl.lattice == "D1V7":
        return cpu_baseline_thermal(wl, target_s)

    nz = 1 if wl.nz == 1 else max(2, (1 << 19) // (wl.nx * wl.ny))
    ny = min(wl.ny, 256) if wl.nz == 1 else wl.ny
    n = wl.nx * ny * nz
    cut = lambda a: None if a is None else a.reshape(wl.nz, wl.ny, wl.nx)[:nz, :ny].reshape(-1)
    m = OracleModel(wl.lattice, wl.nx, ny, nz, tau=wl.tau, E=wl.E, B=wl.B, forcing=wl.forcing, slip=wl.slip)
    mask, s = cut(wl.mask), cut(wl.s)
    f = m.init_state(cut(wl.rho), mask=mask)
    f = m.run(f, 1, mask=mask, s=s)  # first call: thread start-up and page faults, not timed
    t0 = time.perf_counter()
    f = m.run(f, 5, mask=mask, s=s)
    one = (time.perf_counter() - t0) / 5
    steps = max(1, int(target_s / max(one, 1e-4)))
    t0 = time.perf_counter()
    f = m.run(f, steps, mask=mask, s=s)
    dt = time.perf_counter() - t0
    assert np.isfinite(f).all()
    mlups = n * steps / dt / 1e6
    cores = get_threads()
    # the same oracle on one thread, over a shorter window
    set_threads(1)
    try:
        t0 = time.perf_counter()
        f = m.run(f, 1, mask=mask, s=s)
        one1 = time.perf_counter() - t0
        steps1 = max(1, int(target_s / 3 / max(one1, 1e-4)))
        t0 = time.perf_counter()
        f = m.run(f, steps1, mask=mask, s=s)
        mlups1 = n * steps1 / (time.perf_counter() - t0) / 1e6
    finally:
        set_threads(cores)
    model = ""
    try:
        model = next(ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name"))
    except (OSError, StopIteration):
        pass
    dims = f"{wl.nx}x{ny}" + (f"x{nz}" if wl.nz > 1 else "")
    full = f"{wl.nx}x{wl.ny}" + (f"x{wl.nz}" if wl.nz > 1 else "")
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{wl.lattice} {dims} slab of the {full} grid, FP64, {steps} steps in {dt:.1f} s",
            "single_thread_value": round(mlups1, 3), "cpu_model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="throughput_2d", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--storage", default="f32", choices=("f32", "f16", "bf16"))
    ap.add_argument("--rounding", default="nearest", choices=("nearest", "stochastic"),
                    help="rounding of the stored 16-bit values")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the main step")
    ap.add_argument("--inplace", action="store_true",
                    help="time the in-place step (one state buffer) instead of the two-buffer step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB three times with a plain device copy (reference for HBM counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the checkpointed adjoint of the 128^3 soft-porosity workload (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the method runs on a "
              "single device here; multi-GPU domain decomposition is not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_09472_amd.lbm import Simulation

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_pipeline()}), flush=True)
        return

    wl = make_workload(args.workload)
    N = wl.N
    st = args.storage
    elem = 4 if st == "f32" else 2
    thermal = wl.lattice == "D1V7"
    k16 = F16_SCALE[args.workload] if st == "f16" else 0
    sim = Simulation(wl.lattice, wl.nx, wl.ny, wl.nz, tau=wl.tau, E=wl.E, B=wl.B, storage=st,
                     dev_scale_log2=k16, mask=wl.mask, s=wl.s, forcing=wl.forcing, slip=wl.slip,
                     inplace=args.inplace, theta=wl.theta, mu=wl.mu, rounding=args.rounding)
    if thermal:
        sim.init(wl.rho, wl.u, wl.thetabar)
    else:
        sim.init(wl.rho, wl.u)
    wall, ev = timed_steps(sim, args.steps, args.warmup)
    t_launch = ev / args.steps
    mlups = N * args.steps / wall / 1e6
    alg = algorithmic_bytes(wl, sim.Q, elem)
    achieved = alg / t_launch / 1e9
    traffic = None if (args.inplace or args.rounding != "nearest") else traffic_from_profile(
        f"{'k_thermal_step' if thermal else 'k_step'}_{wl.lattice}_{st}_{args.workload}")
    tot = sim.current()
    sim.close()
    del sim

    default = args.workload == "throughput_2d" and st == "f32"
    extras = {}
    if default and not args.no_extras:
        for s16s, k, rnd in (("f16", F16_SCALE["throughput_2d"], "nearest"), ("bf16", 0, "nearest"),
                             ("f16", F16_SCALE["throughput_2d"], "stochastic"), ("bf16", 0, "stochastic")):
            s16 = Simulation(wl.lattice, wl.nx, wl.ny, 1, tau=wl.tau, storage=s16s, dev_scale_log2=k, rounding=rnd)
            s16.init(wl.rho)
            w16, e16 = timed_steps(s16, args.steps, args.warmup)
            t16 = e16 / args.steps
            extras[s16s if rnd == "nearest" else s16s + "_stochastic_rounding"] = {
                "MLUPS": round(N * args.steps / w16 / 1e6, 1),
                "ms_per_step": round(w16 / args.steps * 1e3, 5),
                "achieved_GBs": round(bytes_per_node(s16.Q, 2) * N / t16 / 1e9, 1),
                "dev_scale_log2": k}
            s16.close()
        extras["adjoint"] = {}
        for key, forcing in (("step_only_4096sq", "source"), ("step_only_4096sq_shift", "shift")):
            t_adj, t_fwd = adjoint_ratio(wl, max(20, args.steps // 4), 5, forcing)
            # algorithmic bytes of one adjoint node update (FP32 state, no walls, no soft
            # porosity): read the state's Q values, read lambda(t+1), write lambda(t)
            gbs = 3 * wl_q(wl) * 4 * wl.N / t_adj / 1e9
            extras["adjoint"][key] = {"ms_per_step": round(t_adj * 1e3, 5),
                                      "forward_ms_per_step": round(t_fwd * 1e3, 5),
                                      "ratio_to_forward": round(t_adj / t_fwd, 3),
                                      "achieved_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        extras["adjoint"]["checkpointed_128cube"] = adjoint_pipeline()
        extras["inplace"] = {"f32": inplace_extra(wl, "f32", 0, args.steps, args.warmup),
                             "f16": inplace_extra(wl, "f16", F16_SCALE["throughput_2d"], args.steps, args.warmup)}
        extras["thermal"] = thermal_extra(args.steps, args.warmup)

    kernel = ("k_thermal_aa_pull+k_thermal_aa_local" if thermal and args.inplace else
              "k_thermal_step" if thermal else
              "k_step_aa_pull+k_step_aa_local" if args.inplace else "k_step") + \
        f"<{wl.lattice},{st.upper()}" + (",mask" if wl.mask is not None else "") + \
        (",slip" if wl.slip else "") + (",soft" if wl.s is not None else "") + \
        (",shift" if wl.forcing == "shift" else "") + (",stochastic" if args.rounding == "stochastic" else "") + ">"
    desc = WORKLOAD_DESC[args.workload] + {"f32": ", FP32", "f16": f", FP16 x 2^{k16}", "bf16": ", BF16"}[st] + \
        " deviation storage" + (", stochastic rounding" if args.rounding == "stochastic" else "") + \
        (", in-place step (one state buffer)" if args.inplace else "")
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
        "config": {"workload": desc, "lattice": wl.lattice, "nx": wl.nx, "ny": wl.ny, "nz": wl.nz, "storage": st},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel, "bytes_per_launch": alg,
                     "avg_launch_ms": round(t_launch * 1e3, 5)},
    }
    solid = solid_nodes(wl)
    if solid is not None:
        out["fluid_MLUPS"] = round(int((solid == 0).sum()) * args.steps / wall / 1e6, 1)
    if default:
        out["storage16"] = extras.get("f16") and {key: v for key, v in extras.items()
                                                  if key.startswith(("f16", "bf16"))}
        out["adjoint"] = extras.get("adjoint")
        out["inplace"] = extras.get("inplace")
        out["thermal"] = extras.get("thermal")
    out["mass_after_run"] = tot[0]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
        if default:
            # the stated error of each timed storage format: the oracle (FP64) against the
            # GPU step in the same launch configuration, on sampled blocks after 100 steps
            out["err"] = oracle_errors(wl, [("f32", 0), ("f16", F16_SCALE["throughput_2d"]), ("bf16", 0)])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
