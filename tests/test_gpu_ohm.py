"""Ohm's law on the full 2048x2048 disk packing (Sec. 9.4 at a larger size): E_x = k x 1e-7,
tau = 0.9, 20000 steps, in FP32, FP16 x 2^k and BF16 deviation storage.

* Against the FP64 oracle at the full size and length (``tests/golden/porous_ohm_E<k>e-7``,
  written by ``tests/golden/make_porous_ohm.py``, which calls only the oracle; about 100
  minutes of host time per field): FP32 rho and u on four full rows within 1e-5 (norm-wise,
  on the oracle's largest |rho| and |u| over all fluid nodes) and the FP64 totals M, P_x
  within 1e-5; FP16 total current P_x within 1e-3; BF16 errors stated (bounded loosely).
* The sweep over all 8 fields: the FP32 current is linear in E (J/E constant to 1e-4), and
  FP16 stays within 1e-3 of FP32 for every field.
"""
import glob
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_fields, gpu_sim

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def f16_scale(kE: int) -> int:
    # FP16 scale: deviations are ~ E x (steps to steady state); 2^k chosen per field
    return int(np.floor(np.log2(4096.0 / (kE * 1e-7 * 300.0))))


def _input_hash(wl) -> str:
    # the same recipe as the generator's
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(wl.mask, dtype=np.uint8).tobytes())
    h.update(np.ascontiguousarray(wl.rho, dtype=np.float64).tobytes())
    h.update(repr((wl.lattice, wl.nx, wl.ny, wl.nz, wl.tau, wl.steps)).encode())
    return h.hexdigest()


def _golden_fields():
    ks = []
    for p in sorted(glob.glob(os.path.join(GOLDEN, "porous_ohm_E*e-7.json"))):
        ks.append(int(os.path.basename(p)[len("porous_ohm_E"):-len("e-7.json")]))
    return ks


@pytest.mark.parametrize("kE", _golden_fields())
def test_ohm_full_size_vs_oracle(kE):
    gold = json.load(open(os.path.join(GOLDEN, f"porous_ohm_E{kE}e-7.json")))
    rows = np.load(os.path.join(GOLDEN, f"porous_ohm_E{kE}e-7.npz"))
    wl = W.porous_ohm_2d(Ex=kE * 1e-7)
    assert gold["workload"]["input_sha256"] == _input_hash(wl), "workload changed since the oracle reference"
    assert gold["workload"]["steps"] == wl.steps == 20000
    r = rows["rows"]
    mrow = wl.mask.reshape(wl.ny, wl.nx)[r] == 0
    res = {}
    for st, rounding in (("f32", "nearest"), ("f16", "nearest"), ("bf16", "nearest"), ("f16", "stochastic"),
                         ("bf16", "stochastic")):
        k16 = f16_scale(kE) if st == "f16" else 0
        sim = gpu_sim(wl, storage=st, dev_scale_log2=k16, rounding=rounding)
        sim.step(wl.steps)
        tot = sim.current()
        rho, u = gpu_fields(sim)
        sim.close()
        g = lambda a: a.reshape(wl.ny, wl.nx)[r][mrow]
        er = np.abs(g(rho) - rows["rho"][mrow]).max() / gold["max_abs"]["rho"]
        eux = np.abs(g(u[0]) - rows["ux"][mrow]).max()
        euy = np.abs(g(u[1]) - rows["uy"][mrow]).max()
        eu = max(eux, euy) / max(gold["max_abs"]["ux"], gold["max_abs"]["uy"])
        eM = abs(tot[0] / gold["M"] - 1)
        eP = abs(tot[1] / gold["Px"] - 1)
        res[st if rounding == "nearest" else st + "-sr"] = (er, eu, eM, eP)
        print(f"E = {kE}e-7 {st}{f' x 2^{k16}' if st == 'f16' else ''} {rounding}: rho {er:.2e}, u {eu:.2e} "
              f"(rows {list(r)}), M {eM:.2e}, P_x {eP:.2e}")
    er, eu, eM, eP = res["f32"]
    assert er < 1e-5 and eu < 1e-5 and eM < 1e-5 and eP < 1e-5, res["f32"]
    assert res["f16"][3] < 1e-3, res["f16"]
    assert res["f16"][2] < 1e-5 and res["bf16"][2] < 1e-5
    assert res["bf16"][3] < 2e-2 and res["bf16"][1] < 5e-2, res["bf16"]
    # stochastic rounding (measured at E = 1e-7: P_x 9.4e-7 FP16, 4.7e-6 BF16)
    assert res["f16-sr"][3] < 1e-4 and res["f16-sr"][2] < 1e-5, res["f16-sr"]
    assert res["bf16-sr"][3] < 1e-3 and res["bf16-sr"][1] < 5e-2, res["bf16-sr"]


def test_ohm_sweep_full_size():
    base = W.porous_ohm_2d(Ex=1e-7)
    steps = base.steps
    res = {}
    for kE in range(1, 9):
        E = (kE * 1e-7, 0.0, 0.0)
        k = f16_scale(kE)
        row = {}
        for st in ("f32", "f16", "bf16"):
            sim = gpu_sim(base, storage=st, dev_scale_log2=k if st == "f16" else 0, E=E)
            sim.step(steps)
            t = sim.current()
            row[st] = t[1]
            sim.close()
        res[kE] = row
        print(f"E={kE}e-7 k={k}: Px f32 {row['f32']:.9e} f16 {row['f16']:.9e} ({abs(row['f16']/row['f32']-1):.2e}) "
              f"bf16 {row['bf16']:.9e} ({abs(row['bf16']/row['f32']-1):.2e})")
    ratios = np.array([res[k]["f32"] / (k * 1e-7) for k in res])
    spread = (ratios.max() - ratios.min()) / ratios.mean()
    print(f"FP32 J/E spread over 8 fields: {spread:.2e}")
    assert ratios.min() > 0 and spread < 1e-4
    for k in res:
        assert abs(res[k]["f16"] / res[k]["f32"] - 1) < 1e-3, k
        assert abs(res[k]["bf16"] / res[k]["f32"] - 1) < 2e-2, k
