"""Ohm's law on the full 2048x2048 disk packing (Sec. 9.4 at a larger size): 8 fields
E_x = 1..8 x 1e-7, tau = 0.9, 20000 steps each, in FP32, FP16 x 2^k and BF16 storage.

* FP32: the mean current is linear in E (J/E constant across the 8 fields to 1e-4).
* FP16 and BF16: total current against the FP32 run of the same field (the FP32 path is
  held to 1e-5 of the FP64 oracle by the parity tests; the oracle itself would need
  ~20 minutes of host time per field at this size). FP16 within 1e-3 for every field.
"""
import numpy as np
import pytest

from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_sim

pytestmark = pytest.mark.gpu


def test_ohm_sweep_full_size():
    base = W.porous_ohm_2d(Ex=1e-7)
    steps = base.steps
    res = {}
    for kE in range(1, 9):
        E = (kE * 1e-7, 0.0, 0.0)
        # FP16 scale: deviations are ~ E * (steps to steady state); 2^k chosen per field
        k = int(np.floor(np.log2(4096.0 / (kE * 1e-7 * 300.0))))
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
