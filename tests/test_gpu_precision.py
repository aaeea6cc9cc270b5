"""16-bit deviation storage (FP16 x 2^k and BF16): the codec, and the error of every
workload against the FP64 oracle.

Codec: every one of the 65,536 stored codes decodes exactly (export through the C ABI
against numpy's float16 / a bit-level bfloat16 decode), and encoding is round to nearest
even (initial states whose stored values are one FP32 product each, against numpy).
Errors: the max-norm errors of rho and u and the relative error of the total current
are printed for every workload (they are the stated precision of the 16-bit paths) and
held to the bounds below; the FP16 total current stays within 1e-3 of the oracle.
"""
import numpy as np
import pytest
import torch

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W
from parity_helpers import gpu_fields, gpu_sim, oracle_fields, oracle_window_fields, rel_errors

pytestmark = pytest.mark.gpu


def _bf16_decode(codes):
    with np.errstate(invalid="ignore"):  # signalling NaN codes
        return (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _bf16_rne(x32):
    """Round float32 values to bfloat16 codes, nearest even (bit-level reference)."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x32)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


@pytest.mark.parametrize("storage,k", [("f16", 0), ("f16", 13), ("bf16", 0)])
def test_decode_all_codes(storage, k):
    N = 65536
    sim = lbm.Simulation("D2V9", N, 1, 1, tau=0.8, storage=storage, dev_scale_log2=k, rho0=1e-300)
    codes = np.arange(N, dtype=np.uint16)
    raw = np.zeros(sim.sizes["state"] // 2, dtype=np.uint16)
    raw[:N] = codes  # rest population, which the pull delivers in place
    sim.set_state(torch.from_numpy(raw.view(np.uint8)).cuda())
    # the export adds what_0 rho0 (here ~1e-301) in FP64; take it off again exactly
    f = sim.export_f64().cpu().numpy()[0] - sim.constants["what"][0] * 1e-300
    if storage == "f16":
        want = codes.view(np.float16).astype(np.float64) * 2.0 ** (-k)
    else:
        want = _bf16_decode(codes)
    np.testing.assert_array_equal(np.isnan(f), np.isnan(want))
    ok = ~np.isnan(want)
    np.testing.assert_array_equal(f[ok], want[ok])


@pytest.mark.parametrize("storage,k", [("f16", 0), ("f16", 10), ("bf16", 0)])
def test_encode_round_to_nearest_even(storage, k):
    """u = 0: the stored value of population q at node x is what_q * (rho(x + e_q) - rho0),
    one FP32 product, then encoded."""
    nx, ny = 4096, 2
    rng = np.random.default_rng(9)
    mag = 10.0 ** rng.uniform(-9, -1.5, nx * ny)
    drho = np.where(rng.uniform(size=nx * ny) < 0.5, -mag, mag)
    rho = 1.0 + drho
    sim = lbm.Simulation("D2V9", nx, ny, 1, tau=0.8, storage=storage, dev_scale_log2=k)
    sim.init(rho)
    raw = sim.get_state().cpu().numpy().view(np.uint16).reshape(sim.Q, sim.stride)[:, : nx * ny]
    what = np.array(sim.constants["what"], dtype=np.float32)
    d32 = (rho - 1.0).astype(np.float32).reshape(ny, nx)
    checked = 0
    for q in range(1, sim.Q):
        ex, ey, _ = sim.e[q]
        shell = ex * ex + ey * ey
        target = np.roll(d32, shift=(-ey, -ex), axis=(0, 1)).reshape(-1)  # value at x + e_q
        val = np.float32(what[shell]) * target  # FP32 product, RNE
        if storage == "f16":
            want = (val * np.float32(2.0 ** k)).astype(np.float16).view(np.uint16)
        else:
            want = _bf16_rne(val.astype(np.float32))
        np.testing.assert_array_equal(raw[q], want)
        checked += want.size
    assert checked == 8 * nx * ny


def _f16_scale(wl, steps):
    """dev_scale_log2 with max|d| * 2^k about 2^12, from an FP32 run of the same length."""
    sim = gpu_sim(wl)
    sim.step(steps)
    f = sim.export_f64().cpu().numpy()
    what = np.array(sim.constants["what"])
    sh = (sim.e ** 2).sum(1)
    dev = f - (what[sh] * 1.0)[:, None]
    if wl.mask is not None:
        dev = dev[:, wl.mask == 0]
    m = np.abs(dev).max()
    return int(np.clip(np.floor(np.log2(4096.0 / m)), 0, 40))


def _current_err(sim, tot_ref):
    t = sim.current()
    return abs(t[1] - tot_ref[1]) / abs(tot_ref[1])


# Bounds: measured errors with margin. FP16 keeps 11 significant bits of the scaled
# deviations and BF16 8: where the per-step force increment is ~1e-3 of the stored
# deviations (the Poiseuille channel at t = 2000, whose centre speed still grows by
# 1/1000 per step) the increment is quantised and the flow error reaches ~1e-2 in FP16;
# where the flow is near its steady state (porous media) the FP16 total current stays
# within 1e-3 of the FP64 oracle. At the shock front of the tube the error is largest.
# In the Poiseuille channel BF16 cannot resolve the per-step force increment at all
# (u and the current lag the oracle by ~45 %): that error is stated, not bounded.
#
# Stochastic rounding (-sr) keeps the sub-ulp increments on average: measured on MI355X,
# the Poiseuille u error falls from 9.4e-3 to 5.8e-4 (FP16) and from 0.44 to 5.6e-3
# (BF16), the porous total current from 2.9e-4 to 2.8e-5 (FP16) and from 1.8e-3 to
# 1.7e-4 (BF16). Its rounding errors are zero-mean but up to a whole unit, and they
# random-walk: in the shock tube, whose deviations are large (drho ~ 0.1), BF16 with
# stochastic rounding has the larger max-norm error (u 0.26 against 0.039), FP16 the
# smaller (9.6e-3 against 6.3e-2).
FULL = [
    # name, builder, steps, bounds (rho, u, current) for f16 and bf16, round to nearest and
    # stochastic rounding (-sr)
    ("poiseuille_64x32", W.poiseuille_2d, 2000,
     {"f16": (1e-5, 3e-2, 3e-2), "bf16": (1e-4, 1.0, 1.0), "f16-sr": (5e-6, 3e-3, 5e-4), "bf16-sr": (3e-5, 3e-2, 5e-4)}),
    ("riemann_4096x4", W.riemann_2d, 1500,
     {"f16": (3e-2, 2e-1, None), "bf16": (2e-1, 1.0, None), "f16-sr": (1e-2, 5e-2, None), "bf16-sr": (2e-1, 1.0, None)}),
    ("porous_256sq", lambda: W.porous_ohm_2d(n=256, Ex=4e-7, seed=5), 3000,
     {"f16": (1e-6, 5e-3, 1e-3), "bf16": (1e-5, 5e-2, 1e-2), "f16-sr": (1e-6, 3e-3, 3e-4),
      "bf16-sr": (1e-5, 3e-2, 2e-3)}),
]


@pytest.mark.parametrize("name,builder,steps,bounds", FULL, ids=[c[0] for c in FULL])
def test_16bit_error_full_grid(name, builder, steps, bounds):
    wl = builder()
    rho_o, u_o, m, f_o = oracle_fields(wl, steps)
    tot_o = m.totals(f_o, wl.mask)
    k = _f16_scale(wl, steps)
    res = {}
    for st, rounding in (("f32", "nearest"), ("f16", "nearest"), ("bf16", "nearest"), ("f16", "stochastic"),
                         ("bf16", "stochastic")):
        sim = gpu_sim(wl, storage=st, dev_scale_log2=k if st == "f16" else 0, rounding=rounding)
        sim.step(steps)
        rho, u = gpu_fields(sim)
        er, eu = rel_errors(rho, u, rho_o, u_o, wl.mask)
        ec = _current_err(sim, tot_o) if abs(tot_o[1]) > 0 else float("nan")
        key = st if rounding == "nearest" else st + "-sr"
        res[key] = (er, eu, ec)
        print(f"{name} {st}{'(k=%d)' % k if st == 'f16' else ''} {rounding}: rho {er:.2e} u {eu:.2e} "
              f"current {ec:.2e}")
    for key in ("f16", "bf16", "f16-sr", "bf16-sr"):
        er, eu, ec = res[key]
        br, bu, bc = bounds[key]
        assert er < br and eu < bu, (key, er, eu)
        if bc is not None:
            assert ec < bc, (key, ec)


# The 4096^2 grid is checked at the FP16 scale the benchmark times it with (2^12; its initial
# deviations reach ~0.03, so 2^12 keeps them below FP16's largest value with headroom, while
# every deviation after 100 steps stays in FP16's normal range), in the benchmark's launch
# configuration: the errors the benchmark states.
F16_SCALE_BENCH = 12
SAMPLED = [
    ("throughput_4096sq", W.throughput_2d, 100, [(0, 0, 0), (2048, 2048, 0)], 16,
     {"f16": (1e-5, 3e-3), "bf16": (1e-4, 2e-2)}),
    ("throughput_4096sq_calibrated_k", W.throughput_2d, 100, [(2048, 2048, 0)], 16,
     {"f16": (1e-5, 3e-3), "bf16": (1e-4, 2e-2)}),
    ("hall_duct_3d", W.hall_duct_3d, 30, [(0, 0, 0), (128, 64, 64)], 6, {"f16": (1e-6, 1e-3), "bf16": (1e-6, 5e-3)}),
    ("soft_porous_3d", W.soft_porous_3d, 30, [(64, 64, 64)], 6, {"f16": (1e-6, 1e-3), "bf16": (1e-6, 5e-3)}),
    ("porous_ohm_2048sq", lambda: W.porous_ohm_2d(Ex=8e-7), 200, [(1024, 1500, 0)], 16,
     {"f16": (1e-6, 2e-3), "bf16": (1e-5, 1e-2)}),
]


@pytest.mark.parametrize("name,builder,steps,centres,core,bounds", SAMPLED, ids=[c[0] for c in SAMPLED])
def test_16bit_error_sampled(name, builder, steps, centres, core, bounds):
    wl = builder()
    k = F16_SCALE_BENCH if name == "throughput_4096sq" else _f16_scale(wl, steps)
    ref = [oracle_window_fields(wl, steps, core, c) for c in centres]
    res = {}
    for st in ("f32", "f16", "bf16"):
        sim = gpu_sim(wl, storage=st, dev_scale_log2=k if st == "f16" else 0)
        sim.step(steps)
        rho, u = gpu_fields(sim)
        er = eu = 0.0
        for idx, rho_o, u_o in ref:
            m = None if wl.mask is None else wl.mask[idx]
            a, b = rel_errors(rho[idx], u[:, idx], rho_o, u_o, m)
            er, eu = max(er, a), max(eu, b)
        res[st] = (er, eu)
        print(f"{name} {st}{'(k=%d)' % k if st == 'f16' else ''}: rho {er:.2e} u {eu:.2e} (sampled blocks)")
    for st in ("f16", "bf16"):
        br, bu = bounds[st]
        assert res[st][0] < br and res[st][1] < bu, (st, res[st])
