"""The in-place time step (one state buffer, the AA access pattern), through the C ABI.

* Against the FP64 oracle: rho, u (FP32 bar 1e-5 relative over fluid nodes) and the
  populations, after an odd and an even number of steps (the state is then in the
  streamed and in the two-buffer layout), with obstacles, partial bounce-back, free-slip
  walls, both forcing schemes and ragged rows.
* Against the two-buffer step: bit for bit (same node arithmetic) for every storage,
  at small sizes and at the full 4096^2 D2V9 and 256x128^2 D3V19 sizes, for the fields,
  the FP64 totals, the exported populations and the state that lbm_get_state returns.
* State hand-over: a state taken from an in-place handle after an odd number of steps
  continues on a two-buffer handle and on the in-place handle itself with the same bits.
* lbm_get_state into the handle's own buffer is refused at odd parity.
"""
import numpy as np
import pytest
import torch

from paper_1710_09472_amd import lbm
from paper_1710_09472_amd import workloads as W
from parity_helpers import (gpu_fields, gpu_sim, oracle_fields, oracle_window_fields, permutation_to_oracle,
                            rel_errors)

pytestmark = pytest.mark.gpu

TOL = 1e-5

CASES = [
    # name, lattice, shape, seed, obstacle fraction, soft, E, B, forcing, slip
    ("d2-periodic-EB", "D2V9", (300, 9, 1), 1, 0.0, False, (2e-4, -1e-4, 0), (0, 0, 4e-3), "source", 0),
    ("d2-disks-soft", "D2V9", (257, 7, 1), 2, 0.15, True, (2e-4, 5e-5, 0), (0, 0, 3e-3), "source", 0),
    ("d2-shift-slip", "D2V9", (300, 9, 1), 3, 0.1, False, (2e-4, -1e-4, 0), (0, 0, 4e-3), "shift", 1),
    ("d3-source-bb-B", "D3V19", (33, 7, 5), 5, 0.1, False, (1e-4, 0, 0), (0, 0, 2e-3), "source", 0),
    ("d3-shift-slip-yz-soft", "D3V19", (260, 6, 7), 4, 0.08, True, (1e-4, 3e-5, -2e-5), (2e-3, -1e-3, 3e-3),
     "shift", 3),
    ("d3-tiny", "D3V19", (5, 3, 3), 6, 0.0, False, (1e-4, 0, 0), (0, 0, 1e-3), "shift", 3),
]


def _case(lattice, shape, seed, phi, soft, E, B, forcing, slip):
    wl = W.random_fields(lattice, *shape, seed=seed, solid_fraction=phi, soft=soft, umax=0.02)
    wl.tau, wl.E, wl.B, wl.forcing, wl.slip = 0.7, E, B, forcing, slip
    if wl.s is not None:
        wl.s = 0.3 * wl.s
    return wl


@pytest.mark.parametrize("steps", [25, 26])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_inplace_oracle_parity(case, steps):
    wl = _case(*case[1:])
    sim = gpu_sim(wl, inplace=True)
    sim.step(steps)
    rho, u = gpu_fields(sim)
    rho_o, u_o, m, f_o = oracle_fields(wl, steps)
    solid = m._mask(wl.mask)
    solid = np.zeros(m.N, np.uint8) if solid is None else solid
    er, eu = rel_errors(rho, u, rho_o, u_o, solid)
    assert er < TOL and eu < TOL, (er, eu)
    fl = solid == 0
    perm = permutation_to_oracle(sim, m)
    fo = f_o.reshape(m.Q, m.N)
    for f_gpu in (sim.export_f64(), sim.export_f64(sim.get_state())):
        np.testing.assert_allclose(f_gpu.cpu().numpy()[perm][:, fl], fo[:, fl], rtol=0, atol=2e-6 * np.abs(fo).max())
    tot, tot_o = sim.current(), m.totals(f_o, wl.mask)
    assert abs(tot[0] / tot_o[0] - 1) < 1e-6


def _same(a, b):
    """Both handles hold the same state: fields, totals, populations and returned state."""
    ra, ua = a.moments()
    rb, ub = b.moments()
    assert torch.equal(ra, rb) and torch.equal(ua, ub)
    assert np.array_equal(a.current(), b.current())
    fa = a.export_f64()
    assert torch.equal(fa, b.export_f64())
    assert torch.equal(fa, a.export_f64(b.get_state()))
    assert torch.equal(fa, b.export_f64(a.get_state()))


STORAGES = [("f32", 0), ("f16", 14), ("bf16", 0)]


@pytest.mark.parametrize("steps", [1, 2, 7])
@pytest.mark.parametrize("storage,k", STORAGES, ids=[s for s, _ in STORAGES])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_inplace_matches_two_buffer(case, storage, k, steps):
    wl = _case(*case[1:])
    two = gpu_sim(wl, storage=storage, dev_scale_log2=k)
    one = gpu_sim(wl, storage=storage, dev_scale_log2=k, inplace=True)
    two.step(steps)
    one.step(steps)
    _same(one, two)


@pytest.mark.parametrize("storage,k", STORAGES, ids=[s for s, _ in STORAGES])
def test_state_hand_over(storage, k):
    wl = _case(*CASES[4][1:])
    ref = gpu_sim(wl, storage=storage, dev_scale_log2=k)
    ref.step(12)
    one = gpu_sim(wl, storage=storage, dev_scale_log2=k, inplace=True)
    one.step(5)
    st = one.get_state()
    two = gpu_sim(wl, storage=storage, dev_scale_log2=k)
    two.set_state(st)
    two.step(7)
    _same(two, ref)
    one.set_state(st)  # back to the two-buffer layout of step 5
    one.step(7)
    _same(one, ref)
    # a checkpoint recomputed with lbm_step_from from the in-place handle's state
    dst = one.new_state()
    one2 = gpu_sim(wl, storage=storage, dev_scale_log2=k, inplace=True)
    one2.step(11)
    one2.step_from(one2.get_state(), dst)
    two.set_state(dst)
    _same(two, ref)


def test_get_state_into_own_buffer_refused():
    wl = _case(*CASES[1][1:])
    one = gpu_sim(wl, inplace=True)
    one.step(3)
    with pytest.raises(lbm.LbmError) as err:
        one.get_state(one.bufs[0])
    assert err.value.code == lbm.LBM_EINVAL


FULL = [
    ("throughput_4096sq", W.throughput_2d, [("f32", 0), ("f16", 12), ("bf16", 0)], 41),
    ("hall_duct_3d", W.hall_duct_3d, [("f32", 0), ("f16", 16), ("bf16", 0)], 21),
    ("porous_ohm_2048sq", W.porous_ohm_2d, [("f32", 0), ("f16", 20)], 21),
    ("soft_porous_3d", W.soft_porous_3d, [("f32", 0)], 21),
    ("ohm_paper_3d", lambda: W.ohm_paper_3d(Ex=1e-5), [("f32", 0), ("f16", 20)], 21),
]


@pytest.mark.parametrize("name,builder,storages,steps", FULL, ids=[c[0] for c in FULL])
def test_inplace_full_size_bitwise(name, builder, storages, steps):
    """Odd and even step counts at the workloads' full sizes, every storage."""
    wl = builder()
    for storage, k in storages:
        two = gpu_sim(wl, storage=storage, dev_scale_log2=k)
        one = gpu_sim(wl, storage=storage, dev_scale_log2=k, inplace=True)
        for n in (steps, 1):
            two.step(n)
            one.step(n)
            ra, ua = one.moments()
            rb, ub = two.moments()
            assert torch.equal(ra, rb) and torch.equal(ua, ub), (storage, n)
            assert np.array_equal(one.current(), two.current()), (storage, n)
        fa = one.export_f64(one.get_state())
        assert torch.equal(fa, two.export_f64()), storage
        del fa, one, two
        torch.cuda.empty_cache()


def test_inplace_full_size_oracle_windows():
    """The 4096^2 D2V9 grid after 41 in-place steps (odd layout) against the oracle on
    sampled blocks (their dependence cones)."""
    wl = W.throughput_2d()
    sim = gpu_sim(wl, inplace=True)
    sim.step(41)
    rho, u = gpu_fields(sim)
    for centre in ((0, 0, 0), (4095, 4095, 0), (1000, 3000, 0)):
        glob, rho_o, u_o = oracle_window_fields(wl, 41, 12, centre)
        er, eu = rel_errors(rho[glob], u[:, glob], rho_o, u_o)
        assert er < TOL and eu < TOL, (centre, er, eu)
