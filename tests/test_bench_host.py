"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic bytes that
the roofline divides by the measured launch time, and the rule that HBM traffic from
the committed counters is reported only while the kernel code is the code they were
taken on."""
import shutil
import subprocess
import sys
from pathlib import Path

import numpy as np

import bench
from paper_1710_09472_amd import workloads as W

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    wl = W.throughput_2d(nx=64, ny=32)
    assert bench.algorithmic_bytes(wl, 9, 4) == 64 * 32 * 72
    assert bench.algorithmic_bytes(wl, 9, 2) == 64 * 32 * 36
    # obstacles: fluid nodes move their populations, every node has one byte of flag;
    # a porosity field adds 4 bytes per node
    wl = W.random_fields("D3V19", 10, 6, 5, seed=3, solid_fraction=0.2, soft=True)
    fluid = int((wl.mask == 0).sum())
    assert 0 < fluid < wl.N
    assert bench.algorithmic_bytes(wl, 19, 4) == fluid * 152 + wl.N + 4 * wl.N
    assert bench.wl_q(wl) == 19


def _copy_sources(tmp: Path) -> Path:
    dst = tmp / "paper_1710_09472_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in ("lbm_device.h", "lbm_step_kernels.h", "lbm_kernels.hip", "lbm_thermal.hip"):
        shutil.copy(ROOT / "paper_1710_09472_amd" / "csrc" / name, dst / name)
    return dst


def test_code_hash_ignores_comments_not_code(tmp_path, monkeypatch):
    ref, ref_th = bench.kernel_code_hash(), bench.kernel_code_hash(thermal=True)
    src = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    assert bench.kernel_code_hash() == ref
    f = src / "lbm_kernels.hip"
    f.write_text("// a comment line\n\n" + f.read_text().replace("\n", "  // trailing note\n", 1))
    assert bench.kernel_code_hash() == ref
    f.write_text(f.read_text() + "\nstatic int unused_marker = 0;\n")
    assert bench.kernel_code_hash() != ref
    # the thermal step's hash covers the device header and the thermal kernel file only
    assert bench.kernel_code_hash(thermal=True) == ref_th


def test_traffic_only_for_the_code_it_was_taken_on(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_DIR", tmp_path)
    tag = "k_step_D2V9_f32_throughput_2d"
    assert bench.traffic_from_profile(tag) is None  # no summary
    good = bench.kernel_code_hash()
    (tmp_path / f"{tag}_pmc.txt").write_text(f"hbm_bytes_per_launch: 1.25e+09\nkernel_code_sha256: {good}\n")
    assert np.isclose(bench.traffic_from_profile(tag), 1.25e9)
    (tmp_path / f"{tag}_pmc.txt").write_text("hbm_bytes_per_launch: 1.25e+09\nkernel_code_sha256: " + "0" * 64 + "\n")
    assert bench.traffic_from_profile(tag) is None


def test_oracle_blocks_equal_the_full_grid_oracle(oracle_lib):
    """The error figures of bench.py compare the GPU with the oracle on sampled blocks that the
    oracle recomputes on the windows of their dependence cones: on a grid the oracle runs
    whole, the blocks equal the full-grid run exactly (also where a window wraps around)."""
    wl = W.throughput_2d(nx=96, ny=80, seed=3)
    wl.u = 0.01 * np.random.default_rng(4).standard_normal((2, wl.N))
    steps, core = 12, 8
    centres = ((0, 0, 0), (90, 40, 0), (47, 79, 0))
    idx, rho_b, u_b = bench.oracle_blocks(wl, steps, core, centres)
    m = oracle_lib.OracleModel("D2V9", wl.nx, wl.ny, 1, tau=wl.tau)
    rho, u = m.moments(m.run(m.init_state(wl.rho, wl.u), steps))
    assert idx.size == len(centres) * core * core
    np.testing.assert_array_equal(rho_b, rho[idx])
    np.testing.assert_array_equal(u_b, u[:, idx])
    # the block of centre (90, 40) holds x = 90..95 and 0..1 (wrapped), y = 40..47
    b = idx[core * core:2 * core * core]
    assert set(b % wl.nx) == set(range(90, 96)) | {0, 1} and set(b // wl.nx) == set(range(40, 48))
