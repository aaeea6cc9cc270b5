"""Build the HIP library ``liblbm_hip.so`` in-tree for gfx950.

Sources: ``csrc/lbm_kernels.hip`` (device kernels and launchers; device helpers in
``csrc/lbm_device.h``), ``csrc/lbm_aa.hip`` (the in-place step), ``csrc/lbm_thermal.hip``
(the fourth-order thermal model on D1V7), ``csrc/lbm_density.hip``
(rho <-> mu), ``csrc/lbm_capi.cpp`` (the C ABI of ``include/lbm.h``) and
``csrc/lbm_consts.cpp`` (host FP64 constants).
Every source goes through hipcc with packed-FP32 instruction selection disabled.

Usage: ``python -m paper_1710_09472_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
BUILD = PKG / "_build"
LIB = PKG / "liblbm_hip.so"
SOURCES = ["lbm_kernels.hip", "lbm_aa.hip", "lbm_step_sr.hip", "lbm_aa_sr.hip", "lbm_thermal.hip", "lbm_density.hip", "lbm_capi.cpp", "lbm_consts.cpp"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def compile_flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


def build(verbose: bool = False) -> Path:
    """Compile every source and link the shared library; always rebuilds."""
    BUILD.mkdir(exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = BUILD / (src.replace(".", "_") + ".o")
        objs.append(obj)
        # every source, .cpp included, is compiled as HIP: the host files include the HIP
        # runtime header through lbm_internal.h, and one language keeps one set of flags
        cmd = [hipcc(), *compile_flags(), "-x", "hip", "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
        elif verbose and lines:
            print("\n".join(lines), flush=True)
    if failed:
        msg = "\n\n".join(f"--- {s} ---\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
