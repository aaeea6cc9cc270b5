"""Semiclassical (Fermi-Dirac) lattice Boltzmann step for AMD Instinct MI355X (gfx950).

The compute path is a C-ABI shared library of hand-written HIP kernels
(``liblbm_hip.so``, declared in ``include/lbm.h``); :mod:`.lbm` is its thin ctypes
binding. The library is loaded lazily, so importing this package (for instance for
:mod:`.workloads`) does not need a GPU.
"""

__all__ = ["workloads", "lbm"]
