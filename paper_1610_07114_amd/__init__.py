"""MI355X-native thermal cascaded lattice Boltzmann method (TCLBM) hot path.

The compute path is the HIP library ``libtclbm.so`` (C ABI declared in
``include/tclbm.h``); :mod:`paper_1610_07114_amd.tclbm` is its thin ctypes
binding.  :mod:`paper_1610_07114_amd.workloads` generates seeded inputs.
"""
__all__ = ["tclbm", "workloads"]
