"""MI355X-native classical Ewald summation (energy, forces, dE/dq).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``libewald_mi355x.so``, declared in ``include/ewald.h``); the Python
side only marshals arguments.  Import :mod:`paper_1708_01135_amd.ewald` for the
binding and :mod:`paper_1708_01135_amd.workloads` for seeded inputs.
"""
__all__ = ["ewald", "workloads"]
