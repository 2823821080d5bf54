"""MI355X (gfx950) implementation of the per-sample spectral hot path of
multilevel Monte Carlo for honeycomb materials with random vacancies.

The compute lives in ``libmlmc.so`` (HIP kernels behind the C ABI of
``include/mlmc.h``); :mod:`paper_1611_09784_amd.binding` marshals torch
tensors to it and :mod:`paper_1611_09784_amd.driver` runs the MC / MLMC
sample-allocation loop on the host.  Importing this package does not load
the library; the first binding call does, and fails loudly if it is missing.
"""

__all__ = ["binding", "driver"]
