"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This package holds *data* only: lattice descriptions (geometry, orbital
groups and hopping tables), energy grids and the named workload
configurations.  It contains none of the method's arithmetic (no k-grids,
no Hamiltonian assembly, no eigenvalues, no density of states, no
estimators), so that the oracle and the GPU path can both consume it
without sharing any computation.
"""

from .lattices import Lattice, graphene, graphene_overlap, mos2_shaped, lattice_by_name  # noqa: F401
from .configs import WORKLOADS, energy_grid, Workload  # noqa: F401
