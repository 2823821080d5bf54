"""Named synthetic workloads (sizes, seeds, grids) of the paper's experiments.

Only parameters live here; every computation on them happens either in the
HIP library or in the oracle.  Energies are in eV.

The workloads follow the paper's setting (Section 4): graphene and an
MoS2-shaped 11-orbital honeycomb model, iid vacancies with probability p on an
N x N supercell, a K x K Brillouin-zone grid with N*K held constant across
levels, and a smoothed integrated density of states on a uniform energy grid.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .lattices import Lattice, graphene, lattice_by_name, mos2_shaped

KGRID_MP = 0      # Monkhorst-Pack K x K grid
KGRID_GAMMA = 1   # Gamma-centred K x K grid
KGRID_RHOMBI = 2  # three-rhombus lattice of the hexagonal zone, 3 K^2 points
SMOOTH_GAUSS = 0  # g(x) = erfc(x / sqrt 2) / 2
SMOOTH_CUBIC = 1  # compactly supported cubic meeting the q = 0, 1 moment conditions


def energy_grid(lo: float, hi: float, n: int) -> np.ndarray:
    """Uniform grid of n energies on [lo, hi] (both ends included)."""
    if n == 1:
        return np.array([lo], dtype=np.float64)
    return lo + (hi - lo) * np.arange(n, dtype=np.float64) / (n - 1)


def mos2_energy_window(lat: Lattice) -> tuple:
    """Energy window for MoS2-shaped runs: the per-orbital hopping bound,
    which bounds every spectrum of the model, plus 1 eV, rounded out to 0.5 eV."""
    b = lat.hop_magnitude_bound() + 1.0
    b = math.ceil(b * 2.0) / 2.0
    return (-b, b)


@dataclass(frozen=True)
class Workload:
    name: str
    lattice: str
    N: int                    # supercell side (finest level for MLMC)
    p: float
    K: int                    # k-grid side at N
    kgrid: int
    M: int                    # samples (plain MC) or pilot samples (MLMC)
    seed: int
    n_eps: int
    eps_lo: float
    eps_hi: float
    delta: float
    smoother: int = SMOOTH_GAUSS
    levels: tuple = field(default_factory=tuple)   # MLMC: supercell sides per level
    NK: int = 0                                    # MLMC: N*K held constant
    tol: float = 0.0                               # MLMC: relative tolerance

    def make_lattice(self) -> Lattice:
        return lattice_by_name(self.lattice)

    def eps(self) -> np.ndarray:
        return energy_grid(self.eps_lo, self.eps_hi, self.n_eps)


WORKLOADS = {
    # Plain MC, graphene N=4 (32 sites), MP 4x4, M=100, 201 energies on [-9, 9].
    "graphene_n4_mc": Workload("graphene_n4_mc", "graphene", N=4, p=0.05, K=4,
                               kgrid=KGRID_MP, M=100, seed=101, n_eps=201,
                               eps_lo=-9.0, eps_hi=9.0, delta=0.1),
    # Plain MC, graphene N=16 (512 sites), MP 8x8, M=2000 (128k eigensolves), 401 energies.
    "graphene_n16_mc": Workload("graphene_n16_mc", "graphene", N=16, p=0.05, K=8,
                                kgrid=KGRID_MP, M=2000, seed=202, n_eps=401,
                                eps_lo=-9.0, eps_hi=9.0, delta=0.05),
    # MLMC graphene, levels N = 4, 8, 16, 32 with N*K = 32 (Gamma grids).
    "graphene_mlmc": Workload("graphene_mlmc", "graphene", N=32, p=0.02, K=1,
                              kgrid=KGRID_GAMMA, M=16, seed=303, n_eps=401,
                              eps_lo=-9.0, eps_hi=9.0, delta=0.05,
                              levels=(4, 8, 16, 32), NK=32, tol=1e-3),
    # The graphene N=16 plain-MC workload in the non-orthogonal model of
    # Section 3.1 (t = -3.033 eV, s = 0.129, eps_2p = 0): generalised problems.
    "graphene_n16_overlap_mc": Workload("graphene_n16_overlap_mc", "graphene_overlap", N=16, p=0.05, K=8,
                                        kgrid=KGRID_MP, M=2000, seed=202, n_eps=401,
                                        eps_lo=-8.0, eps_hi=16.0, delta=0.05),
    # MoS2-shaped, N = 4, 8, 16 with a 6x6 grid at every N.
    "mos2_mlmc": Workload("mos2_mlmc", "mos2_shaped", N=16, p=0.02, K=6,
                          kgrid=KGRID_GAMMA, M=16, seed=404, n_eps=401,
                          eps_lo=float("nan"), eps_hi=float("nan"), delta=0.05,
                          levels=(4, 8, 16), NK=0, tol=1e-3),
}


def workload_eps(w: Workload) -> np.ndarray:
    if w.lattice in ("graphene", "graphene_overlap"):
        return w.eps()
    lo, hi = mos2_energy_window(mos2_shaped())
    return energy_grid(lo, hi, w.n_eps)
