"""Pins for the density of states by numerical differentiation of the IDoS
(Section 4.3) and for the host-side C-ABI version of it."""

import math

import numpy as np
import pytest

import oracle
from oracle import mlmc
from mlmc_inputs import energy_grid
from mlmc_inputs.configs import KGRID_GAMMA, SMOOTH_GAUSS


def nonuniform_grid(n, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.uniform(0.05, 0.2, n)) - 3.0


def test_oracle_dos_is_exact_for_quadratics():
    """A three-point second-order formula differentiates quadratics exactly,
    at interior and end points, on an unequal grid."""
    x = nonuniform_grid(40, 1)
    f = 0.3 * x * x - 1.7 * x + 0.25
    assert np.abs(mlmc.dos_from_idos(x, f) - (0.6 * x - 1.7)).max() < 1e-12
    # a cubic is not differentiated exactly: the formula is second order
    assert np.abs(mlmc.dos_from_idos(x, x ** 3) - 3 * x * x).max() > 1e-4


def test_oracle_dos_of_pristine_graphene_matches_the_smoothed_density(glat):
    """The Gaussian-smoothed pristine IDoS has the analytic derivative
    sum_states phi((E - eps)/delta) / delta (per unit area); the numerical
    derivative on a grid of step h is within the O(h^2) error term of it."""
    N, K, delta = 2, 2, 0.4
    eps = energy_grid(-9.0, 9.0, 361)
    I = oracle.level_estimate(glat, N, False, 0.0, K, K, KGRID_GAMMA, 1, 0, 1, eps, delta, SMOOTH_GAUSS)[0]
    E = []
    for kap in oracle.kgrid(KGRID_GAMMA, K)[0]:
        E.append(oracle.eigvalsh(oracle.build_hamiltonian(glat, N, np.zeros((N, N, 2), np.uint8), kap)))
    E = np.concatenate(E)
    norm = K * K * N * N * glat.cell_area
    exact = np.array([np.sum(np.exp(-0.5 * ((E - e) / delta) ** 2)) for e in eps]) / (
        delta * math.sqrt(2 * math.pi) * norm)
    h = eps[1] - eps[0]
    # |f'''| of one smoothed state <= 1 / (delta^3 sqrt(2 pi)) * 2; error <= h^2/6 |f'''| (interior), h^2/3 (ends)
    bound = (h * h / 3.0) * 2.0 / (delta ** 3 * math.sqrt(2 * math.pi)) * E.size / norm
    assert np.abs(mlmc.dos_from_idos(eps, I) - exact).max() <= bound
    # the trapezoid integral of the density recovers the IDoS increase
    D = mlmc.dos_from_idos(eps, I)
    assert abs(np.trapezoid(D, eps) - (I[-1] - I[0])) < 1e-3 * I[-1]


def test_c_abi_dos_matches_oracle():
    from paper_1611_09784_amd import binding as B
    x = nonuniform_grid(57, 2)
    f = np.sin(x) + 0.1 * x ** 3
    assert np.abs(B.mlmc_dos(x, f) - mlmc.dos_from_idos(x, f)).max() < 1e-11
    import ctypes as C
    lib = B.lib()
    a = np.zeros(3)
    assert lib.mlmc_dos(2, a.ctypes.data_as(C.c_void_p), a.ctypes.data_as(C.c_void_p),
                        a.ctypes.data_as(C.c_void_p)) == B.MLMC_ERR_INVALID_ARG
    with pytest.raises(B.MLMCError):
        B.mlmc_dos(np.array([0.0, 1.0, 1.0]), np.zeros(3))   # not increasing
