"""Spectral invariants of the bipartite graphene model with vacancies.

Removing sites keeps the nearest-neighbour model bipartite, so the spectrum
stays symmetric under E -> -E, the sublattice imbalance |n_A - n_B| forces at
least that many zero modes, and (Cauchy) the spectrum of the principal
submatrix interlaces the pristine spectrum.
"""

import numpy as np
import pytest

import oracle
from test_oracle_assembly import folded_graphene_bands


@pytest.mark.parametrize("N,seed,p", [(2, 1, 0.3), (3, 2, 0.2), (4, 3, 0.15), (5, 4, 0.1)])
def test_pm_symmetry_and_zero_modes(glat, N, seed, p):
    mask = oracle.sample_vacancies(glat, N, p, seed, oracle.stream_tag(glat, N), 0, 1)[0]
    kappa = (0.3, 0.45)
    w = oracle.eigvalsh(oracle.build_hamiltonian(glat, N, mask, kappa))
    assert np.abs(w + w[::-1]).max() < 1e-12
    nA = int((mask[..., 0] == 0).sum())
    nB = int((mask[..., 1] == 0).sum())
    zero = int((np.abs(w) < 1e-9).sum())
    assert zero >= abs(nA - nB)


@pytest.mark.parametrize("N,seed", [(3, 9), (4, 10)])
def test_cauchy_interlacing(glat, N, seed):
    mask = oracle.sample_vacancies(glat, N, 0.2, seed, oracle.stream_tag(glat, N), 0, 1)[0]
    kappa = (0.11, 0.52)
    w = oracle.eigvalsh(oracle.build_hamiltonian(glat, N, mask, kappa))
    full = folded_graphene_bands(N, kappa)
    r = full.size - w.size
    for i in range(w.size):
        assert full[i] - 1e-12 <= w[i] <= full[i + r] + 1e-12
