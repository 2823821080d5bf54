"""Pins for S-pair vacancies (Section 3.2: the two S atoms of a cell are
removed together) on the MoS2-shaped lattice."""

import numpy as np

import oracle
from oracle import mlmc
from mlmc_inputs import energy_grid
from mlmc_inputs.configs import KGRID_GAMMA, SMOOTH_GAUSS


def test_pairs_remove_six_orbitals(plat, mlat):
    N = 4
    masks = oracle.sample_vacancies(plat, N, 0.3, 9, oracle.stream_tag(plat, N), 0, 20)
    assert masks.shape == (20, N, N, 2)
    assert (masks[..., 0] == 0).all()            # Mo never vacant
    for m in masks:
        H = oracle.build_hamiltonian(plat, N, m, (0.1, 0.2))
        assert H.shape[0] == 11 * N * N - 6 * int(m[..., 1].sum())
    # an S-pair vacancy equals both single-S vacancies of the same cell in the site model
    m = masks[3]
    single = np.zeros((N, N, 3), np.uint8)
    single[..., 1] = m[..., 1]
    single[..., 2] = m[..., 1]
    for kap in ((0.0, 0.0), (0.3, 0.7)):
        a = oracle.eigvalsh(oracle.build_hamiltonian(plat, N, m, kap))
        b = oracle.eigvalsh(oracle.build_hamiltonian(mlat, N, single, kap))
        assert np.abs(a - b).max() < 1e-12


def test_pair_streams_are_independent_of_site_streams(plat, mlat):
    N = 4
    assert oracle.stream_tag(plat, N) != oracle.stream_tag(mlat, N)


def test_mc_mean_matches_exhaustive_enumeration_pairs(plat):
    """N = 2 with S pairs: 4 removable groups, 16 outcomes; the MC mean falls in
    its CLT band around the exact expectation."""
    N, K, p = 2, 1, 0.3
    b = plat.hop_magnitude_bound() + 1.0
    eps = energy_grid(-b, b, 41)
    delta = 0.5
    exact = mlmc.exhaustive_expectation(plat, N, p, K, KGRID_GAMMA, eps, delta, SMOOTH_GAUSS)
    M = 400
    stats = oracle.level_estimate(plat, N, False, p, K, K, KGRID_GAMMA, 13, 0, M, eps, delta, SMOOTH_GAUSS,
                                  n_threads=4)
    mean, var = mlmc.mean_and_var(stats, M)
    assert np.all(np.abs(mean - exact) <= 4.5 * np.sqrt(var / M) + 1e-15)
