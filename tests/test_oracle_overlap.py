"""Pins for the non-orthogonal graphene model of Section 3.1 (overlap matrix
S, generalised eigenproblem H c = E S c) in the oracle."""

import numpy as np
import pytest
import scipy.linalg

import oracle
from mlmc_inputs import energy_grid, graphene_overlap
from mlmc_inputs.configs import KGRID_GAMMA, SMOOTH_GAUSS

T, SOV = -3.033, 0.129


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("eps2p", [0.0, 0.4])
def test_pristine_bands_closed_form(N, eps2p):
    """The 2x2 primitive pencil gives (eps_2p - E)^2 = |f|^2 (t - E s)^2, so
    E = (eps_2p -+ t|f|) / (1 -+ s|f|) with f = 1 + e^{i k.a1} + e^{i k.a2};
    the pristine N x N supercell at reduced kappa holds these bands at
    k = (kappa + (m, q)) / N (band folding)."""
    lat = graphene_overlap(eps_2p=eps2p)
    mask = np.zeros((N, N, 2), np.uint8)
    for kap in ((0.13, 0.37), (0.0, 0.0), (0.5, 0.25)):
        H = oracle.build_hamiltonian(lat, N, mask, kap)
        S = oracle.build_overlap(lat, N, mask, kap)
        got = oracle.eigvalsh_generalized(H, S)
        want = []
        for m in range(N):
            for q in range(N):
                k1, k2 = (kap[0] + m) / N, (kap[1] + q) / N
                f = abs(1 + np.exp(2j * np.pi * k1) + np.exp(2j * np.pi * k2))
                want += [(eps2p - T * f) / (1 - SOV * f), (eps2p + T * f) / (1 + SOV * f)]
        assert np.abs(got - np.sort(want)).max() < 1e-12


def test_vacancy_spectrum_maps_from_the_bond_matrix():
    """With eps_2p = 0, H = t A and S = I + s A for the Bloch bond matrix A of
    the present sites (vacancies delete rows and columns of both), so every
    generalised eigenvalue is t a / (1 + s a) for an eigenvalue a of A."""
    lat = graphene_overlap()
    N = 4
    masks = oracle.sample_vacancies(lat, N, 0.2, 5, oracle.stream_tag(lat, N), 0, 3)
    for m in masks:
        for kap in ((0.21, 0.64), (0.0, 0.5)):
            H = oracle.build_hamiltonian(lat, N, m, kap)
            S = oracle.build_overlap(lat, N, m, kap)
            a = oracle.eigvalsh(H / T)
            want = np.sort(T * a / (1 + SOV * a))
            assert np.abs(oracle.eigvalsh_generalized(H, S) - want).max() < 1e-12
            assert np.abs(S - (np.eye(S.shape[0]) + SOV * H / T)).max() < 1e-15


def test_against_lapack_generalized_solver():
    lat = graphene_overlap(eps_2p=0.25)
    N = 3
    masks = oracle.sample_vacancies(lat, N, 0.3, 8, oracle.stream_tag(lat, N), 0, 4)
    for m in masks:
        H = oracle.build_hamiltonian(lat, N, m, (0.3, 0.1))
        S = oracle.build_overlap(lat, N, m, (0.3, 0.1))
        want = scipy.linalg.eigh(H, S, eigvals_only=True)
        assert np.abs(oracle.eigvalsh_generalized(H, S) - want).max() < 1e-12
        L = oracle.cholesky(S)
        assert np.abs(L @ L.conj().T - S).max() < 1e-14
        assert np.abs(L - np.linalg.cholesky(S)).max() < 1e-14
        assert np.linalg.eigvalsh(S).min() > 0.5        # |s f| <= 3 s < 0.39


def test_overlap_idos_counts_states():
    lat = graphene_overlap()
    N = 3
    eps = energy_grid(-9.0, 18.0, 41)   # bands span about [-6.6, 14.9] eV
    mask = oracle.sample_vacancies(lat, N, 0.2, 2, oracle.stream_tag(lat, N), 0, 1)[0]
    n = 2 * N * N - int(mask.sum())
    Q = oracle.sample_qoi(lat, N, mask, False, 2, 2, KGRID_GAMMA, eps, 0.05, SMOOTH_GAUSS)
    assert abs(Q[-1] - n / (N * N * lat.cell_area)) < 1e-12
    assert abs(Q[0]) < 1e-12
