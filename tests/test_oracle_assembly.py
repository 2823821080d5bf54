"""Pins for the oracle's Bloch-Hamiltonian assembly and eigensolver on H(k).

Closed forms and invariants fixed by the model of Section 3.1 (graphene
nearest-neighbour pi bands) and by band folding of a periodic supercell.
"""

import numpy as np
import pytest

import oracle


def folded_graphene_bands(N, kappa, t=2.7):
    """Closed-form spectrum of the pristine N x N graphene supercell at
    reduced supercell wave vector kappa: the primitive bands
    +-|t| |1 + e^{i k.a1} + e^{i k.a2}| at k = (kappa + (m, q)) / N."""
    out = []
    for m in range(N):
        for q in range(N):
            k1 = (kappa[0] + m) / N
            k2 = (kappa[1] + q) / N
            f = abs(1 + np.exp(2j * np.pi * k1) + np.exp(2j * np.pi * k2))
            out += [t * f, -t * f]
    return np.sort(out)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("kappa", [(0.0, 0.0), (0.13, 0.37), (0.5, -0.25), (1.0 / 3, 2.0 / 3)])
def test_pristine_graphene_folding(glat, N, kappa):
    mask = np.zeros((N, N, 2), np.uint8)
    H = oracle.build_hamiltonian(glat, N, mask, kappa)
    assert H.shape == (2 * N * N, 2 * N * N)
    assert np.abs(H - H.conj().T).max() == 0.0
    w = oracle.eigvalsh(H)
    assert np.abs(w - folded_graphene_bands(N, kappa)).max() < 1e-13


def test_pristine_mos2_folding(mlat):
    """Spectrum of the pristine 2x2 supercell = union of primitive spectra at
    the four folded wave vectors (tests supercell indexing and phases)."""
    kappa = (0.21, -0.4)
    N = 2
    H = oracle.build_hamiltonian(mlat, N, np.zeros((N, N, 3), np.uint8), kappa)
    w = oracle.eigvalsh(H)
    prim = []
    for m in range(N):
        for q in range(N):
            Hp = oracle.build_hamiltonian(mlat, 1, np.zeros((1, 1, 3), np.uint8),
                                          ((kappa[0] + m) / N, (kappa[1] + q) / N))
            prim += list(np.linalg.eigvalsh(Hp))
    assert np.abs(np.sort(prim) - w).max() < 1e-12


def count_bonds(mask):
    """Present nearest-neighbour A-B bonds of an N x N graphene outcome
    (N >= 2: the three bonds of each A reach three distinct B sites)."""
    N = mask.shape[0]
    bonds = 0
    for i in range(N):
        for j in range(N):
            if mask[i, j, 0]:
                continue
            for (di, dj) in [(0, 0), (-1, 0), (0, -1)]:
                if not mask[(i + di) % N, (j + dj) % N, 1]:
                    bonds += 1
    return bonds


@pytest.mark.parametrize("N,seed", [(2, 1), (3, 2), (4, 3), (6, 4)])
def test_graphene_traces(glat, N, seed):
    mask = oracle.sample_vacancies(glat, N, 0.2, seed, oracle.stream_tag(glat, N), 0, 1)[0]
    H = oracle.build_hamiltonian(glat, N, mask, (0.3, 0.1))
    n_present = int((mask == 0).sum())
    assert H.shape[0] == n_present
    w = oracle.eigvalsh(H)
    assert abs(w.sum()) < 1e-12                     # Tr H = 0 (eps_2p = 0)
    assert abs((w ** 2).sum() - 2 * 2.7 ** 2 * count_bonds(mask)) < 1e-10   # Tr H^2


def test_eigen_sum_rules_mos2(mlat):
    N = 3
    mask = oracle.sample_vacancies(mlat, N, 0.3, 11, oracle.stream_tag(mlat, N), 0, 1)[0]
    H = oracle.build_hamiltonian(mlat, N, mask, (0.25, 0.6))
    assert H.shape[0] == 11 * N * N - 3 * int(mask.sum())
    assert np.abs(H - H.conj().T).max() < 1e-15
    w = oracle.eigvalsh(H)
    assert abs(w.sum() - np.trace(H).real) < 1e-11
    assert abs((w ** 2).sum() - (np.abs(H) ** 2).sum()) < 1e-10
    assert np.abs(w - np.linalg.eigvalsh(H)).max() < 1e-12


@pytest.mark.parametrize("lat_name", ["graphene", "mos2"])
def test_translation_invariance(glat, mlat, lat_name):
    lat = glat if lat_name == "graphene" else mlat
    N = 4
    mask = oracle.sample_vacancies(lat, N, 0.25, 5, oracle.stream_tag(lat, N), 0, 1)[0]
    kappa = (0.17, 0.71)
    w0 = oracle.eigvalsh(oracle.build_hamiltonian(lat, N, mask, kappa))
    shifted = np.roll(np.roll(mask, 1, axis=0), 3, axis=1)
    w1 = oracle.eigvalsh(oracle.build_hamiltonian(lat, N, shifted, kappa))
    assert np.abs(w0 - w1).max() < 1e-12


def test_all_vacant_and_hermitian_random(glat):
    N = 3
    mask = np.ones((N, N, 2), np.uint8)
    H = oracle.build_hamiltonian(glat, N, mask, (0.1, 0.2))
    assert H.shape == (0, 0)
