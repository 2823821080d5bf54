"""Pins for the oracle's three-rhombus k-lattice (Section 4.2): the hexagonal
zone of the supercell as three rhombi with the common corner Gamma, each cut
into K x K rhombi whose corners are the k-points, duplicates kept once."""

import itertools
import math

import numpy as np
import pytest

import oracle
from mlmc_inputs import energy_grid
from mlmc_inputs.configs import KGRID_RHOMBI, SMOOTH_GAUSS

# reciprocal vectors of a1 = (1, 0), a2 = (1/2, sqrt 3 / 2) in units of 2 pi / a
B1 = np.array([1.0, -1.0 / math.sqrt(3.0)])
B2 = np.array([0.0, 2.0 / math.sqrt(3.0)])


def torus_dist(k1, k2):
    """Smallest Cartesian distance between reduced points k1, k2 over the
    reciprocal lattice translates."""
    best = np.inf
    for g1, g2 in itertools.product((-1, 0, 1), repeat=2):
        d = (k1[0] - k2[0] + g1) * B1 + (k1[1] - k2[1] + g2) * B2
        best = min(best, float(np.hypot(*d)))
    return best


@pytest.mark.parametrize("K", [1, 2, 3, 5])
def test_count_weights_and_gamma(K):
    kred, kw = oracle.kgrid(KGRID_RHOMBI, K)
    assert kred.shape == (3 * K * K, 2)
    assert abs(kw.sum() - 1.0) < 1e-14 and np.allclose(kw, kw[0])
    assert (kred >= 0).all() and (kred < 1).all()
    keys = {(round(a * 3 * K), round(b * 3 * K)) for a, b in kred}
    assert len(keys) == 3 * K * K           # all distinct on the zone torus
    assert (0, 0) in keys                   # Gamma is a corner of every rhombus


@pytest.mark.parametrize("K", [1, 2, 4])
def test_points_form_the_hexagonal_lattice_of_the_corners(K):
    """Every point has exactly six nearest neighbours at distance |c|/K, where
    |c| = 2/3 (units 2 pi / a) is the distance from Gamma to a zone corner:
    the points are the corners of congruent 120-degree rhombi of side |c|/K."""
    kred, _ = oracle.kgrid(KGRID_RHOMBI, K)
    side = (2.0 / 3.0) / K
    for i in range(len(kred)):
        d = np.array([torus_dist(kred[i], kred[j]) for j in range(len(kred)) if j != i])
        assert abs(d.min() - side) < 1e-12
        assert np.sum(np.abs(d - side) < 1e-12) == (6 if len(kred) > 3 else 2)


@pytest.mark.parametrize("K", [2, 3])
def test_closed_form_set_and_inversion(K):
    """The kept corners are exactly the points (a, b)/(3K) with 3 | a + b, a set
    closed under k -> -k."""
    kred, _ = oracle.kgrid(KGRID_RHOMBI, K)
    got = {(round(a * 3 * K), round(b * 3 * K)) for a, b in kred}
    want = {(a, b) for a in range(3 * K) for b in range(3 * K) if (a + b) % 3 == 0}
    assert got == want
    assert {((-a) % (3 * K), (-b) % (3 * K)) for a, b in got} == got


def rhombi_idos(lat, N, mask, K, eps, delta):
    kred, kw = oracle.kgrid(KGRID_RHOMBI, K)
    nmax = lat.n_orb * N * N
    W = np.zeros((len(kred), max(nmax, 1)))
    n = np.zeros(len(kred), np.int32)
    for i, kap in enumerate(kred):
        w = oracle.eigvalsh(oracle.build_hamiltonian(lat, N, mask, kap))
        W[i, : w.size] = w
        n[i] = w.size
    return oracle.idos(W, n, kw, N * N * lat.cell_area, eps, delta, SMOOTH_GAUSS)


@pytest.mark.parametrize("N,K", [(1, 3), (2, 2)])
def test_pristine_idos_equals_closed_form_on_the_folded_lattice(glat, N, K):
    """A pristine N x N supercell on the rhombus lattice of side K holds the
    primitive-cell states at k = (kappa + (m, q)) / N, i.e. at the primitive
    points (P, Q) / (3 K N) with 3 | P + Q, where the graphene bands are
    +-|t| |1 + e^{2 pi i k1} + e^{2 pi i k2}|."""
    eps = energy_grid(-9.0, 9.0, 61)
    delta = 0.3
    got = rhombi_idos(glat, N, np.zeros((N, N, 2), np.uint8), K, eps, delta)
    M = 3 * K * N
    energies = []
    for P in range(M):
        for Q in range(M):
            if (P + Q) % 3:
                continue
            f = abs(1 + np.exp(2j * np.pi * P / M) + np.exp(2j * np.pi * Q / M))
            energies += [2.7 * f, -2.7 * f]
    energies = np.array(energies)
    want = np.array([np.sum(0.5 * np.array([math.erfc((E - e) / (delta * math.sqrt(2))) for E in energies]))
                     for e in eps]) / (len(energies) / 2 * glat.cell_area)
    assert np.abs(got - want).max() < 1e-13


@pytest.mark.parametrize("N,Kf", [(4, 1), (2, 2)])
def test_pristine_coupling_vanishes_on_rhombus_lattices(glat, N, Kf):
    """With N K fixed the fine and coarse rhombus lattices fold onto the same
    primitive points, so the control-variate difference vanishes for p = 0."""
    eps = energy_grid(-9.0, 9.0, 41)
    stats, Y, Qf = oracle.level_estimate(glat, N, True, 0.0, Kf, 2 * Kf, KGRID_RHOMBI, 1, 0, 2, eps, 0.2,
                                         SMOOTH_GAUSS, per_sample=True)
    assert np.abs(Y).max() < 1e-13
    assert Qf.max() > 0.0
