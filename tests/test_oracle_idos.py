"""Pins for the oracle's smoothed integrated density of states (eq. (IDoS)
with the nearest-point approximation and the smoothing of
eq. (MLMC_smoothing), Section 4.3)."""

import math

import numpy as np
import pytest

import oracle
from mlmc_inputs import energy_grid
from mlmc_inputs.configs import KGRID_GAMMA, KGRID_MP, SMOOTH_CUBIC, SMOOTH_GAUSS


def supercell_idos(lat, N, mask, kind, K, eps, delta, smoother):
    kred, kw = oracle.kgrid(kind, K)
    nmax = lat.n_orb * N * N
    W = np.zeros((K * K, max(nmax, 1)))
    n = np.zeros(K * K, np.int32)
    for i, kap in enumerate(kred):
        w = oracle.eigvalsh(oracle.build_hamiltonian(lat, N, mask, kap))
        W[i, : w.size] = w
        n[i] = w.size
    return oracle.idos(W, n, kw, N * N * lat.cell_area, eps, delta, smoother), W, n, kw


@pytest.mark.parametrize("N,K,kind", [(1, 8, KGRID_MP), (2, 4, KGRID_MP), (4, 2, KGRID_GAMMA), (3, 3, KGRID_MP)])
def test_pristine_idos_equals_closed_form_primitive(glat, N, K, kind):
    """A pristine N x N supercell on a K x K grid has exactly the states of the
    primitive cell on the folded N K x N K grid (band folding), so its IDoS
    per unit area equals the closed-form primitive IDoS on that grid."""
    eps = energy_grid(-9.0, 9.0, 73)
    delta = 0.3
    got, _, _, _ = supercell_idos(glat, N, np.zeros((N, N, 2), np.uint8), kind, K, eps, delta, SMOOTH_GAUSS)
    t = 2.7
    energies = []
    for r1 in range(K):
        for r2 in range(K):
            if kind == KGRID_MP:
                kap = ((2 * r1 - K + 1) / (2 * K), (2 * r2 - K + 1) / (2 * K))
            else:
                kap = (r1 / K, r2 / K)
            for m in range(N):
                for q in range(N):
                    k1, k2 = (kap[0] + m) / N, (kap[1] + q) / N
                    f = abs(1 + np.exp(2j * np.pi * k1) + np.exp(2j * np.pi * k2))
                    energies += [t * f, -t * f]
    energies = np.array(energies)
    npts = (N * K) ** 2
    want = np.array([sum(0.5 * math.erfc((E - e) / (delta * math.sqrt(2))) for E in energies)
                     for e in eps]) / (npts * glat.cell_area)
    assert np.abs(got - want).max() < 1e-13


def test_idos_limits_and_symmetry(glat):
    N, K = 4, 2
    mask = oracle.sample_vacancies(glat, N, 0.2, 3, oracle.stream_tag(glat, N), 0, 1)[0]
    eps = energy_grid(-9.0, 9.0, 201)
    delta = 0.1
    I, W, n, kw = supercell_idos(glat, N, mask, KGRID_MP, K, eps, delta, SMOOTH_GAUSS)
    total = float((kw * n).sum()) / (N * N * glat.cell_area)
    assert abs(I[-1] - total) < 1e-15            # every state lies below 9 eV - 9 delta
    assert abs(I[0]) < 1e-15
    assert np.all(np.diff(I) >= -1e-16)          # Gaussian-smoothed count is monotone
    # bipartite +- symmetry of the spectrum and symmetric grid
    assert np.abs(I + I[::-1] - total).max() < 1e-14
    assert abs(I[100] - 0.5 * total) < 1e-14


def test_idos_sharp_limit_counts_states(glat):
    """With tiny delta the smoothed IDoS is the plain count of states below eps
    (strict inequality of the indicator in eq. (IDoS)), away from eigenvalues."""
    N, K = 3, 2
    mask = oracle.sample_vacancies(glat, N, 0.3, 4, oracle.stream_tag(glat, N), 0, 1)[0]
    eps = np.array([-7.3, -2.05, -0.61, 0.37, 1.91, 6.4])
    for smoother in (SMOOTH_GAUSS, SMOOTH_CUBIC):
        I, W, n, kw = supercell_idos(glat, N, mask, KGRID_MP, K, eps, 1e-9, smoother)
        counts = np.array([sum(kw[k] * np.sum(W[k, : n[k]] < e) for k in range(K * K)) for e in eps])
        assert np.abs(I - counts / (N * N * glat.cell_area)).max() < 1e-15


def test_smoothers_shape_and_moments():
    for s in (SMOOTH_GAUSS, SMOOTH_CUBIC):
        assert oracle.smooth_step(s, 0.0) == 0.5
        for x in (0.1, 0.4, 0.9, 2.0):
            assert abs(oracle.smooth_step(s, x) + oracle.smooth_step(s, -x) - 1.0) < 1e-15
        assert oracle.smooth_step(s, -12.0) == 1.0
        assert oracle.smooth_step(s, 12.0) < 1e-30
    # cubic: exact endpoint values, and the q = 0, 1 moment conditions of eq. (MLMC_smoothing)
    assert oracle.smooth_step(SMOOTH_CUBIC, -1.0) == 1.0
    assert oracle.smooth_step(SMOOTH_CUBIC, 1.0) == 0.0
    xs, wq = np.polynomial.legendre.leggauss(20)
    for q in (0, 1):
        # integrate x^q (chi(x<0) - g(x)) over [-1, 0] and [0, 1] separately (Gauss-Legendre is exact)
        left = sum(wi * (0.5 * (xi - 1)) ** q * (1.0 - oracle.smooth_step(SMOOTH_CUBIC, 0.5 * (xi - 1)))
                   for xi, wi in zip(xs, wq)) * 0.5
        right = sum(wi * (0.5 * (xi + 1)) ** q * (0.0 - oracle.smooth_step(SMOOTH_CUBIC, 0.5 * (xi + 1)))
                    for xi, wi in zip(xs, wq)) * 0.5
        assert abs(left + right) < 1e-15
    # the Gaussian CDF: derivative at 0 is -1/sqrt(2 pi)
    h = 1e-6
    slope = (oracle.smooth_step(SMOOTH_GAUSS, h) - oracle.smooth_step(SMOOTH_GAUSS, -h)) / (2 * h)
    assert abs(slope + 1 / math.sqrt(2 * math.pi)) < 1e-8
