"""Pins for the oracle's control-variate construction and MC/MLMC estimators
(Sections 2 and 3.3)."""

import math
import os

import numpy as np
import pytest

import oracle
from oracle import mlmc
from mlmc_inputs import energy_grid
from mlmc_inputs.configs import KGRID_GAMMA, KGRID_MP, SMOOTH_GAUSS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_partition_tiles_the_supercell(glat):
    N = 6
    mask = oracle.sample_vacancies(glat, N, 0.4, 2, oracle.stream_tag(glat, N), 0, 1)[0]
    qs = oracle.partition_masks(mask)
    h = N // 2
    rebuilt = np.zeros_like(mask)
    for q in range(4):
        qi, qj = divmod(q, 2)
        rebuilt[qi * h:(qi + 1) * h, qj * h:(qj + 1) * h] = qs[q]
    assert (rebuilt == mask).all()


@pytest.mark.parametrize("lat_name,N,Kf", [("graphene", 4, 2), ("graphene", 8, 1), ("mos2", 4, 1)])
def test_pristine_coupling_vanishes(glat, mlat, lat_name, N, Kf):
    """Without vacancies every quarter is the pristine N/2 supercell, and on
    Gamma-centred grids with N K fixed the fine and coarse grids sample the
    same primitive k-points, so Y = Q_l - Q_l^CV vanishes identically."""
    lat = glat if lat_name == "graphene" else mlat
    eps = energy_grid(-9.0, 9.0, 61)
    stats, Y, Qf = oracle.level_estimate(lat, N, True, 0.0, Kf, 2 * Kf, KGRID_GAMMA, 1, 0, 2, eps, 0.2,
                                         SMOOTH_GAUSS, per_sample=True)
    assert np.abs(Y).max() < 1e-13
    assert Qf.max() > 0.0


def test_level_sums_are_additive_over_sample_ranges(glat):
    eps = energy_grid(-9.0, 9.0, 31)
    args = (glat, 4, True, 0.2, 2, 4, KGRID_GAMMA, 5)
    whole = oracle.level_estimate(*args, 0, 6, eps, 0.2, SMOOTH_GAUSS)
    parts = (oracle.level_estimate(*args, 0, 2, eps, 0.2, SMOOTH_GAUSS)
             + oracle.level_estimate(*args, 2, 4, eps, 0.2, SMOOTH_GAUSS))
    assert np.abs(whole - parts).max() < 1e-12
    threaded = oracle.level_estimate(*args, 0, 6, eps, 0.2, SMOOTH_GAUSS, n_threads=3)
    assert np.array_equal(whole, threaded)


def test_mc_mean_matches_exhaustive_enumeration(glat):
    """Exhaustive N = 2 expectation (all 2^8 outcomes with their probabilities,
    Sections 1 and 4.4) vs the MC estimator of eq. (MC) within its CLT band."""
    N, K, p = 2, 2, 0.3
    eps = energy_grid(-9.0, 9.0, 41)
    delta = 0.5
    exact = mlmc.exhaustive_expectation(glat, N, p, K, KGRID_MP, eps, delta, SMOOTH_GAUSS)
    M = 600
    stats = oracle.level_estimate(glat, N, False, p, K, K, KGRID_MP, 77, 0, M, eps, delta, SMOOTH_GAUSS,
                                  n_threads=4)
    mean, var = mlmc.mean_and_var(stats, M)
    band = 4.5 * np.sqrt(var / M) + 1e-15
    assert np.all(np.abs(mean - exact) <= band)
    # a wrong vacancy probability is detected by the same test
    assert not np.all(np.abs(mean - mlmc.exhaustive_expectation(glat, N, 0.2, K, KGRID_MP, eps, delta,
                                                                SMOOTH_GAUSS)) <= band)


def test_control_variate_is_unbiased(glat):
    """E[Q_l^CV] = E[Q_{l-1}] (eq. (CV_unbiased)): the mean of the four quarter
    IDoS of N = 4 outcomes matches the exhaustive N = 2 expectation."""
    p, Kc = 0.3, 2
    eps = energy_grid(-9.0, 9.0, 41)
    delta = 0.5
    exact = mlmc.exhaustive_expectation(glat, 2, p, Kc, KGRID_GAMMA, eps, delta, SMOOTH_GAUSS)
    M = 150
    stats, Y, Qf = oracle.level_estimate(glat, 4, True, p, 1, Kc, KGRID_GAMMA, 31, 0, M, eps, delta,
                                         SMOOTH_GAUSS, n_threads=4, per_sample=True)
    cv = Qf - Y
    mean = cv.mean(axis=0)
    sd = cv.std(axis=0, ddof=1)
    assert np.all(np.abs(mean - exact) <= 4.5 * sd / math.sqrt(M) + 1e-15)
    # the coupled difference has smaller variance than the fine quantity (D > S)
    assert Y.var(axis=0).max() < Qf.var(axis=0).max()


def test_optimal_samples_closed_form():
    V = np.array([4e-4, 1e-4, 2e-5, 3e-6])
    W = np.array([0.01, 0.05, 0.4, 3.0])
    Ca, theta, tol = 2.0, 0.5, 1e-3
    M = mlmc.optimal_samples(V, W, Ca, theta, tol)
    # the allocation meets the variance constraint with equality ...
    assert abs(Ca ** 2 * np.sum(V / M) - (theta * tol) ** 2) < 1e-12 * (theta * tol) ** 2
    # ... and is the constrained minimiser of total work: M_l ~ sqrt(V_l / W_l)
    r = M / np.sqrt(V / W)
    assert np.allclose(r, r[0], rtol=1e-14, atol=0)
    work = np.sum(M * W)
    rng = np.random.default_rng(0)
    for _ in range(200):
        Mp = M * np.exp(rng.normal(scale=0.3, size=4))
        Mp *= Ca ** 2 * np.sum(V / Mp) / (theta * tol) ** 2   # rescale onto the constraint
        assert np.sum(Mp * W) >= work * (1 - 1e-12)


def _frac(s):
    if "+" in s:
        a, b = s.split("+")
        n, d = b.split("/")
        return float(a) + float(n) / float(d)
    return float(s)


def test_complexity_exponents_golden():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "mos2_conv_table.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        W, S, D, C = map(float, r[1:5])
        fs, mc, ml = mlmc.complexity_exponents(W, S, D, C)
        assert abs(fs - _frac(r[5])) < 1e-12
        assert abs(mc - _frac(r[6])) < 1e-12
        assert abs(ml - _frac(r[7])) < 1e-12
    assert abs(mlmc.mc_splitting(1.5, 2, 4) - 3.0 / 7.0) < 1e-15


def test_mlmc_driver_reaches_tolerance_small(glat):
    """The oracle's own level estimates drive the estimator; it stops exactly
    when the statistical error first drops to theta * TOL_abs."""
    eps = energy_grid(-9.0, 9.0, 31)
    res = mlmc.run_mlmc(glat, [2, 4], [2, 1], 0.1, KGRID_GAMMA, 3, eps, 0.5, SMOOTH_GAUSS, tol_rel=2e-2,
                        pilot=8, max_rounds=6, n_threads=4)
    h = res["history"]
    assert h[-1]["error"] <= 0.5 * h[-1]["tol_abs"]
    assert all(r["error"] > 0.5 * r["tol_abs"] for r in h[:-1])
    # the estimator equals the sum of level means (eq. (MLMC))
    est = sum(st[0] / m for st, m in zip(res["stats"], res["M"]))
    assert np.abs(est - res["estimate"]).max() < 1e-15


# ---------------------------------------------------------------------------
# Statistical error and the adaptive driver against what the mathematics
# fixes: the spread of the estimator over independent replicas, and the
# optimality conditions of the constrained work minimisation behind
# eq. (opt_samples) (equal cost-weighted marginal variance reduction on every
# level, the variance constraint active).
# ---------------------------------------------------------------------------

def test_statistical_error_is_the_estimator_spread():
    """C_alpha sqrt(sum V_l / M_l) over C_alpha is the standard deviation of
    the sum of independent level means: measured over 6000 replicas of a
    two-level estimator with known level variances, and the C_alpha = 2 band
    covers the true mean with the normal probability 0.9545."""
    rng = np.random.default_rng(11)
    V, M, mu = np.array([4.0, 0.25]), np.array([40, 9]), np.array([1.5, -0.2])
    R = 6000
    est = (rng.normal(mu[0], math.sqrt(V[0]), size=(R, M[0])).mean(axis=1)
           + rng.normal(mu[1], math.sqrt(V[1]), size=(R, M[1])).mean(axis=1))
    sd = est.std(ddof=1)
    assert abs(mlmc.statistical_error(V, M, 1.0) / sd - 1.0) < 0.04     # sd of a sd estimate: 1/sqrt(2R) = 0.9 %
    band = mlmc.statistical_error(V, M, 2.0)
    cover = np.mean(np.abs(est - mu.sum()) <= band)
    assert 0.945 < cover < 0.965                                            # 0.9545 +- 3.5 binomial sd
    # closed form at hand-picked values: 2 sqrt(4/16 + 1/4) = sqrt 2
    assert abs(mlmc.statistical_error([4.0, 1.0], [16, 4], 2.0) - math.sqrt(2.0)) < 1e-15


def _synthetic_levels(mu, sigma, n_eps=3, seed=5):
    """Level samplers with known means and standard deviations: sample i of
    level l takes Y = mu_l + sigma_l z_i on energy 0 and half the deviation on
    the others (so V_l is the variance of energy 0); Q_f = Y."""
    def level_fn(l, first, count):
        z = np.random.default_rng([seed, l, first]).normal(size=count)
        scale = np.array([1.0] + [0.5] * (n_eps - 1))
        Y = mu[l] * (1.0 + np.arange(n_eps)) + sigma[l] * z[:, None] * scale[None, :]
        return np.stack([Y.sum(0), (Y * Y).sum(0), Y.sum(0), (Y * Y).sum(0)])
    return level_fn


def check_allocation_rounds(res, C_alpha, theta):
    """Every allocation after a round that has not met the tolerance is the
    minimiser of sum M_l W_l under C_alpha^2 sum V_l / M_l <= (theta TOL)^2:
    the constraint is active (up to rounding the counts up) and the
    Lagrange condition M_l^2 W_l / V_l = const holds on every level that was
    topped up; and the driver stops exactly at the first round whose error is
    within theta TOL_abs."""
    h = res["history"]
    assert h[-1]["error"] <= theta * h[-1]["tol_abs"]
    for r, nxt in zip(h[:-1], h[1:]):
        assert r["error"] > theta * r["tol_abs"]
        V, W, M0, M1 = map(np.asarray, (r["V"], r["W"], r["M"], nxt["M"]))
        grown = M1 > M0
        assert grown.any()
        lhs = C_alpha ** 2 * np.sum(V / M1)
        bound = (theta * r["tol_abs"]) ** 2
        assert lhs <= bound * (1 + 1e-12)
        # rounding up each count by < 1 sample loosens the constraint by < max(1/M)
        assert lhs >= bound * (1 - 1.0 / M1[grown].min()) - 1e-300
        lam = M1[grown] ** 2 * W[grown] / V[grown]
        assert lam.max() / lam.min() - 1.0 <= 2.5 / M1[grown].min()


@pytest.mark.parametrize("C_alpha,theta", [(2.0, 0.5), (3.0, 0.7)])
def test_run_mlmc_allocation_is_the_constrained_optimum(C_alpha, theta):
    mu, sigma, W = [2.0, 0.1, -0.05], [0.8, 0.3, 0.05], [1.0, 6.0, 40.0]
    eps = np.zeros(3)
    res = mlmc.run_mlmc(None, [4, 8, 16], [8, 4, 2], 0.0, 0, 0, eps, 0.1, 0, tol_rel=2e-3, C_alpha=C_alpha,
                        theta=theta, pilot=16, max_rounds=8, level_fn=_synthetic_levels(mu, sigma),
                        cost_fn=lambda l: W[l])
    assert len(res["history"]) >= 2
    check_allocation_rounds(res, C_alpha, theta)
    # the estimate is within the final error band of the true mean (energy 0)
    assert abs(res["estimate"][0] - sum(mu)) <= 1.5 * res["error"]


@pytest.mark.parametrize("mutation", ["no_square", "theta_once", "sqrt_dropped"])
def test_allocation_pin_catches_planted_mistakes(monkeypatch, mutation):
    """Plant a mistake in eq. (opt_samples) inside the oracle and check that
    the optimality pin above rejects the allocation it produces."""
    good = mlmc.optimal_samples

    def bad(V, W, C_alpha, theta, tol):
        V = np.asarray(V, dtype=np.float64)
        W = np.asarray(W, dtype=np.float64)
        total = float(np.sum(np.sqrt(W * V)))
        if mutation == "no_square":
            return (C_alpha / (theta * tol)) * np.sqrt(V / W) * total
        if mutation == "theta_once":
            return (C_alpha / tol) ** 2 / theta * np.sqrt(V / W) * total
        return (C_alpha / (theta * tol)) ** 2 * (V / W) * total

    monkeypatch.setattr(mlmc, "optimal_samples", bad)
    mu, sigma, W = [2.0, 0.1, -0.05], [0.8, 0.3, 0.05], [1.0, 6.0, 40.0]
    res = mlmc.run_mlmc(None, [4, 8, 16], [8, 4, 2], 0.0, 0, 0, np.zeros(3), 0.1, 0, tol_rel=2e-3,
                        pilot=16, max_rounds=3, level_fn=_synthetic_levels(mu, sigma), cost_fn=lambda l: W[l],
                        max_samples=10 ** 7)
    monkeypatch.setattr(mlmc, "optimal_samples", good)
    with pytest.raises(AssertionError):
        check_allocation_rounds(res, 2.0, 0.5)
