"""Monte Carlo / multilevel Monte Carlo estimators on top of the C oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Section 2 of the paper:
  * eq. (MC): the sample mean of iid outcomes;
  * eq. (MLMC): mean of Q_1 plus the means of the coupled differences
    Q_l - Q_l^CV, each level with its own independent outcomes;
  * the estimator variance sum_l Var_l / M_l (Section 2.2);
  * eq. (opt_samples): M_l = (C_alpha / (theta TOL))^2 sqrt(V_l / W_l) sum_k sqrt(W_k V_k);
  * the complexity exponents of eq. (Work_FS), (Work_SLMC) and (Work_MLMC).
"""

from __future__ import annotations

import itertools
import math
import time

import numpy as np

from . import level_estimate, sample_qoi


def mean_and_var(stats: np.ndarray, M: int, row_sum: int = 0, row_sq: int = 1):
    """Sample mean and unbiased sample variance per energy from running sums."""
    s1 = stats[row_sum]
    s2 = stats[row_sq]
    mean = s1 / M
    var = (s2 - M * mean * mean) / (M - 1) if M > 1 else np.zeros_like(mean)
    return mean, np.maximum(var, 0.0)


def optimal_samples(V, W, C_alpha: float, theta: float, tol: float) -> np.ndarray:
    """Real-valued sample counts of eq. (opt_samples)."""
    V = np.asarray(V, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    total = float(np.sum(np.sqrt(W * V)))
    return (C_alpha / (theta * tol)) ** 2 * np.sqrt(V / W) * total


def statistical_error(V, M, C_alpha: float) -> float:
    """C_alpha times the standard deviation of the MLMC estimator, sqrt(sum_l
    V_l / M_l), for independent levels with variances V_l and M_l samples
    (Section 2.2)."""
    V = np.asarray(V, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    return C_alpha * math.sqrt(float(np.sum(V / M)))


def complexity_exponents(W: float, S: float, D: float, C: float):
    """(AC_FS, AC_MC, AC_MLMC) with Work ~ TOL^-AC (eqs. Work_FS, Work_SLMC, Work_MLMC)."""
    return 2.0 * C / S, 2.0 + (C - S) / W, 2.0 + (C - D) / W


def mc_splitting(W: float, S: float, C: float) -> float:
    """Optimal bias/statistical split Theta = 1 / (1 + (C - S)/W) of Section 2.1."""
    return 1.0 / (1.0 + (C - S) / W)


def exhaustive_expectation(lat, N, p, K, kind, eps, delta, smoother):
    """E[Q_N] over every vacancy outcome of an N x N supercell, each weighted by
    p^v (1-p)^(r-v) (the exhaustive approach of Sections 1 and 4.4).  Only
    practical for tiny supercells."""
    G = lat.n_groups
    removable = [bool(lat.group_removable[g % G]) for g in range(N * N * G)]
    slots = [g for g in range(N * N * G) if removable[g]]
    r = len(slots)
    acc = np.zeros(len(eps))
    for bits in itertools.product((0, 1), repeat=r):
        mask = np.zeros(N * N * G, dtype=np.uint8)
        for b, g in zip(bits, slots):
            mask[g] = b
        v = sum(bits)
        weight = (p ** v) * ((1.0 - p) ** (r - v))
        if weight == 0.0:
            continue
        q = sample_qoi(lat, N, mask.reshape(N, N, G), False, K, K, kind, eps, delta, smoother)
        acc += weight * q
    return acc


def dos_from_idos(eps, idos):
    """Density of states as the derivative of the IDoS on the energy grid
    (Section 4.3, numerical differentiation): second-order differences,
    centred inside and one-sided at the ends (numpy.gradient, edge_order 2)."""
    return np.gradient(np.asarray(idos, dtype=np.float64), np.asarray(eps, dtype=np.float64), edge_order=2)


def run_mlmc(lat, levels, Ks, p, kind, seed, eps, delta, smoother, tol_rel, C_alpha=2.0, theta=0.5,
             pilot=16, max_rounds=8, n_threads=1, max_samples=None, level_fn=None, cost_fn=None):
    """Adaptive-sample MLMC driver over fixed levels (eq. (MLMC) + eq. (opt_samples)).

    Level 1 is the plain IDoS on the coarsest supercell; level l >= 2 couples
    the N_l supercell with the mean of its four quarters on the N_{l-1} grid.
    Each round adds samples up to the target counts, forms the sample means
    and variances (V_l = largest variance over the energies), the estimate
    (sum of the level means) and the statistical error C_alpha sqrt(sum V_l /
    M_l); it stops once that error is at most theta * TOL_abs (TOL_abs = tol_rel
    * max |estimate|), otherwise it allocates the next targets by eq.
    (opt_samples) with the measured cost per sample W_l.

    level_fn(l, first, count) -> [4][n_eps] sums replaces the oracle's own
    level estimate (the default draws and solves the outcomes); cost_fn(l)
    -> seconds per sample replaces the measured time.  Returns a dict with the
    estimate, per-level sums, sample counts and the final statistical error."""
    L = len(levels)
    ne = len(eps)
    stats = [np.zeros((4, ne)) for _ in range(L)]
    M = [0] * L
    secs = [0.0] * L
    target = [pilot] * L
    history = []
    for rnd in range(max_rounds):
        for l in range(L):
            add = target[l] - M[l]
            if max_samples is not None:
                add = min(add, max_samples - M[l])
            if add <= 0:
                continue
            t0 = time.perf_counter()
            if level_fn is not None:
                st = level_fn(l, M[l], add)
            else:
                coupled = l > 0
                st = level_estimate(lat, levels[l], coupled, p, Ks[l], Ks[l - 1] if coupled else Ks[l], kind,
                                    seed, M[l], add, eps, delta, smoother, n_threads=n_threads)
            secs[l] += time.perf_counter() - t0
            stats[l] += st
            M[l] += add
        V = []
        means = []
        for l in range(L):
            mean, var = mean_and_var(stats[l], M[l])
            means.append(mean)
            V.append(max(float(var.max()), 1e-300))
        W = [cost_fn(l) if cost_fn is not None else secs[l] / M[l] for l in range(L)]
        estimate = np.sum(means, axis=0)
        tol_abs = tol_rel * float(np.max(np.abs(estimate)))
        err = statistical_error(V, M, C_alpha)
        history.append({"M": list(M), "V": list(V), "W": list(W), "error": err, "tol_abs": tol_abs})
        if err <= theta * tol_abs:
            break
        Mopt = optimal_samples(V, W, C_alpha, theta, tol_abs)
        target = [max(M[l], int(math.ceil(Mopt[l]))) for l in range(L)]
        if max_samples is not None and all(M[l] >= max_samples for l in range(L)):
            break
    return {"estimate": estimate, "stats": stats, "M": M, "seconds": secs, "error": err,
            "tol_abs": tol_abs, "history": history}
