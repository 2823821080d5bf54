"""Host-side MC / MLMC driver over the C ABI (Section 2 of the paper).

All per-sample work runs in ``libmlmc.so`` through ``mlmc_level_estimate``;
this module only keeps the per-level sums (copied back once per level call),
turns them into sample means and variances, asks ``mlmc_optimal_samples``
for the allocation of eq. (opt_samples) and applies the stopping rule
C_alpha * sqrt(sum_l V_l / M_l) <= theta * TOL_abs.

Readings of the paper used here:
  * V_l is the largest sample variance over the energy grid (the
    conservative choice for the "discrete norms" of Section 4.4);
  * TOL_abs = TOL * max_eps |estimate| for a relative tolerance;
  * the levels are fixed in advance, so only the statistical constraint is
    enforced (the bias constraint of Section 2.2 fixes L, which is an input).
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B


@dataclass
class LevelState:
    N: int
    K: int
    coupled: bool
    K_coarse: int
    M: int = 0
    seconds: float = 0.0
    stats: np.ndarray = None  # [4][n_eps]: sum Y, sum Y^2, sum Q_f, sum Q_f^2

    def mean_var(self):
        s1, s2 = self.stats[0], self.stats[1]
        mean = s1 / self.M
        var = (s2 - self.M * mean * mean) / (self.M - 1) if self.M > 1 else np.zeros_like(mean)
        return mean, np.maximum(var, 0.0)


@dataclass
class MLMCResult:
    estimate: np.ndarray
    levels: list
    error: float
    tol_abs: float
    seconds: float
    rounds: list = field(default_factory=list)


class Estimator:
    """Runs level calls on one device with a reusable workspace."""

    def __init__(self, dlat: B.DeviceLattice, eps: np.ndarray, delta: float, p: float, kind: int, seed: int,
                 smoother: int = B.MLMC_SMOOTH_GAUSS, prec: int = B.MLMC_PREC_FP64, chunk_samples: int = 64,
                 stream=None):
        self.dlat = dlat
        self.eps = torch.as_tensor(np.asarray(eps, dtype=np.float64), device=dlat.device)
        self.delta, self.p, self.kind, self.seed = float(delta), float(p), int(kind), int(seed)
        self.smoother, self.prec, self.chunk = int(smoother), int(prec), int(chunk_samples)
        self.stream = stream
        self._work = {}

    def _workspace(self, lvl: LevelState):
        key = (lvl.N, lvl.coupled, lvl.K, lvl.K_coarse)
        if key not in self._work:
            need = B.mlmc_level_workspace(self.dlat, lvl.N, lvl.coupled, lvl.K, lvl.K_coarse, self.kind, self.chunk,
                                          self.prec, self.eps.shape[0])
            self._work[key] = torch.empty((need,), dtype=torch.uint8, device=self.dlat.device)
        return self._work[key]

    def add_samples(self, lvl: LevelState, count: int):
        if count <= 0:
            return
        stats = torch.zeros((4, self.eps.shape[0]), dtype=torch.float64, device=self.dlat.device)
        torch.cuda.synchronize(self.dlat.device)
        t0 = time.perf_counter()
        B.mlmc_level_estimate(self.dlat, lvl.N, lvl.coupled, self.p, lvl.K, lvl.K_coarse, self.kind, self.seed,
                              lvl.M, count, self.eps, self.delta, self.smoother, self.prec, stats=stats,
                              work=self._workspace(lvl), stream=self.stream)
        host = stats.cpu().numpy()
        lvl.seconds += time.perf_counter() - t0
        lvl.stats = host if lvl.stats is None else lvl.stats + host
        lvl.M += count


def make_levels(levels, Ks):
    """Level 1: plain Q on the coarsest supercell; level l >= 2: Y = Q_l - Q_l^CV
    with the quarters solved on level l-1's grid."""
    out = []
    for l, (N, K) in enumerate(zip(levels, Ks)):
        out.append(LevelState(N=N, K=K, coupled=l > 0, K_coarse=Ks[l - 1] if l > 0 else K))
    return out


def run_mlmc(est: Estimator, levels, Ks, tol_rel: float, C_alpha: float = 2.0, theta: float = 0.5, pilot: int = 16,
             max_rounds: int = 10, max_samples: int = 1_000_000) -> MLMCResult:
    """Adaptive-sample MLMC over fixed levels (eq. (MLMC), eq. (opt_samples))."""
    lv = make_levels(levels, Ks)
    t0 = time.perf_counter()
    target = [pilot] * len(lv)
    rounds = []
    err = tol_abs = float("inf")
    estimate = None
    for _ in range(max_rounds):
        for l, st in enumerate(lv):
            est.add_samples(st, min(target[l], max_samples) - st.M)
        means, V = [], []
        for st in lv:
            m, v = st.mean_var()
            means.append(m)
            V.append(max(float(v.max()), 1e-300))
        W = [st.seconds / st.M for st in lv]
        estimate = np.sum(means, axis=0)
        tol_abs = tol_rel * float(np.max(np.abs(estimate)))
        M = [st.M for st in lv]
        err = C_alpha * math.sqrt(sum(v / m for v, m in zip(V, M)))
        rounds.append({"M": M, "V": V, "W": W, "error": err, "tol_abs": tol_abs})
        if err <= theta * tol_abs:
            break
        Mopt = B.mlmc_optimal_samples(V, W, C_alpha, theta, tol_abs)
        target = [max(st.M, int(math.ceil(m))) for st, m in zip(lv, Mopt)]
        if all(st.M >= max_samples for st in lv):
            break
    return MLMCResult(estimate=estimate, levels=lv, error=err, tol_abs=tol_abs, seconds=time.perf_counter() - t0,
                      rounds=rounds)


def run_mc(est: Estimator, N: int, K: int, M: int) -> LevelState:
    """Plain MC (eq. (MC)) with M samples on one supercell size."""
    lvl = LevelState(N=N, K=K, coupled=False, K_coarse=K)
    est.add_samples(lvl, M)
    return lvl
