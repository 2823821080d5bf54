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
    """Runs level calls on one device with a reusable workspace and a
    pipeline context (the chase and back streams of the level calls): the
    caller's ``ctx``, which it keeps, or one of its own that ``close()``
    releases.  A process that runs several estimators one after another
    does best to give them one long-lived context: streams that come and go
    change which of the runtime's few hardware queues a new context's
    streams share, and streams on one queue run their work in order."""

    def __init__(self, dlat: B.DeviceLattice, eps: np.ndarray, delta: float, p: float, kind: int, seed: int,
                 smoother: int = B.MLMC_SMOOTH_GAUSS, prec: int = B.MLMC_PREC_FP64, chunk_samples: int = 64,
                 stream=None, dedup_max_orbitals: int = 0, tuner=None, graphs: bool = False,
                 budget_bytes: int = 48 << 30, ctx: B.Context = None):
        self.dlat = dlat
        self.eps = torch.as_tensor(np.asarray(eps, dtype=np.float64), device=dlat.device)
        self.delta, self.p, self.kind, self.seed = float(delta), float(p), int(kind), int(seed)
        self.smoother, self.prec, self.chunk = int(smoother), int(prec), int(chunk_samples)
        self.stream = stream
        self._own_ctx = ctx is None
        self.ctx = B.Context(dlat.device.index) if ctx is None else ctx
        self._work = {}
        # tuner: an autotune.Tuner; each level then takes its measured chunk
        # size and launch choices.  graphs: levels on the LDS-resident path
        # replay a captured level call (see LevelGraph).
        self.tuner = tuner
        self.graphs = bool(graphs)
        self.budget = int(budget_bytes)  # largest workspace of one level
        self._tuned = {}
        self._graph = {}
        # levels whose matrices have at most this many orbitals solve each
        # distinct outcome once (0: off)
        self.dedup_max_orbitals = int(dedup_max_orbitals)
        self.unique_solved = 0
        # per level: the distinct outcomes solved so far (key -> row of the
        # cached per-outcome IDoS), kept across rounds
        self._outcomes = {}

    def _tuning(self, lvl: LevelState):
        key = (lvl.N, lvl.coupled, lvl.K, lvl.K_coarse)
        if self.tuner is None:
            return None
        if key not in self._tuned:
            self._tuned[key] = self.tuner.tune_level(self.dlat, lvl.N, lvl.coupled, lvl.K, lvl.K_coarse, self.kind,
                                                     self.prec, self.eps, self.delta, self.p, ctx=self.ctx)
        return self._tuned[key]

    def _chunk(self, lvl: LevelState) -> int:
        """The tuned chunk, else the estimator's, halved until the level's
        workspace fits the budget."""
        t = self._tuning(lvl)
        c = self.chunk if t is None else t.chunk
        while c > 1 and B.mlmc_level_workspace(self.dlat, lvl.N, lvl.coupled, lvl.K, lvl.K_coarse, self.kind, c,
                                               self.prec, self.eps.shape[0]) > self.budget:
            c //= 2
        return c

    def _workspace(self, lvl: LevelState):
        key = (lvl.N, lvl.coupled, lvl.K, lvl.K_coarse)
        if key not in self._work:
            need = B.mlmc_level_workspace(self.dlat, lvl.N, lvl.coupled, lvl.K, lvl.K_coarse, self.kind,
                                          self._chunk(lvl), self.prec, self.eps.shape[0])
            self._work[key] = torch.empty((need,), dtype=torch.uint8, device=self.dlat.device)
        return self._work[key]

    def _use_graph(self, lvl: LevelState) -> bool:
        return self.graphs and self.dlat.max_orbitals(lvl.N) <= B.SMALL_MAX[self.prec] and \
            (not lvl.coupled or self.dlat.max_orbitals(lvl.N // 2) <= B.SMALL_MAX[self.prec])

    def add_samples(self, lvl: LevelState, count: int):
        if count <= 0:
            return
        stats = torch.zeros((4, self.eps.shape[0]), dtype=torch.float64, device=self.dlat.device)
        torch.cuda.synchronize(self.dlat.device)
        t0 = time.perf_counter()
        if self.dedup_max_orbitals and self.dlat.max_orbitals(lvl.N) <= self.dedup_max_orbitals:
            self._add_deduplicated(lvl, count, stats)
        else:
            done = 0
            if self._use_graph(lvl):
                g = self._level_graph(lvl)
                reps = count // g.M
                if reps:
                    g.run(lvl.M, reps, stats)
                    done = reps * g.M
            if count > done:
                t = self._tuning(lvl)
                if t is not None:
                    t.configure(self.ctx)
                else:
                    self.ctx.configure()  # the library's defaults (a shared context may hold other choices)
                B.mlmc_level_estimate(self.dlat, lvl.N, lvl.coupled, self.p, lvl.K, lvl.K_coarse, self.kind,
                                      self.seed, lvl.M + done, count - done, self.eps, self.delta, self.smoother,
                                      self.prec, stats=stats, work=self._workspace(lvl), ctx=self.ctx,
                                      stream=self.stream)
        host = stats.cpu().numpy()
        lvl.seconds += time.perf_counter() - t0
        lvl.stats = host if lvl.stats is None else lvl.stats + host
        lvl.M += count

    def _level_graph(self, lvl: LevelState):
        key = (lvl.N, lvl.coupled, lvl.K, lvl.K_coarse)
        if key not in self._graph:
            c = self._chunk(lvl)
            self._graph[key] = LevelGraph(self.dlat, lvl.N, lvl.coupled, self.p, lvl.K, lvl.K_coarse, self.kind,
                                          self.seed, 4 * c, self.eps, self.delta, self.smoother, self.prec, c)
        return self._graph[key]

    def forget_outcomes(self):
        """Drop the per-outcome results kept for duplicate reuse (after a
        warm-up, so that a run starts with none solved)."""
        self._outcomes.clear()
        self.unique_solved = 0

    def close(self):
        if self.ctx is not None and self._own_ctx:
            self.ctx.close()
        self.ctx = None
        self._work.clear()
        self._graph.clear()
        self._outcomes.clear()

    # -- explicit outcomes (steps a3-a7 through the C ABI) -------------------
    def outcome_idos(self, N: int, masks: torch.Tensor, K: int, budget_bytes: int = 1 << 30) -> torch.Tensor:
        """IDoS [ns][n_eps] of the given vacancy outcomes masks [ns][N][N][G]
        (device, uint8) on the K grid of the N x N supercell."""
        dev = self.dlat.device
        ns = masks.shape[0]
        kred, kw = B.mlmc_kgrid(self.kind, K, device=dev.index, stream=self.stream)
        nk = kred.shape[0]
        ld = self.dlat.max_orbitals(N)
        esize = 16 if self.prec == B.MLMC_PREC_FP64 else 8
        chunk = max(1, budget_bytes // max(1, nk * ld * ld * esize))
        out = torch.empty((ns, self.eps.shape[0]), dtype=torch.float64, device=dev)
        dtype = B.MLMC_C128 if self.prec == B.MLMC_PREC_FP64 else B.MLMC_C64
        area = N * N * self.dlat.lat.cell_area
        for a in range(0, ns, chunk):
            b = min(ns, a + chunk)
            H, n = B.mlmc_build_hamiltonians(self.dlat, N, masks[a:b].contiguous(), kred, dtype, stream=self.stream)
            w = B.mlmc_batched_eigvalsh(H, n, prec=self.prec, stream=self.stream)
            B.mlmc_idos(w, n, nk, kw, area, self.eps, self.delta, self.smoother, out=out[a:b], stream=self.stream)
            del H
        return out

    def _add_deduplicated(self, lvl: LevelState, count: int, stats: torch.Tensor):
        """Samples lvl.M .. lvl.M + count - 1 with each distinct outcome solved
        once (Section 4.4: identical outcomes are identified beforehand and not
        recomputed), also across calls: the per-outcome IDoS of every outcome
        solved on this level is kept, so a later round solves only outcomes not
        seen before.  Uncoupled levels identify outcomes up to a translation of
        the supercell (which leaves every H(k) spectrum unchanged); coupled
        levels identify equal outcomes only, since the quarters depend on the
        position of the vacancies."""
        N = lvl.N
        masks = B.mlmc_sample_vacancies(self.dlat, N, self.p, self.seed, self.dlat.tag(N), lvl.M, count,
                                        stream=self.stream)
        keys = outcome_keys(masks.cpu().numpy(), self.dlat.lat.group_removable, translations=not lvl.coupled)
        uniq, first, inverse = np.unique(keys, return_index=True, return_inverse=True)
        cache = self._outcomes.setdefault((N, lvl.coupled, lvl.K, lvl.K_coarse),
                                          {"index": {}, "Qf": None, "Qq": None})
        hkeys = [k.tobytes() if isinstance(k, np.void) else int(k) for k in uniq]
        rows = np.empty(len(hkeys), dtype=np.int64)
        new = []
        for i, h in enumerate(hkeys):
            r = cache["index"].get(h)
            if r is None:
                new.append(i)
            else:
                rows[i] = r
        if new:
            rep = masks[torch.as_tensor(first[new], device=masks.device)]
            Qf_new = self.outcome_idos(N, rep, lvl.K)
            base = 0 if cache["Qf"] is None else cache["Qf"].shape[0]
            cache["Qf"] = Qf_new if cache["Qf"] is None else torch.cat([cache["Qf"], Qf_new])
            if lvl.coupled:
                h = N // 2
                quarters = B.mlmc_partition_masks(self.dlat, N, rep, stream=self.stream)
                G = self.dlat.lat.n_groups
                Qq_new = self.outcome_idos(h, quarters.reshape(-1, h, h, G), lvl.K_coarse).reshape(len(new), 4, -1)
                cache["Qq"] = Qq_new if cache["Qq"] is None else torch.cat([cache["Qq"], Qq_new])
            for j, i in enumerate(new):
                cache["index"][hkeys[i]] = base + j
                rows[i] = base + j
        sel = torch.as_tensor(rows[inverse.reshape(-1)], device=masks.device)
        Qf = cache["Qf"][sel].contiguous()
        Qq = cache["Qq"][sel].contiguous() if lvl.coupled else None
        B.mlmc_level_stats(Qf, Qq, stats=stats, stream=self.stream)
        self.unique_solved += len(new)

    def exhaustive_expectation(self, N: int, K: int) -> np.ndarray:
        """E[Q_N] over every vacancy outcome of the N x N supercell, each with
        probability p^v (1-p)^(r-v) (Sections 1 and 4.4); outcomes equal up to
        a translation of the supercell are solved once and weighted by the
        size of their class."""
        lat = self.dlat.lat
        G = lat.n_groups
        slots = [g for g in range(N * N * G) if lat.group_removable[g % G]]
        r = len(slots)
        if r > 24:
            raise ValueError(f"exhaustive enumeration of 2^{r} outcomes is not supported")
        codes = np.arange(1 << r, dtype=np.int64)
        masks = np.zeros((codes.size, N * N * G), dtype=np.uint8)
        for i, g in enumerate(slots):
            masks[:, g] = (codes >> i) & 1
        masks = masks.reshape(-1, N, N, G)
        keys = outcome_keys(masks, lat.group_removable, translations=True)
        _, first, inverse = np.unique(keys, return_index=True, return_inverse=True)
        v = masks.reshape(codes.size, -1).sum(axis=1)
        prob = (self.p ** v) * ((1.0 - self.p) ** (r - v))
        weight = np.bincount(inverse.reshape(-1), weights=prob, minlength=first.size)
        rep = torch.as_tensor(masks[first], device=self.dlat.device)
        Q = self.outcome_idos(N, rep, K).cpu().numpy()
        self.unique_solved += int(first.size)
        return weight @ Q


class LevelGraph:
    """A level call of M samples captured once as a HIP graph (one stream, no
    pipeline context) and replayed: the first sample index lives in a device
    counter that the call reads when it draws outcomes and advances by M at
    its end, so every replay draws the next M samples.  Replays add their
    level sums into the graph's own sums, which run() adds to the caller's
    (on the device, after the replays)."""

    def __init__(self, dlat, N, coupled, p, K, Kc, kind, seed, M, eps, delta, smoother, prec, chunk):
        dev = dlat.device
        self.M = int(M)
        ne = eps.shape[0]
        self.stats = torch.zeros((4, ne), dtype=torch.float64, device=dev)
        self.counter = torch.zeros((1,), dtype=torch.int64, device=dev)
        need = B.mlmc_level_workspace(dlat, N, coupled, K, Kc, kind, chunk, prec, ne)
        self.work = torch.empty((need,), dtype=torch.uint8, device=dev)
        args = (dlat, N, coupled, p, K, Kc, kind, seed, 0, self.M, eps, delta, smoother, prec)
        # one eager call first: the kernels' first launches happen outside the capture
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            B.mlmc_level_estimate(*args, stats=self.stats, work=self.work, first_counter=self.counter)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize(dev)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            B.mlmc_level_estimate(*args, stats=self.stats, work=self.work, first_counter=self.counter)
        torch.cuda.synchronize(dev)

    def run(self, first: int, reps: int, stats: torch.Tensor):
        """Samples first .. first + reps M - 1 added into stats."""
        self.counter.fill_(int(first))
        self.stats.zero_()
        for _ in range(reps):
            self.graph.replay()
        stats += self.stats


def outcome_keys(masks: np.ndarray, removable: np.ndarray, translations: bool) -> np.ndarray:
    """One key per outcome ([n][N][N][G] uint8): equal keys for equal outcomes,
    or, with ``translations``, for outcomes equal up to a translation of the
    supercell (the smallest code over the N^2 cyclic shifts)."""
    n, N, _, G = masks.shape
    rem = np.flatnonzero(np.asarray(removable, dtype=bool))
    bits = masks[..., rem]                      # [n][N][N][R]
    nbits = N * N * rem.size
    if translations and nbits <= 62:
        weights = (np.int64(1) << np.arange(nbits, dtype=np.int64))
        best = None
        for a in range(N):
            for b in range(N):
                code = np.roll(bits, (a, b), axis=(1, 2)).reshape(n, -1).astype(np.int64) @ weights
                best = code if best is None else np.minimum(best, code)
        return best
    if translations:
        # more removable sites than an int64 holds: the lexicographically
        # smallest packed bit string over the cyclic shifts
        best = None
        rows = np.arange(n)
        for a in range(N):
            for b in range(N):
                code = np.packbits(np.roll(bits, (a, b), axis=(1, 2)).reshape(n, -1), axis=1)
                if best is None:
                    best = code.copy()
                    continue
                diff = code != best
                at = diff.argmax(axis=1)
                less = diff.any(axis=1) & (code[rows, at] < best[rows, at])
                best[less] = code[less]
        return np.ascontiguousarray(best).view(np.dtype((np.void, best.shape[1]))).reshape(-1)
    packed = np.packbits(bits.reshape(n, -1), axis=1)
    return np.ascontiguousarray(packed).view(np.dtype((np.void, packed.shape[1]))).reshape(-1)


def make_levels(levels, Ks):
    """Level 1: plain Q on the coarsest supercell; level l >= 2: Y = Q_l - Q_l^CV
    with the quarters solved on level l-1's grid."""
    out = []
    for l, (N, K) in enumerate(zip(levels, Ks)):
        out.append(LevelState(N=N, K=K, coupled=l > 0, K_coarse=Ks[l - 1] if l > 0 else K))
    return out


def run_mlmc(est: Estimator, levels, Ks, tol_rel: float, C_alpha: float = 2.0, theta: float = 0.5, pilot: int = 16,
             max_rounds: int = 10, max_samples: int = 1_000_000, exact_first: bool = False,
             tol_sequence=None) -> MLMCResult:
    """Adaptive-sample MLMC over fixed levels (eq. (MLMC), eq. (opt_samples)).

    exact_first: level 1 is the exhaustive expectation over every outcome of
    its (small) supercell instead of a sample mean (Section 4.4); it then adds
    no variance and takes no part in the allocation.
    tol_sequence: relative tolerances worked through in order before tol_rel
    (continuation: each stage re-estimates V_l and W_l from all samples so far
    and allocates for its own tolerance; samples are kept from stage to stage).
    """
    lv = make_levels(levels, Ks)
    t0 = time.perf_counter()
    exact = None
    if exact_first:
        t1 = time.perf_counter()
        exact = est.exhaustive_expectation(lv[0].N, lv[0].K)
        lv[0].seconds = time.perf_counter() - t1
    sampled = lv[1:] if exact_first else lv
    target = [pilot] * len(sampled)
    rounds = []
    err = tol_abs = float("inf")
    estimate = None
    stages = list(tol_sequence or []) + [tol_rel]
    stage = 0
    for _ in range(max_rounds * len(stages)):
        if hasattr(est, "add_round"):  # a client of a server: the round's samples of all levels at once
            est.add_round([(st, min(t, max_samples) - st.M) for t, st in zip(target, sampled)])
        else:
            for t, st in zip(target, sampled):
                est.add_samples(st, min(t, max_samples) - st.M)
        means, V = [], []
        for st in sampled:
            m, v = st.mean_var()
            means.append(m)
            V.append(max(float(v.max()), 1e-300))
        W = [st.seconds / st.M for st in sampled]
        estimate = np.sum(means, axis=0) + (exact if exact is not None else 0.0)
        tol_abs = tol_rel * float(np.max(np.abs(estimate)))
        stage_tol = stages[stage] * float(np.max(np.abs(estimate)))
        M = [st.M for st in sampled]
        err = C_alpha * math.sqrt(sum(v / m for v, m in zip(V, M)))
        rounds.append({"M": M, "V": V, "W": W, "error": err, "tol_abs": tol_abs, "stage_tol_rel": stages[stage],
                       "stage_tol_abs": stage_tol})
        if err <= theta * tol_abs:
            break
        while stage + 1 < len(stages) and err <= theta * stage_tol:
            stage += 1
            stage_tol = stages[stage] * float(np.max(np.abs(estimate)))
        Mopt = B.mlmc_optimal_samples(V, W, C_alpha, theta, stage_tol)
        target = [max(st.M, int(math.ceil(m))) for st, m in zip(sampled, Mopt)]
        if all(st.M >= max_samples for st in sampled):
            break
    return MLMCResult(estimate=estimate, levels=lv, error=err, tol_abs=tol_abs, seconds=time.perf_counter() - t0,
                      rounds=rounds)


def continuation_tolerances(tol_rel: float, stages: int = 3, ratio: float = 2.0):
    """Relative tolerances ratio^s * tol_rel for s = stages .. 1 (largest first),
    the sequence a continuation MLMC works through before tol_rel."""
    return [tol_rel * ratio ** s for s in range(stages, 0, -1)]


def run_mc(est: Estimator, N: int, K: int, M: int) -> LevelState:
    """Plain MC (eq. (MC)) with M samples on one supercell size."""
    lvl = LevelState(N=N, K=K, coupled=False, K_coarse=K)
    est.add_samples(lvl, M)
    return lvl
