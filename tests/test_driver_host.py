"""Host logic of the MLMC driver (no GPU): outcome identification for the
duplicate-outcome reuse and exhaustive enumeration (Section 4.4), and the
sample allocation loop with an exact first level and a continuation
sequence of tolerances."""

import itertools
import math

import numpy as np
import pytest

from paper_1611_09784_amd import driver as D


def translates(m):
    N = m.shape[0]
    return [np.roll(m, (a, b), axis=(0, 1)) for a in range(N) for b in range(N)]


@pytest.mark.parametrize("N,G,removable", [(3, 2, [1, 1]), (2, 3, [0, 1, 1]), (4, 2, [1, 1]),
                                           (6, 2, [1, 1]), (8, 2, [1, 1])])   # 72 and 128 removable sites
def test_translation_keys_identify_exactly_the_translates(N, G, removable):
    rng = np.random.default_rng(N * 10 + G)
    masks = (rng.random((60, N, N, G)) < 0.3).astype(np.uint8)
    masks[..., np.flatnonzero(np.array(removable) == 0)] = 0
    masks[30:40] = [translates(masks[i])[(i * 7) % (N * N)] for i in range(10)]   # planted translates
    keys = D.outcome_keys(masks, np.array(removable, np.uint8), translations=True)
    for i, j in itertools.combinations(range(len(masks)), 2):
        same = any(np.array_equal(t, masks[j]) for t in translates(masks[i]))
        assert (keys[i] == keys[j]) == same
    exact = D.outcome_keys(masks, np.array(removable, np.uint8), translations=False)
    for i, j in itertools.combinations(range(len(masks)), 2):
        assert (exact[i] == exact[j]) == np.array_equal(masks[i], masks[j])


class FakeEstimator:
    """Levels with known per-sample variance v_l and cost w_l; sample values
    are drawn from a seeded normal so that the allocation loop can run."""

    def __init__(self, v, w, seed=0):
        self.v, self.w = v, w
        self.rng = np.random.default_rng(seed)
        self.exact_calls = 0

    def add_samples(self, lvl, count):
        if count <= 0:
            return
        l = int(round(math.log2(lvl.N))) - 1
        x = self.rng.normal(1.0 / (l + 1), math.sqrt(self.v[l]), size=(count, 3))
        st = np.stack([x.sum(0), (x * x).sum(0), x.sum(0), (x * x).sum(0)])
        lvl.stats = st if lvl.stats is None else lvl.stats + st
        lvl.M += count
        lvl.seconds += count * self.w[l]

    def exhaustive_expectation(self, N, K):
        self.exact_calls += 1
        return np.full(3, 0.5)


def test_continuation_and_exact_first_allocation():
    v = [4e-3, 1e-3, 2.5e-4, 6e-5]
    w = [1e-4, 4e-4, 1.6e-3, 6.4e-3]
    tol = 2e-3
    est = FakeEstimator(v, w, seed=3)
    seq = D.continuation_tolerances(tol, stages=3, ratio=2.0)
    assert seq == pytest.approx([tol * 8, tol * 4, tol * 2])
    res = D.run_mlmc(est, [2, 4, 8, 16], [4, 2, 1, 1], tol, pilot=8, tol_sequence=seq, exact_first=True,
                     max_rounds=20)
    assert est.exact_calls == 1
    assert res.levels[0].M == 0                       # the exact level is not sampled
    assert res.error <= 0.5 * res.tol_abs             # theta * TOL reached
    stage = [r["stage_tol_rel"] for r in res.rounds]
    assert all(a >= b for a, b in zip(stage, stage[1:]))   # tolerances only tighten
    assert stage[0] == seq[0] and stage[-1] in seq + [tol]
    Ms = [r["M"] for r in res.rounds]
    assert all(all(a <= b for a, b in zip(m0, m1)) for m0, m1 in zip(Ms, Ms[1:]))  # samples are kept
    # estimate = exact level 1 + sample means of the other levels
    means = sum(st.stats[0] / st.M for st in res.levels[1:])
    assert np.allclose(res.estimate, 0.5 + means, rtol=0, atol=1e-15)
