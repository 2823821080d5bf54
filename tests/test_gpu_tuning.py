"""Graph-captured level calls and the autotuner on the GPU.

* A level call captured as a HIP graph (one stream, device-resident first
  sample index) and replayed: every replay, with eager work and
  synchronisation between replays, equals the eager level call on the same
  samples bit for bit (fused path, coupled fused path, two-stage path).
* The autotuner returns launch choices from measured runs, caches them, and a
  tuned estimator's level sums equal the untuned ones to rounding.
* The tuner's trials and several estimators on one caller-owned context give
  the level sums of estimators with contexts of their own.
"""

import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from mlmc_inputs import energy_grid, graphene  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1611_09784_amd import binding
    binding.lib()
    return binding


@pytest.fixture(scope="module")
def gdev(B):
    d = B.DeviceLattice(graphene(), 0)
    yield d
    d.close()


@pytest.mark.parametrize("N,coupled,K,Kc,prec,M,chunk", [
    (4, False, 8, 8, 0, 64, 16),     # fused path
    (8, True, 4, 8, 1, 32, 8),       # coupled, fused fine and quarters, mixed
    (16, False, 1, 1, 0, 8, 4),      # two-stage path (stage 1, chase, bisection on one stream)
])
def test_level_graph_replays_equal_eager_calls(B, gdev, N, coupled, K, Kc, prec, M, chunk):
    from paper_1611_09784_amd.driver import LevelGraph
    say(f"[graph] N={N} coupled={coupled} prec={prec} M={M}")
    eps = torch.as_tensor(energy_grid(-9.0, 9.0, 121), device=DEV)
    p, seed, kind = 0.05, 4321, B.MLMC_KGRID_GAMMA
    g = LevelGraph(gdev, N, coupled, p, K, Kc, kind, seed, M, eps, 0.05, 0, prec, chunk)
    for rep in range(4):
        first = 3 + rep * M
        got = torch.zeros((4, eps.shape[0]), dtype=torch.float64, device=DEV)
        g.run(first, 1, got)
        torch.cuda.synchronize()
        want = B.mlmc_level_estimate(gdev, N, coupled, p, K, Kc, kind, seed, first, M, eps, 0.05, prec=prec,
                                     chunk_samples=chunk)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), want.cpu().numpy()), f"replay {rep}"
    # several replays in one run: the samples continue
    got = torch.zeros((4, eps.shape[0]), dtype=torch.float64, device=DEV)
    g.run(100, 3, got)
    want = B.mlmc_level_estimate(gdev, N, coupled, p, K, Kc, kind, seed, 100, 3 * M, eps, 0.05, prec=prec,
                                 chunk_samples=chunk)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want.cpu().numpy())


def test_autotuner_choices_cached_and_results_unchanged(B, gdev, tmp_path):
    import paper_1611_09784_amd.driver as D
    from paper_1611_09784_amd.autotune import Tuner
    eps = energy_grid(-9.0, 9.0, 101)
    path = str(tmp_path / "tune.json")
    tuner = Tuner(cache_path=path, min_seconds=0.05, chunks=(4, 8, 16), verbose=True)
    t = tuner.tune_level(gdev, 16, True, 2, 4, B.MLMC_KGRID_GAMMA, 0, eps, 0.05, 0.02)
    say(f"[tune] {t}")
    assert t.chunk in (4, 8, 16) and t.update_tile_rows in (32, 64) and t.trials >= 2
    assert os.path.exists(path)
    again = Tuner(cache_path=path).tune_level(gdev, 16, True, 2, 4, B.MLMC_KGRID_GAMMA, 0, eps, 0.05, 0.02)
    assert again == t   # read back from the cache, no new trials
    lv_a = D.make_levels((8, 16), [4, 2])[1]
    lv_b = D.make_levels((8, 16), [4, 2])[1]
    plain = D.Estimator(gdev, eps, 0.05, 0.02, B.MLMC_KGRID_GAMMA, 303, chunk_samples=8)
    tuned = D.Estimator(gdev, eps, 0.05, 0.02, B.MLMC_KGRID_GAMMA, 303, tuner=Tuner(cache_path=path), graphs=True)
    plain.add_samples(lv_a, 20)
    tuned.add_samples(lv_b, 20)
    plain.close()
    tuned.close()
    assert np.allclose(lv_a.stats, lv_b.stats, rtol=1e-12, atol=1e-14)


def test_estimators_and_tuner_on_a_shared_context(B, gdev, tmp_path):
    """The tuner's trials and several estimators on one caller-owned context:
    closing an estimator leaves the context open, a plain estimator resets
    launch choices a tuned one left on it (its level sums equal those of an
    estimator with a context of its own bit for bit), and a tuned one equals
    them to rounding."""
    import paper_1611_09784_amd.driver as D
    from paper_1611_09784_amd.autotune import Tuner
    eps = energy_grid(-9.0, 9.0, 101)
    say("[shared ctx] tuning graphene N = 16, K = 1 on the caller's context")
    with B.Context(0) as ctx:
        tuner = Tuner(cache_path=str(tmp_path / "tune.json"), min_seconds=0.05, chunks=(4, 8))
        t = tuner.tune_level(gdev, 16, False, 1, 1, B.MLMC_KGRID_GAMMA, 0, eps, 0.05, 0.02, ctx=ctx)
        assert t.chunk in (4, 8) and t.trials >= 2
        levels = [D.make_levels((16,), [1])[0] for _ in range(3)]
        tuned = D.Estimator(gdev, eps, 0.05, 0.02, B.MLMC_KGRID_GAMMA, 303, tuner=tuner, ctx=ctx)
        tuned.add_samples(levels[0], 12)
        tuned.close()
        ctx.configure(chase_workgroups=64, update_tile_rows=64)  # choices a plain estimator must not inherit
        shared = D.Estimator(gdev, eps, 0.05, 0.02, B.MLMC_KGRID_GAMMA, 303, chunk_samples=8, ctx=ctx)
        shared.add_samples(levels[1], 12)
        shared.close()
        assert ctx.handle is not None  # still open after both estimators closed
        say("[shared ctx] estimator with a context of its own")
        own = D.Estimator(gdev, eps, 0.05, 0.02, B.MLMC_KGRID_GAMMA, 303, chunk_samples=8)
        own.add_samples(levels[2], 12)
        own.close()
    assert np.array_equal(levels[1].stats, levels[2].stats)
    assert np.allclose(levels[0].stats, levels[2].stats, rtol=1e-12, atol=1e-14)
