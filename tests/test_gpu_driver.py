"""GPU checks of the host driver's paths that go through the C ABI with
explicit outcomes: the exhaustive expectation with translation classes and
the duplicate-outcome reuse (Section 4.4), against the oracle and against the
plain level call on the same samples."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import mlmc as omlmc  # noqa: E402
from mlmc_inputs import energy_grid, graphene, mos2_shaped  # noqa: E402
from mlmc_inputs.configs import KGRID_GAMMA, KGRID_MP, SMOOTH_GAUSS  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1611_09784_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("name,N,K,kind", [("graphene", 2, 2, KGRID_MP), ("spairs", 2, 1, KGRID_GAMMA),
                                           ("mos2", 2, 1, KGRID_GAMMA)])
def test_exhaustive_expectation_with_translation_classes(B, name, N, K, kind):
    from paper_1611_09784_amd import driver as D
    say(f"[exhaustive] {name} N={N} K={K}")
    lat = {"graphene": graphene(), "spairs": mos2_shaped(s_pairs=True), "mos2": mos2_shaped()}[name]
    b = 9.0 if name == "graphene" else lat.hop_magnitude_bound() + 1.0
    eps = energy_grid(-b, b, 41)
    p, delta = 0.3, 0.5
    dl = B.DeviceLattice(lat, 0)
    try:
        est = D.Estimator(dl, eps, delta, p, kind, 1, SMOOTH_GAUSS, B.MLMC_PREC_FP64)
        got = est.exhaustive_expectation(N, K)
        classes = est.unique_solved
    finally:
        dl.close()
    want = omlmc.exhaustive_expectation(lat, N, p, K, kind, eps, delta, SMOOTH_GAUSS)
    assert np.abs(got - want).max() < 1e-10
    G = lat.n_groups
    r = int(sum(lat.group_removable[g % G] for g in range(N * N * G)))
    assert classes < 2 ** r                        # translation classes were merged


@pytest.mark.parametrize("N,coupled,K,Kc,M,prec", [(4, False, 2, 2, 300, 0), (4, True, 2, 4, 40, 0),
                                                   (4, False, 2, 2, 200, 1)])
def test_duplicate_reuse_equals_plain_level_call(B, N, coupled, K, Kc, M, prec):
    from paper_1611_09784_amd import driver as D
    say(f"[dedup] N={N} coupled={coupled} M={M} prec={prec}")
    lat = graphene()
    eps = energy_grid(-9.0, 9.0, 101)
    dl = B.DeviceLattice(lat, 0)
    try:
        plain = D.Estimator(dl, eps, 0.1, 0.05, KGRID_GAMMA, 303, SMOOTH_GAUSS, prec)
        dedup = D.Estimator(dl, eps, 0.1, 0.05, KGRID_GAMMA, 303, SMOOTH_GAUSS, prec, dedup_max_orbitals=512)
        a = D.LevelState(N=N, K=K, coupled=coupled, K_coarse=Kc)
        b = D.LevelState(N=N, K=K, coupled=coupled, K_coarse=Kc)
        for count in (M // 2, M - M // 2):
            plain.add_samples(a, count)
            dedup.add_samples(b, count)
        masks = B.mlmc_sample_vacancies(dl, N, 0.05, 303, dl.tag(N), 0, M).cpu().numpy()
    finally:
        dl.close()
    # every distinct outcome solved exactly once over both rounds (the second
    # round reuses the first round's outcomes)
    keys = D.outcome_keys(masks, lat.group_removable, translations=not coupled)
    assert dedup.unique_solved == np.unique(keys).size < M
    tol = 1e-10 if prec == 0 else 1e-6
    assert np.abs(a.stats[0] - b.stats[0]).max() <= M * tol
    assert np.abs(a.stats[2] - b.stats[2]).max() <= M * tol
    assert np.abs(a.stats[1] - b.stats[1]).max() <= 3 * M * tol
    if prec == 0:
        want = oracle.level_estimate(lat, N, coupled, 0.05, K, Kc, KGRID_GAMMA, 303, 0, M, eps, 0.1, SMOOTH_GAUSS,
                                     n_threads=8)
        assert np.abs(b.stats[0] - want[0]).max() <= M * 1e-10


def test_mlmc_with_exact_first_level_and_continuation(B):
    from paper_1611_09784_amd import driver as D
    say("[mlmc exact first + continuation]")
    lat = graphene()
    eps = energy_grid(-9.0, 9.0, 101)
    dl = B.DeviceLattice(lat, 0)
    try:
        est = D.Estimator(dl, eps, 0.1, 0.05, KGRID_GAMMA, 303, SMOOTH_GAUSS, B.MLMC_PREC_FP64,
                          dedup_max_orbitals=128)
        res = D.run_mlmc(est, [2, 4, 8], [8, 4, 2], 5e-3, exact_first=True,
                         tol_sequence=D.continuation_tolerances(5e-3, 2))
    finally:
        dl.close()
    assert res.levels[0].M == 0
    assert res.error <= 0.5 * res.tol_abs
