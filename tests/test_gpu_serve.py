"""The serving loop on the GPU: a request's rows (Y and Q_f per energy) are
the same bit for bit whether it is served alone or in a mix of requests of
other lattices and supercell sizes that arrive while it runs, in FP64 and in
mixed precision; spot checks against the oracle's single-sample level sums."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from mlmc_inputs import energy_grid, graphene, mos2_shaped  # noqa: E402
from mlmc_inputs.configs import mos2_energy_window  # noqa: E402

pytestmark = pytest.mark.gpu

P = 0.05
DELTA = 0.05


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    from paper_1611_09784_amd import binding
    binding.lib()
    lats = {"graphene": graphene(), "mos2_shaped": mos2_shaped()}
    lo, hi = mos2_energy_window(lats["mos2_shaped"])
    eps = {"graphene": energy_grid(-9.0, 9.0, 101), "mos2_shaped": energy_grid(lo, hi, 101)}
    return binding, lats, eps


def mix():
    from paper_1611_09784_amd.serve import Request
    spec = [("graphene", 4), ("mos2_shaped", 4), ("graphene", 8), ("graphene", 16), ("mos2_shaped", 8),
            ("graphene", 4), ("graphene", 32), ("mos2_shaped", 4), ("graphene", 8), ("mos2_shaped", 16),
            ("graphene", 16), ("graphene", 4), ("mos2_shaped", 8), ("graphene", 8)]
    # staggered arrivals, then a burst of small requests arriving together
    times = [0.004 * i for i in range(len(spec))]
    spec += [("graphene", 4)] * 4 + [("mos2_shaped", 4)] * 3
    times += [0.02] * 7
    out, count = [], {}
    for i, ((lat, N), t) in enumerate(zip(spec, times)):
        k = count.get((lat, N), 0)
        count[(lat, N)] = k + 1
        out.append(Request(rid=i, lattice=lat, N=N, seed=606, index=3 + k, arrival=t))
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [0, 1])
def test_served_alone_equals_in_mix(setup, prec):
    from paper_1611_09784_amd.serve import BatchLimits, GpuExecutor, Request, Server
    B, lats, eps = setup
    ex = GpuExecutor(lats, eps, DELTA, P, prec, slots=3)
    try:
        srv = Server(ex, 100 << 30, slots=3, limits=BatchLimits(max_requests=4))
        reqs = mix()
        say(f"[serve prec={prec}] {len(reqs)} requests in a mix")
        rep = srv.run(reqs)
        say(f"[serve prec={prec}] {rep.summary()}")
        assert rep.max_in_flight >= 2          # batches overlapped on the device
        assert rep.batches < len(reqs)         # and some requests shared a batch
        for r in reqs:
            solo = Request(rid=r.rid, lattice=r.lattice, N=r.N, seed=r.seed, index=r.index, arrival=0.0)
            Server(ex, 100 << 30, slots=1).run([solo])
            assert np.array_equal(solo.Y, r.Y), f"request {r.rid}: Y differs alone and in the mix"
            assert np.array_equal(solo.Q, r.Q), f"request {r.rid}: Q differs alone and in the mix"
        # oracle spot checks on the small classes
        from paper_1611_09784_amd.serve import request_class
        tol = 1e-10 if prec == 0 else 1e-5
        for r in reqs:
            if r.N > 8:
                continue
            c = request_class(r.lattice, r.N)
            want = oracle.level_estimate(lats[r.lattice], r.N, c.coupled, P, c.K, c.K_coarse, B.MLMC_KGRID_GAMMA,
                                         r.seed, r.index, 1, eps[r.lattice], DELTA, 0, n_threads=8)
            assert np.abs(r.Y - want[0]).max() <= tol, f"request {r.rid}"
            assert np.abs(r.Q - want[2]).max() <= tol, f"request {r.rid}"
    finally:
        ex.close()


@pytest.mark.timeout(600)
def test_served_mlmc_client(setup):
    """The MLMC driver as a client of the server beside background requests:
    its level sums after one round equal the plain estimator's over the same
    samples (to summation order), and the adaptive run reaches theta * TOL."""
    import paper_1611_09784_amd.driver as D
    from paper_1611_09784_amd.serve import BatchLimits, GpuExecutor, Server, ServedEstimator, StreamSpec, \
        poisson_requests
    B, lats, eps = setup
    ex = GpuExecutor(lats, eps, DELTA, P, 0, slots=3)
    try:
        srv = Server(ex, 100 << 30, slots=3, limits=BatchLimits(max_requests=16))
        srv.open()
        bg = poisson_requests(StreamSpec(rate=40.0, count=60, Ns=(4, 8), weights=(0.6, 0.4), first_rid=1 << 30))
        srv.submit(bg)
        est = ServedEstimator(srv, "graphene", 303)
        levels, Ks = (4, 8, 16), [8, 4, 2]
        lv = D.make_levels(levels, Ks)
        est.add_round([(st, 6) for st in lv])
        ref = D.Estimator(B.DeviceLattice(lats["graphene"], 0), eps["graphene"], DELTA, P, B.MLMC_KGRID_GAMMA, 303)
        for st in lv:
            want = D.LevelState(N=st.N, K=st.K, coupled=st.coupled, K_coarse=st.K_coarse)
            ref.add_samples(want, 6)
            assert np.allclose(st.stats, want.stats, rtol=1e-12, atol=1e-14), f"level N = {st.N}"
        ref.close()
        r = D.run_mlmc(est, levels, Ks, 1e-2, pilot=8)
        say(f"[served MLMC client] M = {[st.M for st in r.levels]}, error {r.error:.3e}, tol_abs {r.tol_abs:.3e}")
        assert r.error <= 0.5 * r.tol_abs
        srv.drop_pending()
        while srv.busy():
            srv.step()
        assert sum(1 for q in srv.report().requests if (1 << 30) <= q.rid < (1 << 40)) > 0   # background beside
    finally:
        ex.close()
