"""Host-side checks of the serving loop's scheduling policy (continuous
batching, HBM-budget admission, first come first served across request
classes) against a simulated executor: no device work."""

import numpy as np
import pytest

from paper_1611_09784_amd.serve import (BatchLimits, Request, Server, SimClock, SimExecutor, StreamSpec,
                                        poisson_requests, request_class)

GB = 1 << 30
BYTES = {("graphene", 4): 1 * GB, ("graphene", 8): 2 * GB, ("graphene", 16): 6 * GB, ("graphene", 32): 20 * GB,
         ("mos2_shaped", 4): 2 * GB, ("mos2_shaped", 8): 5 * GB, ("mos2_shaped", 16): 15 * GB,
         ("mos2_shaped", 32): 60 * GB}
SOLVES = {k: 80 for k in BYTES}
COST = {4: 0.01, 8: 0.02, 16: 0.1, 32: 1.0}


def make(budget=200 * GB, slots=4, limits=None, cost=None):
    clock = SimClock()
    ex = SimExecutor(clock, cost or (lambda cls, b: COST[cls.N] * (1 + 0.1 * b)), BYTES, SOLVES)
    srv = Server(ex, budget, slots=slots, limits=limits or BatchLimits(max_requests=8, max_solves=4096,
                                                                        max_bytes=200 * GB),
                 clock=clock, sleep=clock.sleep, idle_sleep=1e-3)
    return srv, ex, clock


def test_request_class_levels():
    assert request_class("graphene", 4) == request_class("graphene", 4)
    c = request_class("graphene", 4)
    assert (c.coupled, c.K, c.K_coarse) == (False, 8, 8)
    c = request_class("mos2_shaped", 16)
    assert (c.coupled, c.K, c.K_coarse) == (True, 2, 4)
    with pytest.raises(ValueError):
        request_class("graphene", 5)


def test_every_request_completes_with_its_own_rows():
    srv, ex, _ = make()
    reqs = poisson_requests(StreamSpec(rate=50.0, count=120))
    rep = srv.run(reqs)
    assert all(np.isfinite(r.done) for r in reqs)
    for r in reqs:
        assert r.Y[0] == r.rid and r.Q[0] == -r.rid
        assert r.done >= r.admitted >= r.arrival
    assert rep.peak_bytes <= srv.budget
    assert rep.max_in_flight <= srv.slots


def test_budget_limits_concurrency():
    # four mos2 N=32 requests at once, 60 GB each, budget 130 GB: at most two in flight
    srv, ex, _ = make(budget=130 * GB, limits=BatchLimits(max_requests=1))
    reqs = [Request(i, "mos2_shaped", 32, 1, i, 0.0) for i in range(4)]
    rep = srv.run(reqs)
    assert rep.peak_bytes <= 130 * GB
    assert rep.max_in_flight == 2
    starts = sorted(t for t, *_ in ex.launched)
    assert starts[1] == 0.0 and starts[2] > 0.9   # the third waits for a completion


def test_request_larger_than_budget_is_refused():
    srv, _, _ = make(budget=50 * GB)
    with pytest.raises(ValueError):
        srv.run([Request(0, "mos2_shaped", 32, 1, 0, 0.0)])


def test_first_come_first_served_across_classes():
    # a big request waiting for memory is not overtaken by later small ones
    srv, ex, _ = make(budget=70 * GB, slots=4, limits=BatchLimits(max_requests=1))
    reqs = [Request(0, "mos2_shaped", 32, 1, 0, 0.0), Request(1, "mos2_shaped", 32, 1, 1, 0.001)]
    reqs += [Request(2 + i, "graphene", 4, 1, i, 0.002 + 0.001 * i) for i in range(5)]
    srv.run(reqs)
    order = [rids[0] for _, _, _, rids in ex.launched]
    assert order[:2] == [0, 1]
    t1 = next(t for t, _, _, rids in ex.launched if rids == [1])
    assert t1 > 0.9                       # waited for request 0's memory
    assert all(reqs[k].admitted >= t1 for k in range(2, 7))


def test_continuous_batching_admits_into_free_slots():
    # a long batch holds one slot; requests arriving later use the other slots at once
    srv, ex, _ = make(slots=2, limits=BatchLimits(max_requests=4))
    reqs = [Request(0, "graphene", 32, 1, 0, 0.0)]
    reqs += [Request(1 + i, "graphene", 4, 1, i, 0.1 + 0.05 * i) for i in range(6)]
    srv.run(reqs)
    for r in reqs[1:]:
        assert r.admitted - r.arrival < 0.05      # never waits for the long batch
        assert r.done < reqs[0].done


def test_batches_group_waiting_requests_of_one_class():
    srv, ex, _ = make(slots=1, limits=BatchLimits(max_requests=3))
    reqs = [Request(0, "graphene", 16, 1, 0, 0.0)] + [Request(1 + i, "graphene", 8, 1, i, 0.01) for i in range(7)]
    srv.run(reqs)
    sizes = [len(rids) for *_, rids in ex.launched]
    assert sizes == [1, 3, 3, 1]


def test_solve_limit_caps_batches():
    srv, ex, _ = make(slots=1, limits=BatchLimits(max_requests=64, max_solves=200))
    reqs = [Request(i, "graphene", 8, 1, i, 0.0) for i in range(10)]
    srv.run(reqs)
    assert max(len(rids) for *_, rids in ex.launched) == 2   # 80 solves per request


def test_poisson_stream_shape():
    spec = StreamSpec(rate=20.0, count=4000)
    reqs = poisson_requests(spec)
    arr = np.array([r.arrival for r in reqs])
    assert arr[0] == 0.0 and np.all(np.diff(arr) >= 0)
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 1 / 20.0) < 0.1 / 20.0
    Ns = np.array([r.N for r in reqs])
    for N, w in zip(spec.Ns, spec.weights):
        assert abs(np.mean(Ns == N) - w) < 0.03
    lats = np.array([r.lattice == "graphene" for r in reqs])
    assert abs(lats.mean() - 0.5) < 0.03
    # indices count up per (lattice, N) stream
    seen = {}
    for r in reqs:
        assert r.index == seen.get((r.lattice, r.N), 0)
        seen[(r.lattice, r.N)] = r.index + 1


def test_heavy_classes_leave_a_slot_for_light_requests():
    # heavy requests (N = 32) hold at most slots - 1 slots; light ones arriving later start at once
    srv, ex, _ = make(slots=3, limits=BatchLimits(max_requests=1))
    reqs = [Request(i, "graphene", 32, 1, i, 0.0) for i in range(4)]
    reqs += [Request(4 + i, "graphene", 4, 1, i, 0.05 + 0.02 * i) for i in range(4)]
    rep = srv.run(reqs)
    heavy_starts = sorted(r.admitted for r in reqs[:4])
    assert heavy_starts[:2] == [0.0, 0.0] and heavy_starts[2] > 0.9   # two heavy slots of three
    for r in reqs[4:]:
        assert r.admitted - r.arrival < 0.03
    assert rep.max_in_flight == 3
