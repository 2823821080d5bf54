"""Serving loop: continuous batching of MLMC sample requests on one GPU.

A request asks for one sample of one MLMC level (Sections 2.2 and 3.3): the
vacancy outcome with index ``index`` of the stream (``seed``, tag of the
lattice and N) on the N x N supercell of a lattice, and returns that
outcome's per-energy values Y = Q_f [- (1/4) sum_q Q_q] and Q_f (the smoothed
IDoS of the fine supercell, eq. (IDoS) and eq. (MLMC_smoothing); on levels
N > the smallest, minus the mean of the four re-periodised quarters' IDoS,
the control variate of Figure "CV").  Every step runs in ``libmlmc.so``:
the outcome is drawn by ``mlmc_sample_vacancies`` into its slot of a batch's
mask buffer and the batch goes through ``mlmc_level_outcomes`` (assembly,
reduction, chase, bisection, IDoS, per-outcome rows), all device-resident,
with only the rows copied back.

Scheduling (``Server.run``):

* requests are grouped by class (lattice, N), each class with its k-grids
  (N K held constant) and its own batch limits;
* whenever a slot is free, the class of the oldest waiting request is served
  next (first come, first served across classes, so a large request is not
  starved by a stream of small ones): as many of its waiting requests as the
  class's batch limit and the free device memory allow form one batch;
* admission is by an HBM budget: a batch's device bytes (its level
  workspace, masks and rows) are reserved before launch and released when
  it completes; a class whose next request does not fit waits, and no other
  class is admitted before it;
* each slot owns one stream (a batch is a single pass, so it gains nothing
  from a pipeline context's extra streams, and one stream per slot keeps
  the slots on separate hardware queues), so up to ``slots`` batches run on
  the device at once, their kernels overlapping; a request that arrives
  while others run is admitted as soon as a slot and memory free up;
* heavy classes (large supercells, seconds per request) may hold at most
  ``heavy_slots`` slots at once, so light requests always find a slot; the
  oldest waiting light request goes first while every heavy slot is busy.

Per-outcome rows depend on the outcome alone (the kernels reduce every
matrix on its own, in a fixed order), so a request's result is the same bit
for bit alone and in any mix.  Latency is the time from a request's arrival
to the host seeing its batch complete.

The executor interface (``bytes_for``, ``launch``, handle ``done``/
``collect``/``release``) separates the policy from the device, so the policy
is also tested against a simulated executor on the CPU.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

SMALLEST_LEVEL_N = 4   # the uncoupled first level of the hierarchies
NK = 32                # N * K held constant across levels


@dataclass
class Request:
    rid: int
    lattice: str
    N: int
    seed: int
    index: int
    arrival: float                 # seconds after the start of the run
    admitted: float = math.nan
    done: float = math.nan
    batch: int = -1
    Y: np.ndarray = None
    Q: np.ndarray = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass(frozen=True)
class RequestClass:
    lattice: str
    N: int
    coupled: bool
    K: int
    K_coarse: int


def request_class(lattice: str, N: int, nk: int = NK, smallest: int = SMALLEST_LEVEL_N) -> RequestClass:
    """Level of an N x N supercell: K = nk / N; above the smallest level the
    sample is coupled with its four N/2 quarters on the K grid of N/2."""
    if N < 1 or nk % N != 0:
        raise ValueError(f"N = {N} does not divide N K = {nk}")
    coupled = N > smallest
    K = nk // N
    return RequestClass(lattice, N, coupled, K, (nk // (N // 2)) if coupled else K)


@dataclass
class BatchLimits:
    max_requests: int = 64
    max_solves: int = 4096          # eigensolves per batch (fine and quarters)
    max_bytes: int = 32 << 30       # device bytes per batch
    heavy_orbitals: int = 2048      # classes whose fine matrices have at least this many orbitals are heavy


@dataclass
class _Running:
    slot: int
    cls: RequestClass
    reqs: list
    handle: object
    nbytes: int
    launched: float


@dataclass
class ServeReport:
    requests: list
    seconds: float
    batches: int
    solves: int
    peak_bytes: int
    max_in_flight: int
    budget_bytes: int

    def latencies(self) -> np.ndarray:
        return np.array([r.latency for r in self.requests], dtype=np.float64)

    def summary(self) -> dict:
        lat = self.latencies()
        return {"requests": len(self.requests), "seconds": round(self.seconds, 4),
                "requests_per_s": round(len(self.requests) / self.seconds, 3) if self.seconds > 0 else None,
                "eigensolves": self.solves,
                "eigensolves_per_s": round(self.solves / self.seconds, 3) if self.seconds > 0 else None,
                "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3) if lat.size else None,
                "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3) if lat.size else None,
                "mean_ms": round(1e3 * float(lat.mean()), 3) if lat.size else None,
                "batches": self.batches, "max_batches_in_flight": self.max_in_flight,
                "peak_reserved_gb": round(self.peak_bytes / 1e9, 3), "budget_gb": round(self.budget_bytes / 1e9, 3)}


class Server:
    """Continuous-batching scheduler over an executor (see module docstring)."""

    def __init__(self, executor, budget_bytes: int, slots: int = 4, limits: BatchLimits = None,
                 clock=time.perf_counter, sleep=time.sleep, idle_sleep: float = 2e-4, heavy_slots: int = None):
        if slots < 1:
            raise ValueError("slots must be >= 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.heavy_slots = max(1, self.slots - 1) if heavy_slots is None else int(heavy_slots)
        self.limits = limits or BatchLimits()
        self.clock = clock
        self.sleep = sleep
        self.idle_sleep = idle_sleep

    def _heavy(self, cls: RequestClass) -> bool:
        return self.ex.orbitals(cls) >= self.limits.heavy_orbitals

    def _batch_size(self, cls: RequestClass, waiting: int, free_bytes: int) -> int:
        per = self.ex.solves_per_request(cls)
        b = min(waiting, self.limits.max_requests, max(1, self.limits.max_solves // max(1, per)))
        while b > 1 and (self.ex.bytes_for(cls, b) > min(free_bytes, self.limits.max_bytes)):
            b -= 1
        if self.ex.bytes_for(cls, b) > free_bytes:
            return 0
        return b

    # -- incremental use: open, submit, step / wait_for, report ---------------
    def open(self, on_complete=None):
        """Start a session: time 0 is now; requests submitted later carry
        arrival times relative to it."""
        self._pending = []          # not yet arrived, sorted by (arrival, rid)
        self._queues = {}           # class -> arrived requests in arrival order
        self._running = []
        self._free = list(range(self.slots))
        self._used = self._peak = self._max_in_flight = self._batches = self._solves = 0
        self._served = []
        self._on_complete = on_complete
        self._t0 = self.clock()

    def now(self) -> float:
        return self.clock() - self._t0

    def submit(self, requests: list):
        for r in requests:
            cls = request_class(r.lattice, r.N)
            if self.ex.bytes_for(cls, 1) > self.budget:
                raise ValueError(f"request {r.rid} ({r.lattice}, N = {r.N}) needs more than the HBM budget")
        self._pending = sorted(self._pending + list(requests), key=lambda r: (r.arrival, r.rid))

    def busy(self) -> bool:
        return bool(self._pending) or any(self._queues.values()) or bool(self._running)

    def drop_pending(self) -> int:
        """Forget requests that have not arrived yet; returns how many."""
        n = len(self._pending)
        self._pending = []
        return n

    def step(self):
        """One scheduler turn: arrivals, completions, admissions; sleeps
        briefly when none of them happened."""
        now = self.now()
        k = 0
        while k < len(self._pending) and self._pending[k].arrival <= now:
            r = self._pending[k]
            self._queues.setdefault(request_class(r.lattice, r.N), []).append(r)
            k += 1
        self._pending = self._pending[k:]
        progressed = False
        still = []
        for job in self._running:
            if job.handle.done():
                t = self.now()
                Y, Q = job.handle.collect()
                for i, r in enumerate(job.reqs):
                    r.done = t
                    r.Y = Y[i]
                    r.Q = Q[i]
                    self._served.append(r)
                    if self._on_complete is not None:
                        self._on_complete(r)
                job.handle.release()
                self._used -= job.nbytes
                self._free.append(job.slot)
                progressed = True
            else:
                still.append(job)
        self._running = still
        # admissions: oldest waiting request's class first (heavy classes
        # only while they hold fewer than heavy_slots slots)
        while self._free:
            heavy_busy = sum(1 for job in self._running if self._heavy(job.cls))
            heads = [(q[0].arrival, q[0].rid, c) for c, q in self._queues.items()
                     if q and (heavy_busy < self.heavy_slots or not self._heavy(c))]
            if not heads:
                break
            _, _, cls = min(heads, key=lambda h: (h[0], h[1]))
            q = self._queues[cls]
            b = self._batch_size(cls, len(q), self.budget - self._used)
            if b == 0:
                break  # wait for memory; no other class goes first
            reqs, self._queues[cls] = q[:b], q[b:]
            nbytes = self.ex.bytes_for(cls, b)
            slot = self._free.pop(0)
            t = self.now()
            for r in reqs:
                r.admitted = t
                r.batch = self._batches
            handle = self.ex.launch(slot, cls, reqs)
            self._running.append(_Running(slot, cls, reqs, handle, nbytes, t))
            self._used += nbytes
            self._peak = max(self._peak, self._used)
            self._max_in_flight = max(self._max_in_flight, len(self._running))
            self._batches += 1
            self._solves += b * self.ex.solves_per_request(cls)
            progressed = True
        if not progressed:
            wait = self.idle_sleep
            if self._pending and not self._running and not any(self._queues.values()):
                wait = max(0.0, min(0.05, self._pending[0].arrival - now))
            if wait > 0:
                self.sleep(wait)

    def wait_for(self, requests: list):
        """Step until every request in `requests` is complete."""
        while any(math.isnan(r.done) for r in requests):
            self.step()

    def report(self) -> ServeReport:
        reqs = self._served
        seconds = max((r.done for r in reqs), default=0.0)
        return ServeReport(requests=list(reqs), seconds=seconds, batches=self._batches, solves=self._solves,
                           peak_bytes=self._peak, max_in_flight=self._max_in_flight, budget_bytes=self.budget)

    def run(self, requests: list, on_complete=None) -> ServeReport:
        """Serve `requests` (arrival times relative to the start of the run);
        returns when all are complete.  on_complete(req) is called for each
        request as its batch completes."""
        self.open(on_complete)
        self.submit(requests)
        while self.busy():
            self.step()
        return self.report()


class ServedEstimator:
    """An MLMC client of a Server (the estimator of the MLMC driver): each
    round submits the round's new samples of every level as requests of one
    lattice and seed (outcome index = sample number of the level), waits for
    them while the server goes on with whatever else arrives, and turns the
    returned rows into level sums with the library's level-sum kernel.  A
    level's cost per sample W is its requests' share of their batches'
    service times."""

    def __init__(self, server: Server, lattice: str, seed: int, device=0):
        import torch
        from . import binding as B
        self.srv, self.lattice, self.seed = server, lattice, int(seed)
        self.B, self.torch = B, torch
        self.device = torch.device("cuda", device)
        self._rid = 1 << 40
        self.requests = []

    def add_round(self, items):
        """items: [(LevelState, count)]; adds `count` samples to each level."""
        torch, B = self.torch, self.B
        now = self.srv.now()
        per_level = []
        for lvl, count in items:
            reqs = []
            for i in range(max(0, count)):
                reqs.append(Request(rid=self._rid, lattice=self.lattice, N=lvl.N, seed=self.seed, index=lvl.M + i,
                                    arrival=now))
                self._rid += 1
            per_level.append((lvl, reqs))
        allr = [r for _, reqs in per_level for r in reqs]
        self.srv.submit(allr)
        self.srv.wait_for(allr)
        self.requests += allr
        for lvl, reqs in per_level:
            if not reqs:
                continue
            Y = torch.as_tensor(np.stack([r.Y for r in reqs]), device=self.device)
            Q = torch.as_tensor(np.stack([r.Q for r in reqs]), device=self.device)
            sy = B.mlmc_level_stats(Y).cpu().numpy()   # [sum Y, sum Y^2, ...]
            sq = B.mlmc_level_stats(Q).cpu().numpy()   # [sum Q, sum Q^2, ...]
            host = np.stack([sy[0], sy[1], sq[0], sq[1]])
            sizes = {}
            for r in self.srv._served:
                if r.batch >= 0:
                    sizes[r.batch] = sizes.get(r.batch, 0) + 1
            cost = sum((r.done - r.admitted) / sizes.get(r.batch, 1) for r in reqs)
            lvl.seconds += cost
            lvl.stats = host if lvl.stats is None else lvl.stats + host
            lvl.M += len(reqs)

    def add_samples(self, lvl, count: int):
        self.add_round([(lvl, count)])


# ---------------------------------------------------------------------------
# The device executor: batches through the C ABI.
# ---------------------------------------------------------------------------

class GpuExecutor:
    """Runs batches of one request class on a slot's stream and pipeline
    context: masks by mlmc_sample_vacancies (each request its own seed and
    index), then mlmc_level_outcomes, then the rows copied to pinned host
    memory; completion is an event on the slot's stream."""

    def __init__(self, lattices: dict, eps: dict, delta: float, p: float, prec: int, slots: int, device=0,
                 kind: int = None, max_rows: int = 64):
        import torch
        from . import binding as B
        self.B, self.torch = B, torch
        self.device = torch.device("cuda", device)
        self.kind = B.MLMC_KGRID_GAMMA if kind is None else kind
        self.dlat = {name: B.DeviceLattice(lat, device) for name, lat in lattices.items()}
        self.eps = {name: torch.as_tensor(np.asarray(e, dtype=np.float64), device=self.device)
                    for name, e in eps.items()}
        self.delta, self.p, self.prec = float(delta), float(p), int(prec)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]
        # rows come back through pinned buffers of each slot, allocated once
        # (a pinned allocation during the run could wait for the device)
        ne = max(e.shape[0] for e in self.eps.values())
        self.max_rows = max_rows
        self.hY = [torch.empty((max_rows, ne), dtype=torch.float64, pin_memory=True) for _ in range(slots)]
        self.hQ = [torch.empty((max_rows, ne), dtype=torch.float64, pin_memory=True) for _ in range(slots)]
        self._ws = {}

    def orbitals(self, cls: RequestClass) -> int:
        return self.dlat[cls.lattice].max_orbitals(cls.N)

    def solves_per_request(self, cls: RequestClass) -> int:
        B = self.B
        n = B.mlmc_kgrid_points(self.kind, cls.K)
        if cls.coupled:
            n += 4 * B.mlmc_kgrid_points(self.kind, cls.K_coarse)
        return n

    def _level_bytes(self, cls: RequestClass, b: int) -> int:
        key = (cls, b)
        if key not in self._ws:
            self._ws[key] = self.B.mlmc_level_outcomes_workspace(self.dlat[cls.lattice], cls.N, cls.coupled, cls.K,
                                                                 cls.K_coarse, self.kind, b, self.prec,
                                                                 self.eps[cls.lattice].shape[0])
        return self._ws[key]

    def bytes_for(self, cls: RequestClass, b: int) -> int:
        lat = self.dlat[cls.lattice].lat
        ne = self.eps[cls.lattice].shape[0]
        return self._level_bytes(cls, b) + b * cls.N * cls.N * lat.n_groups + 2 * b * ne * 8

    def launch(self, slot: int, cls: RequestClass, reqs: list):
        torch, B = self.torch, self.B
        dl = self.dlat[cls.lattice]
        eps = self.eps[cls.lattice]
        b = len(reqs)
        s = self.streams[slot]
        with torch.cuda.stream(s):
            work = torch.empty((self._level_bytes(cls, b),), dtype=torch.uint8, device=self.device)
            mask = torch.empty((b, cls.N, cls.N, dl.lat.n_groups), dtype=torch.uint8, device=self.device)
            Y = torch.empty((b, eps.shape[0]), dtype=torch.float64, device=self.device)
            Q = torch.empty_like(Y)
        if b > self.max_rows:
            raise ValueError(f"batch of {b} requests exceeds the executor's {self.max_rows} rows")
        tag = dl.tag(cls.N)
        for i, r in enumerate(reqs):
            B.mlmc_sample_vacancies(dl, cls.N, self.p, r.seed, tag, r.index, 1, out=mask[i], stream=s)
        B.mlmc_level_outcomes(dl, cls.N, cls.coupled, cls.K, cls.K_coarse, self.kind, mask, eps, self.delta,
                              prec=self.prec, Y=Y, Q=Q, work=work, stream=s, want_stats=False)
        ne = eps.shape[0]
        hY, hQ = self.hY[slot][:b, :ne], self.hQ[slot][:b, :ne]
        with torch.cuda.stream(s):
            hY.copy_(Y, non_blocking=True)
            hQ.copy_(Q, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return _GpuBatch(ev, (work, mask, Y, Q), hY, hQ, s)

    def close(self):
        for d in self.dlat.values():
            d.close()


class _GpuBatch:
    def __init__(self, ev, device_bufs, hY, hQ, stream):
        self.ev, self.bufs, self.hY, self.hQ, self.stream = ev, device_bufs, hY, hQ, stream

    def done(self) -> bool:
        return self.ev.query()

    def collect(self):
        # copies: the slot's pinned buffers take the next batch's rows
        return self.hY.numpy().copy(), self.hQ.numpy().copy()

    def release(self):
        # the caching allocator may hand these blocks to the next batch of any
        # stream only after this stream's work on them is complete
        for t in self.bufs:
            t.record_stream(self.stream)
        self.bufs = None


# ---------------------------------------------------------------------------
# A simulated executor (CPU tests of the policy).
# ---------------------------------------------------------------------------

class SimClock:
    """A clock that only moves when slept on (simulated time)."""

    def __init__(self):
        self.now = 0.0

    def __call__(self):
        return self.now

    def sleep(self, dt):
        self.now += dt


class SimExecutor:
    """Executor whose batches take `cost(cls, b)` seconds of a shared clock
    and whose rows are the request ids, so the policy can be checked without
    a device.  Batches in flight at once run concurrently."""

    def __init__(self, clock, cost, bytes_per_request: dict, solves: dict):
        self.clock, self.cost = clock, cost
        self.bpr, self.solves = bytes_per_request, solves
        self.launched = []

    def solves_per_request(self, cls):
        return self.solves[(cls.lattice, cls.N)]

    def orbitals(self, cls):
        return (11 if cls.lattice == "mos2_shaped" else 2) * cls.N * cls.N

    def bytes_for(self, cls, b):
        return b * self.bpr[(cls.lattice, cls.N)]

    def launch(self, slot, cls, reqs):
        t = self.clock()
        self.launched.append((t, slot, cls, [r.rid for r in reqs]))
        return _SimBatch(self.clock, t + self.cost(cls, len(reqs)), [r.rid for r in reqs])


class _SimBatch:
    def __init__(self, clock, end, rids):
        self.clock, self.end, self.rids = clock, end, rids

    def done(self):
        return self.clock() >= self.end

    def collect(self):
        a = np.array(self.rids, dtype=np.float64)[:, None]
        return a, -a

    def release(self):
        pass


def summarize_classes(requests: list) -> dict:
    """Latency percentiles per request class."""
    out = {}
    for r in requests:
        out.setdefault(f"{r.lattice}_N{r.N}", []).append(r.latency)
    return {k: {"count": len(v), "p50_ms": round(1e3 * float(np.percentile(v, 50)), 3),
                "p99_ms": round(1e3 * float(np.percentile(v, 99)), 3)} for k, v in sorted(out.items())}


@dataclass
class StreamSpec:
    """Poisson request stream: rate (requests/s), lattice uniform over
    `lattices`, N drawn with `weights`."""
    rate: float
    count: int
    lattices: tuple = ("graphene", "mos2_shaped")
    Ns: tuple = (4, 8, 16, 32)
    weights: tuple = (0.55, 0.30, 0.12, 0.03)
    seed: int = 5050
    sample_seed: int = 7070
    first_rid: int = 0
    extra: dict = field(default_factory=dict)


def poisson_requests(spec: StreamSpec) -> list:
    """Requests of a Poisson stream (exponential inter-arrival times with
    mean 1/rate from numpy's Generator(Philox(seed))); request i draws outcome
    i of its (sample_seed, lattice, N) stream."""
    rng = np.random.Generator(np.random.Philox(spec.seed))
    gaps = rng.exponential(1.0 / spec.rate, size=spec.count) if spec.rate > 0 else np.zeros(spec.count)
    arrivals = np.cumsum(gaps) - (gaps[0] if spec.count else 0.0)
    lat_idx = rng.integers(0, len(spec.lattices), size=spec.count)
    w = np.asarray(spec.weights, dtype=np.float64)
    n_idx = rng.choice(len(spec.Ns), size=spec.count, p=w / w.sum())
    counters = {}
    reqs = []
    for i in range(spec.count):
        lat, N = spec.lattices[lat_idx[i]], spec.Ns[n_idx[i]]
        k = counters.get((lat, N), 0)
        counters[(lat, N)] = k + 1
        reqs.append(Request(rid=spec.first_rid + i, lattice=lat, N=int(N), seed=spec.sample_seed, index=k,
                            arrival=float(arrivals[i])))
    return reqs
