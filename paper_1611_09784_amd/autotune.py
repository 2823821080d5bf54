"""Autotuner of the level calls' launch choices, from measured runs.

For one level configuration (lattice, N, coupling, k-grids, precision) it
measures samples per second of consecutive level calls (the same calls the
MLMC driver and the benchmark make: one pipeline context, two alternating
caller streams, one workspace) and picks, by coordinate descent,

1. the chunk size (samples per pass, which sets the workspace and the batch
   of every kernel launch), among powers of two that fit a memory budget;
2. on the two-stage path (matrices above the LDS-resident size): the number
   of persistent chase workgroups beside the next chunk's dense-to-band
   stage, and the row height of that stage's rank-2k update tiles (32 x 64 or
   64 x 64).

Choices are cached per device and configuration in a JSON file (the
``MLMC_TUNE_CACHE`` environment variable, else ``~/.cache/mlmc_autotune.json``)
and reused by later runs.  Every trial runs the full computation on fresh
samples; the tuner changes only launch shapes, never the results' meaning
(per-outcome results do not depend on them; the update tile changes rounding
only).
"""

from __future__ import annotations

import json
import os
import sys
import time
from dataclasses import asdict, dataclass

import numpy as np
import torch

from . import binding as B

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mlmc_autotune.json")


@dataclass
class LevelTuning:
    chunk: int
    chase_workgroups: int = 0     # 0: the library's default (3/4 of the CUs)
    update_tile_rows: int = 32
    samples_per_s: float = 0.0
    trials: int = 0

    def configure(self, ctx: B.Context):
        ctx.configure(chase_workgroups=self.chase_workgroups, update_tile_rows=self.update_tile_rows)


def _cache_path():
    return os.environ.get("MLMC_TUNE_CACHE", DEFAULT_CACHE)


def _device_name(dev) -> str:
    p = torch.cuda.get_device_properties(dev)
    return f"{p.name}|{p.multi_processor_count}"


def level_key(dlat, N, coupled, K, Kc, kind, prec, n_eps) -> str:
    lat = dlat.lat
    return (f"{_device_name(dlat.device)}|lat{lat.lattice_id}:{lat.n_orb}:{lat.n_groups}|N{N}|c{int(bool(coupled))}"
            f"|K{K}:{Kc}|g{kind}|p{prec}|e{n_eps}")


class Tuner:
    """Measured launch choices per level configuration, cached on disk."""

    def __init__(self, cache_path: str = None, budget_bytes: int = 48 << 30, min_seconds: float = 0.25,
                 chunks=(1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048), verbose: bool = False,
                 max_call_seconds: float = 1.0, chase_fractions=(0.5, 0.625, 0.75, 0.875, 1.0),
                 max_trial_seconds: float = 3.0):
        self.path = cache_path or _cache_path()
        self.budget = int(budget_bytes)
        self.min_seconds = float(min_seconds)
        self.max_call_seconds = float(max_call_seconds)
        self.fractions = tuple(chase_fractions)
        self.max_trial_seconds = float(max_trial_seconds)
        self.chunks = tuple(chunks)
        self.verbose = verbose
        self.cache = {}
        try:
            with open(self.path) as f:
                self.cache = json.load(f)
        except (OSError, ValueError):
            self.cache = {}

    def _save(self):
        try:
            os.makedirs(os.path.dirname(self.path), exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass

    # -- one measurement ----------------------------------------------------
    def _measure(self, dlat, N, coupled, K, Kc, kind, prec, eps, delta, p, seed, chunk, cfg, first,
                 samples_per_call=None, ctx=None):
        """Samples/s of consecutive level calls with the given choices, on
        the caller's context if one is given (else on a context of its own)."""
        dev = dlat.device
        need = B.mlmc_level_workspace(dlat, N, coupled, K, Kc, kind, chunk, prec, eps.shape[0])
        work = torch.empty((need,), dtype=torch.uint8, device=dev)
        stats = torch.zeros((4, eps.shape[0]), dtype=torch.float64, device=dev)

        # Calls (of four chunks, or of the caller's size) issued back to back
        # on alternating streams as the driver and the benchmark issue them,
        # so that every chunk but the last of the window runs in the pipelined
        # shape being measured.
        per_call = 4 * chunk if samples_per_call is None else int(samples_per_call)
        own = ctx is None
        if own:
            ctx = B.Context(dev.index)
        try:
            ctx.configure(chase_workgroups=cfg.chase_workgroups, update_tile_rows=cfg.update_tile_rows)
            streams = [ctx.stream(0), ctx.stream(1)]
            streams[0].wait_stream(torch.cuda.current_stream(dev))  # the workspace is ready

            def call(i):
                B.mlmc_level_estimate(dlat, N, coupled, p, K, Kc, kind, seed, first + i * per_call, per_call, eps,
                                      delta, prec=prec, stats=stats, work=work, ctx=ctx, stream=streams[i % 2])

            call(0)  # warm-up (first launches, workspace first touch)
            torch.cuda.synchronize(dev)
            t0 = time.perf_counter()
            call(1)
            torch.cuda.synchronize(dev)
            one = time.perf_counter() - t0
            calls = int(min(64, max(2, -(-self.min_seconds // max(one, 1e-6)))))
            t0 = time.perf_counter()
            for i in range(calls):
                call(2 + i)
            torch.cuda.synchronize(dev)
            el = time.perf_counter() - t0
            first += (calls + 2) * per_call
        finally:
            if own:
                ctx.close()
            else:
                ctx.configure()  # back to the library's defaults
        del work
        return calls * per_call / el, first, el / calls

    # -- coordinate descent -------------------------------------------------
    def tune_level(self, dlat, N, coupled, K, Kc, kind, prec, eps, delta, p, seed=987654321, retune=False,
                   max_chunk=None, samples_per_call=None, ctx=None) -> LevelTuning:
        """Launch choices for one level configuration.  samples_per_call:
        the size of the calls the caller makes (default four chunks).  ctx:
        the pipeline context the caller will run the level on; the trials
        then run on its streams (left configured with the library's defaults
        afterwards), which is what they should measure.  A context made and
        destroyed per trial is not the same thing: the runtime shares a few
        hardware queues among a process's streams, and after streams have
        come and gone a new context's chase stream can share a queue with one
        of its caller streams; work on one queue runs in order, so the chase
        then no longer overlaps the next chunk's reduction (measured: 23.0k
        against 25.9k FP64 eigensolves/s on the graphene N = 16 workload)."""
        eps = eps if isinstance(eps, torch.Tensor) else torch.as_tensor(np.asarray(eps, dtype=np.float64),
                                                                        device=dlat.device)
        key = level_key(dlat, N, coupled, K, Kc, kind, prec, eps.shape[0]) + \
            ("" if samples_per_call is None else f"|call{int(samples_per_call)}")
        if not retune and key in self.cache:
            return LevelTuning(**self.cache[key])
        ne = eps.shape[0]
        chunks = [c for c in self.chunks if (max_chunk is None or c <= max_chunk) and
                  B.mlmc_level_workspace(dlat, N, coupled, K, Kc, kind, c, prec, ne) <= self.budget]
        if not chunks:
            chunks = [1]
        start = min(8, chunks[-1])  # small chunks only where larger ones do not fit
        chunks = [c for c in chunks if c >= start]
        first = 1 << 40  # samples the tuner draws are never those of a run
        best = LevelTuning(chunk=chunks[0])
        trials = 0
        rates = {}
        slow = False
        for c in chunks:
            cfg = LevelTuning(chunk=c)
            t0 = time.perf_counter()
            r, first, per_call = self._measure(dlat, N, coupled, K, Kc, kind, prec, eps, delta, p, seed, c, cfg,
                                               first, samples_per_call, ctx)
            slow = time.perf_counter() - t0 > self.max_trial_seconds
            trials += 1
            rates[c] = r
            if self.verbose:
                print(f"[tune] {key} chunk {c}: {r:.1f} samples/s", file=sys.stderr, flush=True)
            if r > best.samples_per_s:
                best = LevelTuning(chunk=c, samples_per_s=r)
            elif r < 0.9 * best.samples_per_s:
                break  # past the optimum
            if per_call > self.max_call_seconds:
                break  # larger chunks only lengthen each call
        small_cap = B.SMALL_MAX[prec]
        # two-stage path: chase share and update tile (not for levels whose
        # trials are too long to afford a sweep)
        if dlat.max_orbitals(N) > small_cap and not slow:
            cus = torch.cuda.get_device_properties(dlat.device).multi_processor_count
            for tile in (32, 64):
                for frac in self.fractions:
                    g = max(1, int(round(cus * frac)))
                    cfg = LevelTuning(chunk=best.chunk, chase_workgroups=g, update_tile_rows=tile)
                    if (g, tile) == (int(cus * 0.75), 32) and best.chase_workgroups == 0:
                        continue  # the default, measured above
                    r, first, _ = self._measure(dlat, N, coupled, K, Kc, kind, prec, eps, delta, p, seed,
                                                best.chunk, cfg, first, samples_per_call, ctx)
                    trials += 1
                    if self.verbose:
                        print(f"[tune] {key} chase {g} tile {tile}: {r:.1f} samples/s", file=sys.stderr, flush=True)
                    if r > best.samples_per_s:
                        best = LevelTuning(chunk=best.chunk, chase_workgroups=g, update_tile_rows=tile,
                                           samples_per_s=r)
        best.trials = trials
        self.cache[key] = asdict(best)
        self._save()
        return best
