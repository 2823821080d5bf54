"""Benchmark of the per-sample spectral hot path on one MI355X.

Workload (default): plain Monte Carlo on graphene, N = 16 supercell (512
sites, n <= 512 per H(k)), vacancy probability p = 0.05, 8 x 8
Monkhorst-Pack grid (64 H(k) per sample), 401 energies on [-9, 9] eV,
Gaussian smoothing delta = 0.05 eV, seed 202.  The full workload is 2000
samples = 128,000 eigensolves.

One step = one call of ``mlmc_level_estimate`` over a batch of samples: vacancy
sampling, k-grid, H(k) assembly, Householder tridiagonalisation, Sturm
bisection, smoothed IDoS and the level sums, all on the GPU with inputs and
workspace already resident.  The default 8 steps x 250 samples cover exactly
the 2000 samples of the workload.

Prints one JSON line.  ``value`` is eigensolves per second of the whole job.
``roofline`` reports the dominant kernel (timed with HIP events on the
library's stream during the timed region) against the FP64 peak, using the
algorithmic 16/3 n^3 real flops of a Hermitian tridiagonal reduction per
eigensolve.  ``cpu_baseline`` times the FP64 C oracle (unchanged) on a bounded
number of samples of the same workload on the host cores.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H(k) eigensolves/sec + MLMC IDoS time-to-TOL, mixed/served vs plain FP64 path"
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=250, help="samples per step")
    ap.add_argument("--chunk", type=int, default=32, help="samples per internal pass (workspace size)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--workload", default="graphene_n16_mc")
    ap.add_argument("--cpu-baseline", dest="cpu_baseline", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--cpu-samples", type=int, default=0, help="oracle samples (0: one per host thread)")
    return ap.parse_args()


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in DESIGN.md, not implemented)"}))
        sys.exit(2)

    import torch
    from mlmc_inputs import WORKLOADS
    from mlmc_inputs.configs import workload_eps
    from paper_1611_09784_amd import binding as B

    wl = WORKLOADS[args.workload]
    lat = wl.make_lattice()
    eps = workload_eps(wl)
    prec = B.MLMC_PREC_FP64 if args.precision == "fp64" else B.MLMC_PREC_MIXED
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    dlat = B.DeviceLattice(lat, 0)
    d_eps = torch.as_tensor(eps, device=dev)
    N, K = wl.N, wl.K
    nk = K * K
    need = B.mlmc_level_workspace(dlat, N, False, K, K, args.chunk, prec, eps.size)
    work = torch.empty((need,), dtype=torch.uint8, device=dev)
    stats = torch.zeros((4, eps.size), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(first):
        B.mlmc_level_estimate(dlat, N, False, wl.p, K, K, wl.kgrid, wl.seed, first, args.batch, d_eps, wl.delta,
                              wl.smoother, prec, stats=stats, work=work, stream=stream)

    print(f"[bench] workload={wl.name} N={N} K={K} batch={args.batch} steps={args.steps} warmup={args.warmup} "
          f"precision={args.precision} workspace={need / 2**30:.2f} GiB", file=sys.stderr, flush=True)
    for w in range(args.warmup):
        step((args.steps + w) * args.batch)
    torch.cuda.synchronize()
    stats.zero_()
    B.mlmc_timer_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i * args.batch)
        print(f"[bench] step {i + 1}/{args.steps} queued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    B.mlmc_timer_enable(False)
    kernels = {}
    for name in ("sample_vacancies", "kgrid", "assemble", "small_fused", "tridiag", "bisect", "idos",
                 "level_stats"):
        ms, cnt = B.mlmc_timer_read(name)
        if cnt:
            kernels[name] = {"ms": round(ms, 3), "launches": cnt}
    solves = args.steps * args.batch * nk
    value = solves / elapsed

    # Algorithmic work of the timed eigensolves: 16/3 n^3 real flops per H(k).
    masks = B.mlmc_sample_vacancies(dlat, N, wl.p, wl.seed, dlat.tag(N), 0, args.steps * args.batch).cpu().numpy()
    orb_per_group = np.bincount(lat.orb_group, minlength=lat.n_groups)
    vac_orbs = (masks.reshape(masks.shape[0], -1, lat.n_groups) * orb_per_group).sum(axis=(1, 2))
    n_per_sample = lat.n_orb * N * N - vac_orbs
    flops = float(nk * np.sum(16.0 / 3.0 * n_per_sample.astype(np.float64) ** 3))
    dom = max(kernels, key=lambda k: kernels[k]["ms"]) if kernels else None
    roofline = None
    if "tridiag" in kernels or "small_fused" in kernels:
        kname = "tridiag" if "tridiag" in kernels else "small_fused"
        kms = kernels[kname]["ms"]
        achieved = flops / (kms * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS if prec == B.MLMC_PREC_FP64 else FP32_PEAK_TFLOPS
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                    "frac": round(achieved / peak, 4), "traffic": None, "kernel": kname,
                    "avg_launch_ms": round(kms / kernels[kname]["launches"], 3),
                    "flops_per_launch": flops / kernels[kname]["launches"]}

    cpu = None
    if args.cpu_baseline:
        import oracle
        threads = host_threads()
        ns = args.cpu_samples or threads
        print(f"[bench] cpu baseline: oracle on {ns} samples with {threads} threads", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        oracle.level_estimate(lat, N, False, wl.p, K, K, wl.kgrid, wl.seed, 0, ns, eps, wl.delta, wl.smoother,
                              n_threads=threads)
        ct = time.perf_counter() - t1
        cpu = {"value": round(ns * nk / ct, 3), "unit": "eigensolves/s", "cores": threads, "kind": "oracle",
               "sample": f"{ns} samples x {nk} k-points of {wl.name} (samples 0..{ns - 1}), {ct:.1f} s",
               "cpu_model": cpu_model()}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "eigensolves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == B.MLMC_PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "lattice": wl.lattice, "N": N, "p": wl.p, "K": K,
                   "kgrid": "monkhorst-pack" if wl.kgrid == 0 else "gamma", "n_eps": int(eps.size),
                   "delta": wl.delta, "samples_per_step": args.batch, "eigensolves_per_step": args.batch * nk,
                   "precision": args.precision},
        "samples_per_s": round(args.steps * args.batch / elapsed, 3),
        "kernels_ms": kernels,
        "dominant_kernel": dom,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    dlat.close()


if __name__ == "__main__":
    main()
