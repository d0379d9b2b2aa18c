#!/usr/bin/env python3
"""Benchmark of the Swendsen-Wang sweep on one MI355X.

Default workload (the plain path): a 2D Ising lattice L=8192 at T_c and a 3D
lattice L=256 at T=4.5115, periodic, J=1, seed 1, random +-1 starts.  One step
is one sweep of both lattices (bonds, tile labelling, border merge, cluster
flip).  `value` is site-updates per second over the K timed steps with the
lattices resident in device memory.

Extra objects on the JSON line:
  roofline      the dominant kernel: algorithmic bytes per launch / its mean
                duration from HIP events recorded around every launch in the
                timed region, against the 8 TB/s HBM peak; `traffic` comes from
                the rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/ when
                it was taken on the current kernel sources, else null
  cpu_baseline  the CPU oracle (single thread) on a bounded sample
  batched       (--batched) 512 uneven replicas: batched phase launches replayed from a hipGraph
                vs plain per-lattice launches, site-updates/s each

Usage: python bench.py [--gpus 1] [--steps 200] [--warmup 5] [--no-cpu-baseline]
       [--batched] [--copy-probe]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SW site-updates/sec (batched vs plain) + % HBM roofline; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per site of each kernel: what the kernel must move,
# whatever it actually fetches
ALGO_BYTES_PER_SITE = {
    "k1_bond_label": 3.0,     # read the int8 spin, write the 16-bit tile label
    "k3_flip": 3.0,           # read the 16-bit tile label, write the int8 spin
    "k3_resolve": 0.25,       # read the border bitmap, write the border flip bits (1 bit each per site)
}
KERNEL_SYMBOLS = {"k1_bond_label": "k1_kernel", "k2_merge": "k2_kernel", "k3_flip": "k3_kernel",
                  "k3_resolve": "k3a_kernel"}
SOURCES = ["paper_0808_2109_amd/csrc/sw_device.hpp", "paper_0808_2109_amd/csrc/sw_kernels.hip"]


def source_hash() -> str:
    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(ROOT, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(workload):
    """The oracle, untuned, on one sweep of each lattice from its start."""
    import oracle

    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    sites = 0
    t0 = time.perf_counter()
    for rep in workload.replicas:
        spins = oracle.init_spins(rep.dim, rep.L, rep.seed)
        thr = oracle.threshold(rep.J, rep.T)
        oracle.sweep(rep.dim, rep.L, rep.seed, 0, thr, spins)
        sites += rep.nsites
    dt = time.perf_counter() - t0
    return {"value": sites / dt, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "sample": "sweep 0 of each lattice of the workload (8192^2 at T_c and 256^3 at T=4.5115) "
                      f"from the seed-1 start, {sites} site-updates in {dt:.1f} s, single thread"}


def traffic_from_profile(kernel_key: str, launch_sites: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", "traffic_pmc.json")
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    if prof.get("source_hash") != source_hash():
        return None
    k = prof.get("kernels", {}).get(kernel_key)
    if not k or k.get("sites") != launch_sites:
        return None
    return k.get("hbm_bytes_per_launch")


def copy_probe():
    """A plain device copy of known size, for scaling the FETCH/WRITE counters."""
    import torch

    n = 256 << 20
    src = torch.ones(n, dtype=torch.int8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 5}), flush=True)


def run_batched(swgpu, workloads, sweeps_batched: int, sweeps_plain: int):
    import torch

    wl = workloads.batched()
    params = [swgpu.params_from_replica(r) for r in wl.replicas]
    sites = sum(r.nsites for r in wl.replicas)
    out = {"replicas": len(params), "sites": sites}
    with swgpu.Lattice(params) as lat:
        lat.autotune(sweeps=2)
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep(sweeps_batched)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["batched"] = {"site_updates_per_s": sites * sweeps_batched / dt, "sweeps": sweeps_batched,
                          "seconds": dt}
        lat.set_mode(swgpu.SW_MODE_PLAIN)
        lat.sweep(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep(sweeps_plain)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["plain"] = {"site_updates_per_s": sites * sweeps_plain / dt, "sweeps": sweeps_plain, "seconds": dt}
    out["batched_over_plain"] = out["batched"]["site_updates_per_s"] / out["plain"]["site_updates_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--batched", action="store_true", help="also time the 512-replica batched workload")
    ap.add_argument("--batched-sweeps", type=int, default=100)
    ap.add_argument("--copy-probe", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

    import torch
    from paper_0808_2109_amd import swgpu, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    wl = workloads.plain()
    lats = []
    for rep in wl.replicas:
        lat = swgpu.Lattice(swgpu.params_from_replica(rep))
        if not args.no_autotune:
            lat.autotune(sweeps=3)
        lats.append(lat)
    shapes = [swgpu.tile_shapes(r.dim)[lat.tile_shape(0)] for r, lat in zip(wl.replicas, lats)]
    log(f"workload {wl.name}: {[r.nsites for r in wl.replicas]} sites, warmup {args.warmup}, steps {args.steps}")

    for _ in range(args.warmup):
        for lat in lats:
            lat.sweep(1)
    torch.cuda.synchronize()
    for lat in lats:
        lat.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for lat in lats:
            lat.sweep(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timings = [lat.timing() for lat in lats]
    sites = sum(r.nsites for r in wl.replicas)
    value = sites * args.steps / dt
    log(f"{args.steps} steps in {dt:.4f} s -> {value:.4e} site-updates/s")

    # per-kernel mean durations (HIP events around every launch of the timed region)
    kernels = {}
    for rep, tm in zip(wl.replicas, timings):
        tag = f"{rep.dim}d_L{rep.L}"
        for key, (ms, n) in tm.items():
            if n == 0 or key not in ALGO_BYTES_PER_SITE:
                continue
            avg_ms = ms / n
            algo = ALGO_BYTES_PER_SITE[key] * rep.nsites
            kernels[f"{key}:{tag}"] = {"kernel": key, "lattice": tag, "sites": rep.nsites, "mean_us": avg_ms * 1e3,
                                       "total_ms": ms, "launches": n,
                                       "algo_bytes_per_launch": algo,
                                       "achieved_GBs": algo / (avg_ms * 1e-3) / 1e9}
    dom = max(kernels.values(), key=lambda k: k["total_ms"])
    log("kernels:", json.dumps(kernels, indent=1))
    traffic = traffic_from_profile(f"{dom['kernel']}:{dom['lattice']}", dom["sites"])
    roofline = {"bound": "hbm", "kernel": f"{KERNEL_SYMBOLS[dom['kernel']]} ({dom['lattice']})",
                "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                "algo_bytes_per_site": ALGO_BYTES_PER_SITE[dom["kernel"]], "mean_launch_us": dom["mean_us"]}

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": "plain: 2D Ising L=8192 periodic at T_c=2/ln(1+sqrt2) + 3D Ising L=256 periodic "
                               "at T=4.5115, J=1, seed 1, one sweep of each lattice per step",
                   "lattices": [{"dim": r.dim, "L": r.L, "T": r.T, "seed": r.seed} for r in wl.replicas],
                   "tile_shapes": [list(s) for s in shapes],
                   "kernel_means_us": {k: round(v["mean_us"], 2) for k, v in kernels.items()}},
        "roofline": roofline,
    }
    for lat in lats:
        lat.close()
    if args.batched:
        result["batched"] = run_batched(swgpu, workloads, args.batched_sweeps, max(args.batched_sweeps // 10, 2))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        result["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
