#!/usr/bin/env python3
"""Benchmark of the Swendsen-Wang sweep on one MI355X.

`value` (the plain path): a 2D Ising lattice L=8192 at T_c and a 3D lattice
L=256 at T=4.5115, periodic, J=1, seed 1, random +-1 starts.  One step is one
sweep of both lattices (bonds, tile labelling, border merge, cluster flip);
`value` is site-updates per second over the K timed steps with the lattices
resident in device memory.

Objects on the JSON line besides the contract's fields:
  roofline           the dominant kernel (K1 on 8192^2): the method's bytes per
                     site-update (2 B: read the int8 spin, write it back) times the
                     sites of one launch, over its mean duration from HIP events
                     recorded around every launch of the timed region, against the
                     8 TB/s HBM peak.  `traffic` is the measured HBM bytes per launch
                     from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary in profiles/
                     when it was taken on the current kernel sources, else null.
                     The kernel's own design bytes (spin in, 16-bit label out) are
                     reported beside it, and so is the whole sweep's rate in method
                     bytes against the peak.
  batched            the 512-replica workload (2D, L in {64..2048}, T in [2.0, 2.6]):
                     500 sweeps batched (phase launches replayed from a hipGraph)
                     and 500 sweeps of plain per-lattice launches, and their ratio
  pcc                64 replicas of 2D L=2048 with probability-changing cluster
                     feedback, batched: site-updates/s, the sweeps timed, and the
                     replicas' mean p against the critical FK value 2 - sqrt(2)
  serving            the first jobs of the Poisson job stream (rate 50/s) through
                     the continuous-batching server: p50 / p99 latency and
                     aggregate site-updates/s (the job count is stated)
  cpu_baseline       the CPU oracle, single thread, on a bounded sample of the
                     plain workload
  cpu_baseline_batched  the oracle run replica-parallel on the machine's host cores
                     (one process per core) on a sample of the batched workload

Usage: python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--no-cpu-baseline]
       [--no-batched] [--no-pcc] [--no-serving] [--pcc-sweeps K] [--serving-jobs J]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SW site-updates/sec (batched vs plain) + % HBM roofline; p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
# the method's HBM bytes per site-update: every sweep must read each int8 spin
# and write it back, whatever the kernels move in between
METHOD_BYTES_PER_SITE = 2.0
# the bytes each kernel of this design must move per site (its own input and
# output), reported beside the method's figure
ALGO_BYTES_PER_SITE = {
    "k1_bond_label": 3.0,     # read the int8 spin, write the 16-bit tile label
    "k3_flip": 3.0,           # read the 16-bit tile label, write the int8 spin
}
HOST_CORES = 16               # the host-core share of one GPU on the measurement box
KERNEL_SYMBOLS = {"k1_bond_label": "k1_kernel", "k2_merge": "k2_kernel", "k3_flip": "k3_kernel",
                  "k3_resolve": "k3a_kernel"}
SOURCES = ["paper_0808_2109_amd/csrc/sw_device.hpp", "paper_0808_2109_amd/csrc/sw_kernels.hip"]


def source_hash() -> str:
    """Hash of the kernel sources' code: comments and blank lines are left
    out, so that a counter summary stays valid across comment-only edits."""
    import re

    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(ROOT, s)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(workload, sweeps: int = 3):
    """The oracle, untuned, on the first sweeps of each lattice from its start."""
    import oracle

    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    sites = 0
    t0 = time.perf_counter()
    for rep in workload.replicas:
        spins = oracle.init_spins(rep.dim, rep.L, rep.seed)
        thr = oracle.threshold(rep.J, rep.T)
        for s in range(sweeps):
            spins, _ = oracle.sweep(rep.dim, rep.L, rep.seed, s, thr, spins)
            sites += rep.nsites
    dt = time.perf_counter() - t0
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": sites / dt, "unit": "site-updates/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_threads": os.cpu_count(),
            "sample": f"sweeps 0-{sweeps - 1} of each lattice of the workload (8192^2 at T_c and 256^3 at "
                      f"T=4.5115) from the seed-1 start, {sites} site-updates in {dt:.1f} s, single thread"}


def _oracle_replica_sweeps(args):
    """Worker: `sweeps` oracle sweeps of one replica from its start (site-updates done)."""
    dim, L, seed, T, sweeps = args
    import oracle

    oracle.run(dim, L, seed, sweeps, T=T, record_series=False, keep_labels=False)
    return L ** dim * sweeps


def cpu_baseline_batched(workload, sweeps: int = 3, cores: int = HOST_CORES):
    """The oracle on the batched workload, replicas spread over `cores` worker
    processes (the replicas are independent); started before anything touches
    the GPU, with the spawn method."""
    import multiprocessing as mp

    import oracle

    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    cores = max(1, min(cores, os.cpu_count() or 1))
    jobs = [(r.dim, r.L, r.seed, r.T, sweeps) for r in workload.replicas]
    jobs.sort(key=lambda j: -j[1])                 # largest first: better balance
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        done = sum(pool.map(_oracle_replica_sweeps, jobs, chunksize=1))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"sweeps 0-{sweeps - 1} of all {len(jobs)} replicas of the batched workload from their "
                      f"starts, one process per core, {done} site-updates in {dt:.1f} s"}


def traffic_from_profile(kernel_key: str, launch_sites: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", PROFILE_PREFIX + "_traffic_pmc.json")
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


PROFILE_LATTICES = {2: ("2d_L8192", 8192 * 8192), 3: ("3d_L256", 256 ** 3)}
PROFILE_PREFIX = "plain_2d8192_3d256"   # the plain sweep workload: 8192^2 at T_c + 256^3 at T=4.5115


def _kernel_of(name: str):
    """(kernel key, lattice tag, sites) of a plain-path kernel name in a rocprofv3 database."""
    import re

    for key, sym in KERNEL_SYMBOLS.items():
        if f"sw::{sym}<" in name:
            m = re.search(r"TileCfg<(\d)", name)
            if m and int(m.group(1)) in PROFILE_LATTICES:
                tag, sites = PROFILE_LATTICES[int(m.group(1))]
                return key, tag, sites
    return None


def _db_rows(db_dir: str, query: str):
    import glob
    import sqlite3

    dbs = sorted(glob.glob(os.path.join(db_dir, "**", "*_results.db"), recursive=True))
    if not dbs:
        raise SystemExit(f"no rocprofv3 database under {db_dir}")
    con = sqlite3.connect(dbs[-1])
    try:
        return list(con.execute(query))
    finally:
        con.close()


def summarize_profiles(prof_dir: str, out_dir: str, trace_cmd: str, pmc_cmd: str, copy_cmd: str,
                       event_steps: int = 200):
    """Kernel-trace statistics and HBM traffic per launch from rocprofv3 runs.

    prof_dir holds the databases of five runs: trace/ (--kernel-trace --stats),
    fetch/ and write/ (--pmc FETCH_SIZE, --pmc WRITE_SIZE on the same bench
    command) and copy_fetch/, copy_write/ (the same counters on a plain device
    copy of known size, which gives the scale of each counter).
    """
    import collections

    os.makedirs(out_dir, exist_ok=True)
    # 1) kernel trace: calls, mean / min / max duration per kernel, and the
    #    mean over the last `event_steps` launches of each plain-path kernel:
    #    the pass in which the bench times every launch with events, with the
    #    lattices' sweeps one after the other (in the pass before it the two
    #    lattices' kernels may overlap)
    rows = _db_rows(os.path.join(prof_dir, "trace"), "select name, duration from kernels order by start")
    stats = collections.defaultdict(list)
    for name, dur in rows:
        stats[name].append(dur / 1e3)
    total = sum(sum(v) for v in stats.values())
    lines = [f"# rocprofv3 kernel trace, plain sweep workload (8192^2 at T_c + 256^3 at T=4.5115)",
             f"# command: {trace_cmd}",
             f"# event_pass_us: mean over the last {event_steps} launches (the bench's event-timed pass, each kernel alone)",
             "#",
             f"# {'calls':>6} {'mean_us':>10} {'event_pass_us':>14} {'min_us':>10} {'max_us':>10} {'share':>7}  kernel"]
    trace_means = {}
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        k = _kernel_of(name)
        tail = v[-event_steps:] if k and len(v) >= event_steps else None
        ev = f"{sum(tail) / len(tail):14.2f}" if tail else f"{'-':>14}"
        lines.append(f"  {len(v):6d} {sum(v) / len(v):10.2f} {ev} {min(v):10.2f} {max(v):10.2f} "
                     f"{100 * sum(v) / total:6.1f}%  {name[:110]}")
        if tail:
            trace_means[f"{k[0]}:{k[1]}"] = sum(tail) / len(tail)
    with open(os.path.join(out_dir, PROFILE_PREFIX + "_kernel_trace.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    # 2) counters: KiB per dispatch summed over the counter's instances
    def per_dispatch(sub: str, counter: str):
        q = ("select k.dispatch_id, k.name, p.counter_value from pmc_events p join kernels k "
             f"on p.dispatch_id = k.dispatch_id where p.counter_name = '{counter}'")
        acc = collections.defaultdict(float)
        names = {}
        for did, name, val in _db_rows(os.path.join(prof_dir, sub), q):
            acc[did] += val
            names[did] = name
        by = collections.defaultdict(list)
        for did, v in acc.items():
            by[names[did]].append(v)
        return {n: sum(v) / len(v) for n, v in by.items()}

    fetch, write = per_dispatch("fetch", "FETCH_SIZE"), per_dispatch("write", "WRITE_SIZE")
    cf, cw = per_dispatch("copy_fetch", "FETCH_SIZE"), per_dispatch("copy_write", "WRITE_SIZE")
    copy_kib = COPY_PROBE_BYTES / 1024.0
    cname = [n for n in cf if "copyBuffer" in n or "copy" in n.lower()]
    if not cname:
        raise SystemExit("no copy kernel in the copy-probe databases")
    fetch_scale = copy_kib / cf[cname[0]]
    write_scale = copy_kib / cw[cname[0]]
    kernels = {}
    lines = [f"# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (KiB per dispatch, summed over",
             f"# instances), each scaled by what the counter reads for a device copy of {COPY_PROBE_BYTES} bytes",
             f"# (FETCH_SIZE reads {cf[cname[0]]:.0f} KiB -> x{fetch_scale:.3f}; WRITE_SIZE reads {cw[cname[0]]:.0f} KiB "
             f"-> x{write_scale:.3f})",
             f"# commands: {pmc_cmd}", f"#           {copy_cmd}", "#",
             f"# {'fetch_MB':>10} {'write_MB':>10} {'algo_MB':>10} {'traffic/algo':>12}  kernel"]
    for name in sorted(fetch):
        k = _kernel_of(name)
        fb = fetch[name] * 1024 * fetch_scale
        wb = write.get(name, 0.0) * 1024 * write_scale
        algo = None
        if k:
            key, tag, sites = k
            algo = ALGO_BYTES_PER_SITE.get(key, 0.0) * sites
            kernels[f"{key}:{tag}"] = {"sites": sites, "hbm_bytes_per_launch": fb + wb, "fetch_bytes": fb,
                                       "write_bytes": wb, "trace_mean_us": trace_means.get(f"{key}:{tag}")}
        ratio = f"{(fb + wb) / algo:12.2f}" if algo else f"{'-':>12}"
        lines.append(f"  {fb / 1e6:10.2f} {wb / 1e6:10.2f} {(algo or 0) / 1e6:10.2f} {ratio}  {name[:100]}")
    with open(os.path.join(out_dir, PROFILE_PREFIX + "_hbm_traffic.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, PROFILE_PREFIX + "_traffic_pmc.json"), "w") as f:
        json.dump({"source_hash": source_hash(), "fetch_scale": fetch_scale, "write_scale": write_scale,
                   "kernels": kernels}, f, indent=1)
    print(json.dumps({"written": [os.path.join(out_dir, PROFILE_PREFIX + n) for n in
                                  ("_kernel_trace.txt", "_hbm_traffic.txt", "_traffic_pmc.json")]}))


SQ_ORDER = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM", "SQ_INSTS_BRANCH",
            "SQ_ACTIVE_INST_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_ACTIVE_INST_LDS", "SQ_LDS_IDX_ACTIVE",
            "SQ_LDS_BANK_CONFLICT", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
            "SQ_ACTIVE_INST_ANY")


def summarize_sq(prof_dir: str, out_dir: str, cmd_a: str, cmd_b: str):
    """SQ counters of the plain path's kernels (last dispatch of each) from two
    rocprofv3 --pmc passes under prof_dir/sq_a and prof_dir/sq_b."""
    import collections

    cols = collections.OrderedDict()    # column title -> {counter: value}
    durs = collections.defaultdict(list)
    for sub in ("sq_a", "sq_b"):
        q = ("select k.dispatch_id, k.name, k.duration, p.counter_name, p.counter_value from pmc_events p "
             "join kernels k on p.dispatch_id = k.dispatch_id")
        last = {}                           # column -> dispatch id of its last launch
        vals = collections.defaultdict(lambda: collections.defaultdict(float))
        info = {}
        for did, name, dur, cname, val in _db_rows(os.path.join(prof_dir, sub), q):
            k = _kernel_of(name)
            if not k:
                continue
            key, tag, _ = k
            col = f"{key} {tag}"
            vals[did][cname] += val
            info[did] = (col, dur)
            if did > last.get(col, -1):
                last[col] = did
        for col, did in sorted(last.items()):
            cols.setdefault(col, {}).update(vals[did])
            durs[col].append(info[did][1] / 1e3)
    names = list(cols)
    lines = ["# rocprofv3 SQ counters, plain sweep workload (8192^2 at T_c + 256^3 at T=4.5115), last dispatch of each kernel",
             "# commands (two passes, at most 8 SQ counters each):", f"#   {cmd_a}", f"#   {cmd_b}",
             "# counter values are summed over the counter's instances", "#",
             "# " + f"{'counter':26s}" + "".join(f"{n:>22s}" for n in names)]
    for c in SQ_ORDER:
        if any(c in cols[n] for n in names):
            lines.append("  " + f"{c:26s}" + "".join(f"{cols[n].get(c, float('nan')):22.0f}" for n in names))
    lines.append("  " + f"{'duration_us (pass a, b)':26s}" +
                 "".join(f"{' / '.join(f'{d:.1f}' for d in durs[n]):>22s}" for n in names))
    lines += ["#", "# derived (per kernel):"]
    for n in names:
        v = cols[n]
        w = v.get("SQ_WAVES", 0.0) or float("nan")
        lanes = v.get("SQ_THREAD_CYCLES_VALU", 0.0) / (v.get("SQ_ACTIVE_INST_VALU", 0.0) or float("nan"))
        confl = v.get("SQ_LDS_BANK_CONFLICT", 0.0) / (v.get("SQ_LDS_IDX_ACTIVE", 0.0) or float("nan"))
        lines.append(f"#   {n}: VALU instructions per wave {v.get('SQ_INSTS_VALU', 0) / w:.0f}, "
                     f"SALU {v.get('SQ_INSTS_SALU', 0) / w:.0f}, LDS {v.get('SQ_INSTS_LDS', 0) / w:.0f}, "
                     f"VMEM {v.get('SQ_INSTS_VMEM', 0) / w:.0f}; active lanes per VALU instruction {lanes:.1f} of 64; "
                     f"LDS bank-conflict cycles / LDS active cycles {confl:.2f}")
    path = os.path.join(out_dir, PROFILE_PREFIX + "_sq_counters.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({"written": [path]}))


COPY_PROBE_BYTES = 256 << 20


def copy_probe():
    """A plain device copy of known size, for scaling the FETCH/WRITE counters."""
    import torch

    n = COPY_PROBE_BYTES
    src = torch.ones(n, dtype=torch.int8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n, "launches": 5}), flush=True)


def run_batched(swgpu, workloads, sweeps_batched: int, sweeps_plain: int):
    """The 512-replica workload: batched sweeps (graph replay) against plain
    per-lattice launches of the same replicas from the same state."""
    import torch

    wl = workloads.batched()
    params = [swgpu.params_from_replica(r) for r in wl.replicas]
    sites = sum(r.nsites for r in wl.replicas)
    out = {"workload": wl.name, "replicas": len(params), "sites": sites}
    # the timed sweeps run as calls of `chunk` sweeps, the way a driver loop
    # calls sw_sweep; the first call of that size (untimed) captures the
    # hipGraph that the timed calls replay
    chunk = max(1, min(100, sweeps_batched))
    with swgpu.Lattice(params) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(10)                       # warm-up: the tuner times the current state
        lat.autotune(sweeps=2)
        out["tile_shape"] = list(swgpu.tile_shapes(2)[lat.tile_shape(0)])
        out["workgroups_per_cu"] = lat.batch_grid()
        out["engine"] = ("graph", "persistent")[lat.batch_engine()[0]]
        out["merge_width"] = lat.merge_width()
        lat.sweep(chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < sweeps_batched:
            lat.sweep(min(chunk, sweeps_batched - done))
            done += min(chunk, sweeps_batched - done)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["batched"] = {"site_updates_per_s": sites * sweeps_batched / dt, "sweeps": sweeps_batched,
                          "seconds": dt}
        # the other batched engine on the same state, for the record (one call
        # of `chunk` sweeps after an untimed one)
        engine, _ = lat.batch_engine()
        other = 1 - engine
        lat.set_batch_engine(other)
        lat.sweep(chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep(chunk)
        torch.cuda.synchronize()
        dt_other = time.perf_counter() - t0
        out["engines"] = {out["engine"]: out["batched"]["site_updates_per_s"],
                          ("graph", "persistent")[other]: sites * chunk / dt_other,
                          "persistent_grid": lat.batch_engine()[1]}
        lat.set_batch_engine(engine)
        lat.set_mode(swgpu.SW_MODE_PLAIN)
        lat.sweep(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.sweep(sweeps_plain)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["plain"] = {"site_updates_per_s": sites * sweeps_plain / dt, "sweeps": sweeps_plain, "seconds": dt}
    out["batched_over_plain"] = out["batched"]["site_updates_per_s"] / out["plain"]["site_updates_per_s"]
    out["method_bytes_frac_of_hbm_peak"] = (out["batched"]["site_updates_per_s"] * METHOD_BYTES_PER_SITE
                                            / (HBM_PEAK_GBS * 1e9))
    return out


def run_pcc(swgpu, workloads, sweeps: int, replicas: int = 64, trace_every: int = 0):
    """Probability-changing cluster feedback: `replicas` replicas of 2D L=2048, batched."""
    import torch

    wl = workloads.pcc(n=replicas, sweeps=sweeps)
    params = [swgpu.params_from_replica(r) for r in wl.replicas]
    sites = sum(r.nsites for r in wl.replicas)
    stream = torch.cuda.Stream()
    chunk = max(1, min(100, sweeps))        # timed as calls of `chunk` sweeps; the warm-up call builds their graph
    trace = []
    with swgpu.Lattice(params, stream=ctypes.c_void_p(stream.cuda_stream)) as lat:
        lat.set_mode(swgpu.SW_MODE_BATCHED)
        lat.sweep(chunk)
        torch.cuda.synchronize()
        warm = chunk
        t0 = time.perf_counter()
        done = 0
        while done < sweeps:
            lat.sweep(min(chunk, sweeps - done))
            done += min(chunk, sweeps - done)
            if trace_every and (done % trace_every == 0 or done == sweeps):
                torch.cuda.synchronize()
                t_pause = time.perf_counter()
                ps = [lat.state(r)[1] for r in range(len(params))]
                m = sum(ps) / len(ps)
                trace.append({"sweep": warm + done, "p_mean": m,
                              "p_std": (sum((p - m) ** 2 for p in ps) / len(ps)) ** 0.5})
                log(f"pcc: sweep {warm + done}: mean p {m:.5f}")
                t0 += time.perf_counter() - t_pause     # reading p is not part of the timed work
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ps = [lat.state(r)[1] for r in range(len(params))]
    n = len(ps)
    mean = sum(ps) / n
    out = {"workload": wl.name, "replicas": n, "sites": sites, "sweeps_timed": sweeps,
           "sweeps_total": warm + sweeps, "seconds": dt,
           "site_updates_per_s": sites * sweeps / dt, "p_mean": mean,
           "p_std": (sum((p - mean) ** 2 for p in ps) / n) ** 0.5,
           "p_c_fk_2d": 2.0 - 2.0 ** 0.5}
    if trace:
        out["p_trajectory"] = trace
    return out


def run_serving(swgpu, workloads, n_jobs: int, budget_gib: float, slots: int, tick: int, rate: float = 50.0,
                deadline: float = 0.0):
    """Open-loop Poisson job stream (rate jobs/s) through the continuous-batching server.

    With a deadline (seconds of wall time, 0: none), jobs still queued or
    running then are cancelled and the result says so; latencies are then
    those of the jobs that finished."""
    import torch

    jobs = workloads.serving(n_jobs=n_jobs, rate=rate)
    stream = torch.cuda.Stream()
    srv = swgpu.Server(int(budget_gib * (1 << 30)), max_slots=slots, sweeps_per_tick=tick,
                       stream=ctypes.c_void_p(stream.cuda_stream))
    ids = []
    nxt = 0
    wall0 = last_log = time.perf_counter()
    t0 = srv.now()
    while True:
        now = srv.now() - t0
        while nxt < len(jobs) and jobs[nxt].arrival <= now:
            j = jobs[nxt]
            ids.append(srv.submit(swgpu.params_from_replica(j.replica), j.sweeps))
            nxt += 1
        active = srv.step()
        if deadline and time.perf_counter() - wall0 > deadline:
            cut = 0
            for jid in ids:
                if srv.poll(jid) in ("queued", "running"):
                    srv.cancel(jid)
                    cut += 1
            log(f"serving: deadline of {deadline:.0f} s reached, {cut} jobs cancelled, {len(jobs) - nxt} never submitted")
            break
        if time.perf_counter() - last_log > 10.0:
            last_log = time.perf_counter()
            log(f"serving: {nxt} submitted, {srv.stats()['done']} done, {active} queued or running")
        if active == 0:
            if nxt == len(jobs):
                break
            time.sleep(max(0.0, jobs[nxt].arrival - (srv.now() - t0)))
    wall = time.perf_counter() - wall0
    lat = []
    for jid in ids:
        if srv.poll(jid) == "done":
            r = srv.result(jid)
            lat.append(r["t_done"] - r["t_submit"])
    st = srv.stats()
    srv.close()
    lat.sort()

    def pct(q):
        return lat[min(len(lat) - 1, int(q * len(lat)))] if lat else None

    return {"jobs": n_jobs, "of_stream": 2000, "submitted": nxt, "done": st["done"], "rejected": st["rejected"],
            "cancelled_at_deadline": len(ids) - st["done"] - st["rejected"], "deadline_s": deadline or None,
            "rate_per_s": rate,
            "seconds": wall, "site_updates": st["site_updates"], "site_updates_per_s": st["site_updates"] / wall,
            "p50_latency_s": pct(0.5), "p99_latency_s": pct(0.99), "hbm_budget_gib": budget_gib,
            "slots": slots, "sweeps_per_tick": tick}


def run_plain(swgpu, workloads, steps: int, warmup: int, autotune: bool):
    """The plain workload: one sweep of each lattice per step, HIP-event kernel times."""
    import torch

    wl = workloads.plain()
    # one stream per lattice: the two lattices are independent, so their sweeps
    # may overlap on the device (a latency-bound merge of one lattice beside
    # the labelling of the other)
    streams = [torch.cuda.Stream() for _ in wl.replicas]
    lats = [swgpu.Lattice(swgpu.params_from_replica(rep), stream=ctypes.c_void_p(st.cuda_stream))
            for rep, st in zip(wl.replicas, streams)]
    log(f"workload {wl.name}: {[r.nsites for r in wl.replicas]} sites, warmup {warmup}, steps {steps}")
    # warm up first: the autotuner times the tile shapes on a copy of the
    # current (equilibrated) state
    for _ in range(warmup):
        for lat in lats:
            lat.sweep(1)
    torch.cuda.synchronize()
    if autotune:
        for lat in lats:
            lat.autotune(sweeps=3)
    shapes = [swgpu.tile_shapes(r.dim)[lat.tile_shape(0)] for r, lat in zip(wl.replicas, lats)]
    torch.cuda.synchronize()
    # the timed steps: nothing but the sweeps, each lattice on its own stream
    t0 = time.perf_counter()
    for _ in range(steps):
        for lat in lats:
            lat.sweep(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same number of steps again with a HIP event pair around every
    # launch, for the per-kernel durations; here each lattice's sweep waits
    # for the other's to end, so that every event-timed duration is the
    # kernel's own (neither the events nor the waits are in `value`'s pass)
    for lat in lats:
        lat.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for lat, st in zip(lats, streams):
            lat.sweep(1)
            st.synchronize()
    torch.cuda.synchronize()
    dt_events = time.perf_counter() - t0
    timings = [lat.timing() for lat in lats]
    for lat in lats:
        lat.close()
    return wl, shapes, dt, dt_events, timings


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-replica batched workload")
    ap.add_argument("--batched-sweeps", type=int, default=500)
    ap.add_argument("--batched-plain-sweeps", type=int, default=500)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-pcc", action="store_true", help="skip the 64 x 2048^2 PCC feedback workload")
    ap.add_argument("--pcc-sweeps", type=int, default=1000)
    ap.add_argument("--pcc-trace-every", type=int, default=0,
                    help="record the replicas' mean p every this many timed sweeps")
    ap.add_argument("--no-serving", action="store_true", help="skip the Poisson job stream through the server")
    ap.add_argument("--serving-jobs", type=int, default=16)
    ap.add_argument("--serving-budget-gib", type=float, default=200.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-load", type=float, default=None,
                    help="run the same jobs again with arrivals scaled so that the offered load is this "
                         "fraction of the throughput the first (saturated) run measured")
    ap.add_argument("--serving-tick", type=int, default=25)
    ap.add_argument("--serving-rate", type=float, default=50.0, help="Poisson arrival rate of the job stream (jobs/s)")
    ap.add_argument("--serving-deadline", type=float, default=0.0,
                    help="stop the stream after this many seconds (cancel what is left; 0: run to the end)")
    ap.add_argument("--only", choices=["pcc", "serving", "batched"], default=None,
                    help="run only this workload (its JSON object alone)")
    ap.add_argument("--summarize", metavar="PROF_DIR",
                    help="write the profiles/ summaries from rocprofv3 runs under PROF_DIR (no GPU needed)")
    ap.add_argument("--summary-commands", nargs=3, metavar=("TRACE", "PMC", "COPY"), default=("?", "?", "?"))
    ap.add_argument("--sq-commands", nargs=2, metavar=("PASS_A", "PASS_B"), default=None,
                    help="with --summarize: also summarise the SQ counter passes under PROF_DIR/sq_a, sq_b")
    args = ap.parse_args()

    if args.summarize:
        summarize_profiles(args.summarize, os.path.join(ROOT, "profiles"), *args.summary_commands)
        if args.sq_commands:
            summarize_sq(args.summarize, os.path.join(ROOT, "profiles"), *args.sq_commands)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the sweep library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    from paper_0808_2109_amd import workloads

    # the CPU legs run first, before anything touches the GPU (their worker
    # processes are started from a process that has not initialised it)
    cpu = {}
    if not args.no_cpu_baseline and args.only is None and not args.copy_probe:
        log("timing the CPU oracle ...")
        cpu["cpu_baseline"] = cpu_baseline(workloads.plain())
        if not args.no_batched:
            log("timing the CPU oracle on the batched workload, replica-parallel ...")
            cpu["cpu_baseline_batched"] = cpu_baseline_batched(workloads.batched())

    if args.copy_probe:
        copy_probe()
        return

    import torch
    from paper_0808_2109_amd import swgpu

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.only:
        if args.only == "pcc":
            res = run_pcc(swgpu, workloads, args.pcc_sweeps, trace_every=args.pcc_trace_every)
        elif args.only == "batched":
            res = run_batched(swgpu, workloads, args.batched_sweeps, args.batched_plain_sweeps)
        else:
            res = {"serving": run_serving(swgpu, workloads, args.serving_jobs, args.serving_budget_gib,
                                          args.serving_slots, args.serving_tick, rate=args.serving_rate,
                                          deadline=args.serving_deadline)}
            if args.serving_load:
                res["serving_at_load"] = serving_at_load(swgpu, workloads, args, res["serving"])
        print(json.dumps({"only": args.only, **(res if args.only == "serving" else {args.only: res})}), flush=True)
        return

    wl, shapes, dt, dt_events, timings = run_plain(swgpu, workloads, args.steps, args.warmup, not args.no_autotune)
    sites = sum(r.nsites for r in wl.replicas)
    value = sites * args.steps / dt
    log(f"{args.steps} steps in {dt:.4f} s -> {value:.4e} site-updates/s "
        f"({dt_events:.4f} s with an event pair around every launch)")

    # per-kernel mean durations (HIP events around every launch of the second pass)
    kernels = {}
    for rep, tm in zip(wl.replicas, timings):
        tag = f"{rep.dim}d_L{rep.L}"
        for key, (ms, n) in tm.items():
            if n == 0 or key not in ALGO_BYTES_PER_SITE:
                continue
            avg_ms = ms / n
            kernels[f"{key}:{tag}"] = {"kernel": key, "lattice": tag, "sites": rep.nsites, "mean_us": avg_ms * 1e3,
                                       "total_ms": ms, "launches": n}
    dom = max(kernels.values(), key=lambda k: k["total_ms"])
    log("kernels:", json.dumps(kernels, indent=1))
    traffic = traffic_from_profile(f"{dom['kernel']}:{dom['lattice']}", dom["sites"])
    secs = dom["mean_us"] * 1e-6
    achieved = METHOD_BYTES_PER_SITE * dom["sites"] / secs / 1e9
    design = ALGO_BYTES_PER_SITE[dom["kernel"]] * dom["sites"] / secs / 1e9
    roofline = {"bound": "hbm", "kernel": f"{KERNEL_SYMBOLS[dom['kernel']]} ({dom['lattice']})",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "method_bytes_per_site": METHOD_BYTES_PER_SITE, "mean_launch_us": dom["mean_us"],
                "sites_per_launch": dom["sites"],
                "kernel_design_bytes_per_site": ALGO_BYTES_PER_SITE[dom["kernel"]],
                "kernel_design_frac": design / HBM_PEAK_GBS,
                "sweep_method_bytes_frac": value * METHOD_BYTES_PER_SITE / (HBM_PEAK_GBS * 1e9),
                "events_pass_ms_per_step": dt_events / args.steps * 1e3}

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
    if not args.no_batched:
        log("batched workload ...")
        result["batched"] = run_batched(swgpu, workloads, args.batched_sweeps, args.batched_plain_sweeps)
    if not args.no_pcc:
        log("pcc workload ...")
        result["pcc"] = run_pcc(swgpu, workloads, args.pcc_sweeps, trace_every=args.pcc_trace_every)
    if not args.no_serving:
        log("serving workload ...")
        result["serving"] = run_serving(swgpu, workloads, args.serving_jobs, args.serving_budget_gib,
                                        args.serving_slots, args.serving_tick, rate=args.serving_rate,
                                        deadline=args.serving_deadline)
        if args.serving_load:
            result["serving_at_load"] = serving_at_load(swgpu, workloads, args, result["serving"])
    result.update(cpu)
    print(json.dumps(result), flush=True)


def serving_at_load(swgpu, workloads, args, saturated):
    """The same jobs (the generator draws the same numbers at any rate), arrivals
    spaced so that the offered site-updates/s is the asked fraction of the
    capacity the saturated run measured."""
    cap = saturated["site_updates_per_s"]
    jobs = workloads.serving(n_jobs=args.serving_jobs)
    work = sum(j.replica.nsites * j.sweeps for j in jobs) / len(jobs)
    rate = args.serving_load * cap / work
    log(f"serving at {args.serving_load:.0%} of {cap:.3e} site-updates/s: {rate:.3f} jobs/s")
    res = run_serving(swgpu, workloads, args.serving_jobs, args.serving_budget_gib, args.serving_slots,
                      args.serving_tick, rate=rate)
    res.update({"load": args.serving_load, "capacity_site_updates_per_s": cap, "mean_site_updates_per_job": work})
    return res


if __name__ == "__main__":
    main()
