"""Throughput of the MI355X PIC-MCC step.

One step = one pass of the whole hot path over every particle: gather, Boris
push, move, boundary handling, collisions, compaction/births, deposition,
and the field solve.  Default workload: the E x B drift-instability box
(4e6 electrons + 4e6 xenon ions, 1024 cells, periodic, B = 0.02 T,
E = 2e4 V/m), particles resident in HBM before timing starts.  Prints one
JSON line.
"""
import argparse
import json
import os
import re
import sys
import time
import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PARTICLE_STEP = 40      # read cell, off, vx, vy, vz; write the same (no draws: no id)
PUSH_SOURCES = ("pic_push.hip", "pic_device.h", "pic_internal.h")
COUNTERS = os.path.join(ROOT, "profiles", "push_kernel_exb_counters.txt")
STATS = os.path.join(ROOT, "profiles", "push_kernel_exb_stats.txt")
PUSH_KERNEL = "push_kernel<4, 1024, false, false>"


_TOKENS = re.compile(r'"(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\'|//[^\n]*|/\*.*?\*/', re.S)


def code_only(text):
    """C++ source without its comments, trailing blanks and empty lines:
    what a kernel is compiled from (string and character literals kept)."""
    text = _TOKENS.sub(lambda m: m.group(0) if m.group(0)[0] in "\"'" else " ", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def push_source_hash():
    """SHA-256 over the code (comments and layout aside) of the sources the
    push kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in PUSH_SOURCES:
        with open(os.path.join(ROOT, "paper_2609_17151_amd", "csrc", name)) as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per push launch from the committed FETCH_SIZE / WRITE_SIZE
    counter summary, each scaled by the factor a plain copy of known size
    gives; None when the summary is absent or the kernel has changed since."""
    try:
        kv = {}
        with open(COUNTERS) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != push_source_hash():
            return None
        fetch = float(kv["push_fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["push_write_kib_per_dispatch"]) * float(kv["write_scale"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def rocprof_push_us():
    """Average duration (us) of the E x B push in the committed rocprofv3
    kernel statistics, and the file; None when the summary is absent or the
    kernel has changed since it was taken."""
    try:
        avg = None
        sha = None
        with open(STATS) as f:
            for line in f:
                if line.startswith("kernel_source_sha256:"):
                    sha = line.split(":", 1)[1].strip()
                elif PUSH_KERNEL in line:
                    avg = float(line.split(")", 1)[1].split()[1])
        if sha != push_source_hash() or avg is None:
            return None
        return avg
    except (OSError, ValueError, IndexError):
        return None


def c5_summary():
    """The second half of the metric, wall time per converged discharge (plain
    against batched and warm-started), from its committed summary: those runs
    take about an hour of GPU time, so this bench does not repeat them."""
    try:
        with open(os.path.join(ROOT, "profiles", "c5_wall_time_summary.json")) as f:
            s = json.load(f)
        keys = ("draws", "plain_s_per_converged_discharge", "cold_batched_s_per_converged_discharge",
                "batched_warm_s_per_converged_discharge", "median_periods_to_converge_warm",
                "median_periods_to_converge_cold")
        out = {k: s[k] for k in keys}
        out.update(source=s["commands_and_results"], measured_in_this_run=False)
        return out
    except (OSError, KeyError, ValueError):
        return None


def rocprof_entry(per_launch_bytes):
    """The same roofline figure from the committed rocprofv3 statistics."""
    us = rocprof_push_us()
    if us is None:
        return None
    gbs = per_launch_bytes / (us * 1e-6) / 1e9
    return {"file": os.path.relpath(STATS, ROOT), "avg_launch_ms": us * 1e-3, "achieved": gbs,
            "frac": gbs / HBM_PEAK_GBS}


def host_threads():
    """Threads the host gives this process (its CPU affinity), for the oracle."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(cfg, steps, steps_one):
    """The FP64 oracle on the host: its parallel step (OpenMP, fixed chunks of
    particles, the same result for every thread count) on every thread the
    host gives, and its sequential step on one."""
    import oracle
    n = sum(sp["n_init"] for sp in cfg["species"])
    threads = host_threads()
    t0 = time.perf_counter()
    o = oracle.Oracle(cfg)
    t1 = time.perf_counter()
    o.set_threads(threads)
    o.step(steps)
    t2 = time.perf_counter()
    o.set_threads(0)
    o.step(steps_one)
    t3 = time.perf_counter()
    return dict(value=n * steps / (t2 - t1), unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"full E x B box ({n} particles): {steps} steps of the parallel FP64 C oracle on "
                       f"{threads} threads, then {steps_one} steps of its sequential step on one "
                       f"(load {t1 - t0:.1f} s not counted)",
                single_thread=n * steps_one / (t3 - t2),
                cpu=cpu_model(), host_cores=os.cpu_count())


def cpu_model():
    """The host CPU's model name (Linux), for the CPU baseline's record."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def timed_rate(sim, torch, steps):
    """particle-steps/s and us per step over `steps` steps (particles counted
    before and after, averaged), whether captured graphs ran them, and the
    per-kernel launch times of as many profiled steps after them"""
    sim.step(64)
    sim.sync()
    count = lambda: sum(sum(sim.counts(b)["count"]) for b in range(sim.B))
    n0 = count()
    g0 = sim.graphs()["steps"]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    graph_steps = sim.graphs()["steps"] - g0
    n = 0.5 * (n0 + count())
    sim.profile(True)
    sim.step(steps)
    t = sim.timing()
    sim.profile(False)
    per = lambda k: 1e3 * t[k + "_ms"] / max(t[k + "_n"], 1.0)
    return dict(particle_steps_per_s=n * steps / (ms * 1e-3), us_per_step=ms / steps * 1e3, particles=int(n),
                graph_steps=graph_steps,
                kernel_us={"push": per("push"), "events": per("events"), "finalize": per("finalize")})


def tuned(sim, tune):
    """The autotuner's schedule for the workload (timed on the live run), a
    given one ("ppt,threads,compact_every,events_in_push"), or the default
    one; returns what ran: the choice and each candidate's time."""
    if isinstance(tune, str):
        ppt, thr, cmp_, fuse = (int(v) for v in tune.split(","))
        sim.config_tiles(ppt, thr, 0, cmp_)
        sim.config_events(bool(fuse))
        return dict(choice=dict(ppt=ppt, threads=thr, sort_every=0, compact_every=cmp_, fuse=fuse))
    if not tune:
        return dict(choice="default")
    from paper_2609_17151_amd import autotune
    choice, table = autotune.tune(sim, steps=32, warm=16)
    return dict(choice=choice, us_per_step={"%d/%d/%d/%d" % (r["ppt"], r["threads"], r["compact_every"], r["fuse"]):
                                            round(1e3 * r["ms_per_step"], 2) for r in table})


def sweep_counts(W, sweep_particles=0):
    """The 64-discharge sweep's macro-particles per species and their
    weights: the steady-state counts at the pilot weight, or those counts
    scaled to `sweep_particles` in all (both species; at least 1000 each)
    with each weight scaled by the inverse of its count's factor, so that
    every discharge keeps its densities."""
    counts0 = W.steady_counts(64)
    counts = counts0
    if sweep_particles:
        counts = np.maximum(1000, np.rint(counts0 * (sweep_particles / (2.0 * counts0.sum())))).astype(int)
    return counts, W.PILOT_WEIGHT * counts0 / counts


def secondary(P, W, torch, steps, only=None, warm=3200, graphs=True, tune=True, sweep_particles=0):
    """The bounded, colliding path at steady-state counts: one argon RF
    discharge (2.5 cm, 30 mTorr, 200 V, 13.56 MHz, 1600 steps per period,
    2e5 macro-particles per species) and the sweep of 64 such discharges
    (10-200 mTorr, 100-400 V, 1.5-4 cm; 5e4-2e6 per species, seeded) in one
    batched step.  Each discharge starts from a half-sine density at those
    counts (electrons 3 eV, ions at the gas temperature) and runs `warm`
    steps before it is timed; with `tune` the autotuner then picks the step
    schedule (tile shape and compaction interval) on the live run.  With
    `sweep_particles` the sweep's counts are scaled to that total (both
    species), keeping their log-uniform spread, and each discharge's
    macro-particle weight by the inverse of its own factor, so that its
    densities, and so its state, are those of the unscaled sweep."""
    out = {}
    dens, temp = W.discharge_profile()
    if only in (None, "argon_rf"):
        n = W.STEADY_COUNT_C2
        sim = P.Sim(W.argon_rf(capacity=4 * n), W.argon_tables())
        sim.use_graphs(graphs)
        sim.load_profiles(dens, temp, [n, n])
        sim.step(warm)
        sched = tuned(sim, tune)
        out["argon_rf_single"] = dict(timed_rate(sim, torch, steps), schedule=sched)
        sim.close()
    if only not in (None, "argon_sweep"):
        return out
    draws = W.sweep_draws(64, seed=4)
    counts, weights = sweep_counts(W, sweep_particles)
    cfgs = [W.argon_rf(gap=d["gap"], n_cells=d["n_cells"], pressure_mtorr=d["pressure_mtorr"], v_amp=d["v_amp"],
                       seed=1000 + i, capacity=4 * int(counts[i]) + 65536, weight=float(weights[i]))
            for i, d in enumerate(draws)]
    sim = P.Sim(cfgs, W.argon_tables())
    sim.use_graphs(graphs)
    for b in range(64):
        sim.load_profiles(dens, temp, [counts[b], counts[b]], batch=b)
    sim.step(warm)
    sched = tuned(sim, tune)
    out["argon_rf_batched_64"] = dict(timed_rate(sim, torch, steps), schedule=sched)
    sim.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    # the GPU's clocks settle over the first ~1000 steps (~0.1 s); warm up past that
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--ppt", type=int, default=4)
    ap.add_argument("--threads", type=int, default=1024)
    ap.add_argument("--sort-every", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the argon RF single and batched lines")
    ap.add_argument("--secondary-steps", type=int, default=320)
    ap.add_argument("--secondary-warm", type=int, default=3200, help="steps before the argon lines are timed")
    ap.add_argument("--cpu-steps", type=int, default=400, help="oracle steps on all host threads")
    ap.add_argument("--cpu-steps-one", type=int, default=60, help="oracle steps of the sequential step")
    ap.add_argument("--no-graph", action="store_true", help="direct launches (counter runs)")
    ap.add_argument("--no-tune", action="store_true", help="argon lines: the default schedule, no autotuning")
    ap.add_argument("--schedule", default=None, metavar="PPT,THREADS,COMPACT,FUSE",
                    help="argon_rf / argon_sweep: this schedule instead of autotuning (counter runs)")
    ap.add_argument("--sweep-particles", type=float, default=0.0,
                    help="argon_sweep: scale the 64 discharges' counts to this total (both species), their weights inversely")
    ap.add_argument("--workload", choices=["exb", "argon_rf", "argon_sweep"], default="exb",
                    help="argon_rf / argon_sweep: only that secondary workload (profiling runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n * 4, "reads_bytes": n * 4, "writes_bytes": n * 4}))
        return
    if args.gpus != 1:
        print("bench.py: the step runs on one GPU; --gpus must be 1 (the design for more GPUs is described, not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    import paper_2609_17151_amd as P

    torch.cuda.set_device(0)
    if args.workload != "exb":
        r = secondary(P, W, torch, args.secondary_steps, only=args.workload, warm=args.secondary_warm,
                      graphs=not args.no_graph, tune=args.schedule or not args.no_tune,
                      sweep_particles=args.sweep_particles)
        print(json.dumps(dict(workload=args.workload, **r[next(iter(r))])), flush=True)
        return
    cfg = W.exb()
    n = sum(sp["n_init"] for sp in cfg["species"])
    sim = P.Sim(cfg)
    sim.config_tiles(args.ppt, args.threads, args.sort_every)
    if args.no_graph:
        sim.use_graphs(False)
    sim.step(args.warmup)
    sim.sync()
    stream = sim.stream
    torch.cuda.synchronize()
    # timed region: the step loop replayed from captured HIP graphs
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    g0 = sim.graphs()["steps"]
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    torch.cuda.synchronize()
    sim.sync()
    ms = start.elapsed_time(end)
    graph_steps = sim.graphs()["steps"] - g0     # steps of the timed region run from captured graphs
    # the same number of steps again with an event pair around every kernel
    # launch (direct launches) for the per-kernel durations
    sim.profile(True)
    sim.step(args.steps)
    sim.sync()
    tm = sim.timing()
    sim.profile(False)
    ms_step = ms / args.steps
    value = n * args.steps / (ms * 1e-3)
    push_avg_ms = tm["push_ms"] / max(tm["push_n"], 1.0)
    per_launch_bytes = n * BYTES_PER_PARTICLE_STEP        # one launch moves every species
    achieved = per_launch_bytes / (push_avg_ms * 1e-3) / 1e9
    out = {
        "metric": "particle-steps/s",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "exb_drift_box: 4e6 e- + 4e6 Xe+, 1024 cells, periodic, "
                               "B=0.02 T, E=2e4 V/m, dt=5e-12 s",
                   "particles": n, "cells": cfg["n_cells"], "particles_per_thread": args.ppt, "threads_per_group": args.threads,
                   "sort_every": args.sort_every, "graphs": graph_steps > 0,
                   "graph_steps": graph_steps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "push_kernel", "avg_launch_ms": push_avg_ms,
                     "bytes_per_particle_step": BYTES_PER_PARTICLE_STEP,
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "rocprof": rocprof_entry(per_launch_bytes)},
        "breakdown_ms_per_step": {"push": tm["push_ms"] / args.steps,
                                  "finalize": float(tm["finalize_ms"]) / args.steps,
                                  "finalize_avg_launch_ms": float(tm["finalize_ms"] / max(tm["finalize_n"], 1))},
    }
    if not args.no_secondary:
        sim.close()
        out["secondary"] = secondary(P, W, torch, args.secondary_steps, warm=args.secondary_warm,
                                     graphs=not args.no_graph, tune=not args.no_tune)
    if not args.no_cpu:
        sim.close()
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps, args.cpu_steps_one)
    out["wall_time_per_converged_discharge"] = c5_summary()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
