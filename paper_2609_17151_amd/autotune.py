"""Autotuner of the step schedule: particles per thread, threads per
workgroup, the interval of the sort by cell, the interval of the hole
compaction and, for 256-thread tiles of one to four particles per thread in
the general kernel, whether the push workgroups process their own events
(collisions, renewals, secondary emission) instead of the events kernel.

None of the choices it makes changes the results: the deposit sums are
exact integers, the random draws are keyed by particle id and step, and the
compaction keeps the canonical order.  Sorting permutes the particles, which
the physics does not see as long as nothing is born: births take their ids
in the order of their parents, so after a sort they would draw other random
numbers.  The sort is therefore a candidate only where no particle can be
born (the streaming kernel: periodic, no collisions).  The tuner times the
candidates on the live run itself (every timed step is a real step of the
simulation), keeps the fastest, and remembers the choice in a JSON cache
keyed by the shape of the workload.
"""
from __future__ import annotations

import json
import os

STREAMING = [(ppt, thr) for ppt, thr in ((4, 1024), (4, 512), (4, 256), (8, 256), (2, 256), (1, 256))]
GENERAL = [(4, 1024), (8, 512), (4, 512), (8, 256), (4, 256), (2, 256), (1, 256)]
SORT_EVERY = (0, 32, 16)
# intervals that divide the 32-step chunk a captured graph replays
COMPACT_EVERY = (16, 32, 8)
# a compaction interval is accepted only if the slots in use (live particles,
# holes and the births of the interval) stay below this share of the capacity
HEADROOM = 0.9


def signature(sim):
    """Workload key: discharges, species, boundary, mesh and particle count
    (to the nearest power of two), and whether the general kernel runs."""
    cfg = sim.cfgs[0]
    n = sum(sum(sim.counts(b)["count"]) for b in range(sim.B))
    general = any(c["bc"] == 1 or c["gas_density"] > 0.0 for c in sim.cfgs)
    cells = max(c["n_cells"] for c in sim.cfgs)
    return "B%d-S%d-bc%d-cells%d-n2^%d-%s" % (sim.B, sim.S, cfg["bc"], cells, max(n, 1).bit_length(),
                                              "general" if general else "streaming")


def candidates(general):
    shapes = GENERAL if general else STREAMING
    out = []
    for ppt, thr in shapes:
        for srt in (SORT_EVERY if not general else (0,)):
            for cmp_ in (COMPACT_EVERY if general else (16,)):
                for fuse in ((0, 1) if general and thr == 256 and ppt <= 4 else (0,)):
                    out.append(dict(ppt=ppt, threads=thr, sort_every=srt, compact_every=cmp_, fuse=fuse))
    return out


def apply(sim, c):
    """Apply a schedule (a candidate or a cached choice)."""
    sim.config_tiles(c["ppt"], c["threads"], c["sort_every"], c["compact_every"])
    sim.config_events(bool(c.get("fuse", 0)))


def birth_rate(sim, steps=4):
    """Births per step of every discharge and species, from the growth of
    the id counters over `steps` real steps: {(b, s): rate}."""
    before = {b: sim.counts(b)["next_id"] for b in range(sim.B)}
    sim.step(steps)
    out = {}
    for b in range(sim.B):
        after = sim.counts(b)["next_id"]
        for s in range(sim.S):
            out[(b, s)] = max(0, after[s] - before[b][s]) / steps
    return out


def fits(sim, compact_every, rate):
    """Whether holes and births can pile up for `compact_every` steps: for
    every discharge and species, the slots in use plus the interval's births
    at twice the measured rate stay within HEADROOM of the capacity."""
    for b in range(sim.B):
        if b in getattr(sim, "retired", ()):
            continue
        c0 = sim.counts(b)
        for s in range(sim.S):
            cap = sim.cfgs[b]["species"][s]["capacity"]
            if c0["count"][s] + 2.0 * rate[(b, s)] * compact_every > HEADROOM * cap:
                return False
    return True


def _time_steps(sim, n):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(n)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def tune(sim, steps=64, warm=32, cache=None, timer=None, verbose=False):
    """Pick the fastest schedule for `sim`'s workload, apply it and return
    (choice, table of ms per step).  With a cache file, a known workload is
    applied without timing.  `timer(sim, n)` returns ms per step over n steps
    (default: HIP events on the context's stream)."""
    timer = timer or _time_steps
    key = signature(sim)
    store = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            store = json.load(f)
        if key in store:
            c = store[key]["choice"]
            apply(sim, c)
            return c, store[key]["table"]
    general = key.endswith("general")
    rate = birth_rate(sim) if general else None
    cands = candidates(general)
    if general:
        ok = [c for c in cands if fits(sim, c["compact_every"], rate)]
        # no interval leaves the headroom (a discharge near its capacity):
        # the most frequent compaction is the least bad
        cands = ok or [c for c in cands if c["compact_every"] == min(COMPACT_EVERY)]
    table = []
    for c in cands:
        apply(sim, c)
        if warm:
            sim.step(warm)
        ms = timer(sim, steps)
        table.append(dict(c, ms_per_step=ms))
        if verbose:
            print("autotune", key, c, "%.4f ms/step" % ms, flush=True)
    best = min(table, key=lambda r: r["ms_per_step"])
    choice = {k: best[k] for k in ("ppt", "threads", "sort_every", "compact_every", "fuse")}
    apply(sim, choice)
    if cache:
        store[key] = dict(choice=choice, table=table)
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(store, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return choice, table
