"""Wall time per converged discharge: the plain method against batched sweeps
started from the learned warm start.

    python -m paper_2609_17151_amd.experiments plain   --out c2.npz
    python -m paper_2609_17151_amd.experiments sweep   --set train --start 0 --count 64 --out t0.npz
    python -m paper_2609_17151_amd.experiments train   --data t0.npz t1.npz ... --out model.npz
    python -m paper_2609_17151_amd.experiments sweep   --set heldout --out cold.npz
    python -m paper_2609_17151_amd.experiments warm    --model model.npz --cold cold.npz --out warm.npz
    python -m paper_2609_17151_amd.experiments plainset --cold cold.npz --warm warm.npz --out plain.npz

Converged (steady): the 5-period windows stay within 2 % (relative L2, each
of n_e, n_i, <eps> at 256 points; or three times the windows' own scatter
when that is larger) of the reference, the mean of the last 50 periods of
the cold run, for 10 windows in a row; the convergence time is the end of
the first of those windows.  Every run prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as W

from . import steady, warm
from .sweep import Sweep

# Warm-start draws over 10-50 MHz: below about 9 MHz most cold starts of
# these discharges die out (no steady discharge to learn) and a period costs
# up to 10^4 steps.
WARM_F = (10e6, 50e6)
SETS = {
    "c4": lambda: W.sweep_draws(64, seed=4),
    "train": lambda: W.warm_draws(2048, seed=5, f_range=WARM_F),
    "heldout": lambda: W.warm_draws(64, seed=6, f_range=WARM_F),
}


def _sim(cfgs):
    from . import Sim
    return Sim(cfgs, W.argon_tables())


def weight_of(draw, a):
    """Particles per macro: the pilot weight times --weight-scale, and with
    --weight-law f2 also times (f / 13.56 MHz)^2, so that draws whose density
    grows with the square of the frequency keep comparable particle counts."""
    w = W.PILOT_WEIGHT * a.weight_scale
    if a.weight_law == "f2":
        w *= (draw.get("freq", 13.56e6) / 13.56e6) ** 2
    return w


def convergence(windows, ref, tol=steady.TOL, window_periods=5):
    """(first converged window, periods to convergence) or (None, None)."""
    i = steady.converged_at(windows, ref, tol=tol)
    return (None, None) if i is None else (i, (i + 1) * window_periods)


def _tuning(a):
    """--tune: the autotuner picks each batch's step schedule first (its
    choices cached in --tune-cache, keyed by the workload's shape)."""
    return dict(tune=a.tune, tune_cache=a.tune_cache)


def cold_tolerance(windows, ref):
    """2 % or three times the scatter of the reference windows."""
    return steady.noise_tolerance([steady.distance(w, ref) for w in windows])


def cmd_plain(a):
    """One cold discharge (the 2.5 cm, 30 mTorr, 200 V, 13.56 MHz case) for
    `periods` RF periods."""
    draw = dict(pressure_mtorr=30.0, v_amp=200.0, freq=13.56e6, gap=0.025, n_cells=400, see_gamma=0.1)
    cfg = warm.config(draw, weight=weight_of(draw, a), seed=2)
    sim = _sim([cfg])
    sw = Sweep(sim, [warm.steps_per_period(draw)], max_periods=a.periods, **_tuning(a)).run()
    ref = sw.reference(0)
    tol = cold_tolerance(sw.windows[0], ref)
    i, per = convergence(sw.windows[0], ref, tol)
    t_conv = sw.window_time[0][i] if i is not None else None
    out = dict(kind="plain", periods=a.periods, counts=sim.counts(0)["count"], tolerance=tol,
               converged_window=i, converged_periods=per, seconds_to_converge=t_conv,
               seconds_total=sw.window_time[0][-1], steps=sw.window_step[0][-1],
               us_per_step=sw.window_time[0][-1] / sw.window_step[0][-1] * 1e6)
    np.savez(a.out, dist=np.array([steady.distance(w, ref) for w in sw.windows[0]]), ref=ref,
             times=np.array(sw.window_time[0]), steps=np.array(sw.window_step[0]), x=warm.inputs(draw))
    print(json.dumps(out), flush=True)


def cmd_sweep(a):
    """Cold runs of a set of draws, in batches of up to `batch` discharges
    grouped by frequency; windows, references and timings per draw."""
    every = SETS[a.set]()
    pick = [int(i) for i in a.ids.split(",")] if a.ids else list(range(a.start, min(a.start + a.count, len(every))))
    draws = [every[i] for i in pick]
    order = sorted(range(len(draws)), key=lambda i: -draws[i].get("freq", 13.56e6))
    X, REF, DIST, TIMES, STEPS, CONV, CNT, TOL, FLG = [], [], [], [], [], [], [], [], []
    ids = []
    total = 0.0

    def save():
        # compact: the reference and each window's distance to it, not the windows
        nw = max(len(t) for t in TIMES)
        pad = lambda rows: np.array([np.pad(np.asarray(r, dtype=np.float64), (0, nw - len(r)),
                                            constant_values=np.nan) for r in rows])
        np.savez(a.out, ids=np.array(ids), x=np.array(X), y=np.array(REF), dist=pad(DIST), times=pad(TIMES),
                 steps=pad(STEPS), conv=np.array(CONV), counts=np.array(CNT), tol=np.array(TOL),
                 flags=np.array(FLG))

    for k in range(0, len(order), a.batch):
        grp = order[k:k + a.batch]
        cfgs = [warm.config(draws[i], weight=weight_of(draws[i], a), seed=1000 + pick[i],
                            capacity=a.capacity) for i in grp]
        sim = _sim(cfgs)
        t0 = time.perf_counter()
        sw = Sweep(sim, [warm.steps_per_period(draws[i]) for i in grp], max_periods=a.periods,
                   **_tuning(a)).run()
        total += time.perf_counter() - t0
        for j, i in enumerate(grp):
            ref = sw.reference(j)
            ids.append(pick[i])
            X.append(warm.inputs(draws[i]))
            REF.append(steady.to_features(ref))
            DIST.append([steady.distance(w, ref) for w in sw.windows[j]])
            TIMES.append(sw.window_time[j])
            STEPS.append(sw.window_step[j])
            TOL.append(steady.noise_tolerance(DIST[-1]))
            CONV.append(convergence(sw.windows[j], ref, TOL[-1])[1] or -1)
            CNT.append(sim.counts(j)["count"])
            FLG.append(sw.flags[j])
        cnt = [sim.counts(j)["count"] for j in range(len(grp))]
        flags = [sw.flags[j] for j in range(len(grp))]
        print(json.dumps(dict(batch=k // a.batch, discharges=len(grp), seconds=time.perf_counter() - t0,
                              flags=sorted(set(flags)), min_count=int(np.min(cnt)), max_count=int(np.max(cnt)),
                              total=int(np.sum(cnt)), schedule=sw.schedule)), flush=True)
        sim.close()
        save()
    print(json.dumps(dict(kind="sweep", set=a.set, draws=len(draws), seconds=total,
                          converged=int(np.sum(np.array(CONV) > 0)),
                          mean_periods_to_converge=float(np.mean([c for c in CONV if c > 0])) if any(
                              c > 0 for c in CONV) else None)), flush=True)


def cmd_train(a):
    """Train on the references of the sustained discharges (a discharge that
    died out, or stopped early on a device flag, has no steady profile to
    learn)."""
    X, Y = [], []
    for f in a.data:
        d = np.load(f)
        alive = np.array([s["alive"] for s in cold_summary(d)], dtype=bool)
        X.append(d["x"][alive])
        Y.append(d["y"][alive])
    X, Y = np.concatenate(X), np.concatenate(Y)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(X))
    nv = max(1, len(X) // 10)
    va, tr = perm[:nv], perm[nv:]
    t0 = time.perf_counter()
    m = warm.Model().fit(X[tr], Y[tr], steps=a.steps, lr=a.lr, batch=a.batch)
    secs = time.perf_counter() - t0
    st = m.state()
    np.savez(a.out, **st, history=np.array(m.history))
    print(json.dumps(dict(kind="train", samples=len(tr), validation=len(va), steps=a.steps, seconds=secs,
                          train_loss=m.loss(X[tr], Y[tr]), validation_loss=m.loss(X[va], Y[va]))), flush=True)


def cold_summary(cold):
    """Per cold draw: tolerance, periods to convergence and whether the
    discharge survived (from the stored distances and counts).  A discharge
    that stopped before the others (a device flag latched, e.g. its particle
    store filled up) has no valid reference and counts as not alive."""
    out = []
    full = max(int(np.sum(np.isfinite(cold["dist"][k]))) for k in range(len(cold["ids"])))
    for k in range(len(cold["ids"])):
        d = cold["dist"][k]
        d = d[np.isfinite(d)]
        tol = steady.noise_tolerance(d)
        ok = [x <= tol for x in d]
        i = next((j for j in range(len(ok) - steady.NRUN + 1) if all(ok[j:j + steady.NRUN])), None)
        alive = int(cold["counts"][k][0]) > 0 and int(cold["counts"][k][1]) > 0 and len(d) == full
        if "flags" in cold.files:
            alive = alive and int(cold["flags"][k]) == 0
        t = cold["times"][k]
        out.append(dict(tol=tol, periods=(i + 1) * 5 if i is not None else None, alive=alive,
                        steps=int(cold["steps"][k][i]) if i is not None else None,
                        batch_seconds=float(t[i]) if i is not None else None))
    return out


def cmd_warm(a):
    """Held-out draws started from the network, run together until each has
    converged to its cold run's reference (then retired)."""
    cold = np.load(a.cold)
    summ = cold_summary(cold)
    st = np.load(a.model)
    draws = SETS["heldout"]()
    keep = [k for k in range(len(cold["ids"])) if summ[k]["alive"]]
    ids = [int(cold["ids"][k]) for k in keep]
    ref_prof = [steady.from_features(cold["y"][k]) for k in keep]
    tols = [summ[k]["tol"] for k in keep]
    t0 = time.perf_counter()
    m = warm.Model(widths=tuple(int(w) for w in st["widths"]))
    m.set_state(st)
    feats = m.predict(np.array([warm.inputs(draws[i]) for i in ids]))
    cfgs = [warm.config(draws[i], weight=weight_of(draws[i], a), seed=1000 + i, capacity=a.capacity,
                        cold=False) for i in ids]
    sim = _sim(cfgs)
    for j in range(len(ids)):
        warm.start_from_features(sim, j, cfgs[j], feats[j])
    sim.sync()
    t_ready = time.perf_counter() - t0

    def stop(j, sw):
        return steady.converged_at(sw.windows[j], ref_prof[j], tol=tols[j]) is not None

    sw = Sweep(sim, [warm.steps_per_period(draws[i]) for i in ids], max_periods=a.periods,
               **_tuning(a)).run(stop=stop)
    conv, t_conv, steps_conv = [], [], []
    for j in range(len(ids)):
        i, per = convergence(sw.windows[j], ref_prof[j], tols[j])
        conv.append(per if per is not None else -1)
        t_conv.append(t_ready + sw.window_time[j][i] if i is not None else None)
        steps_conv.append(sw.window_step[j][i] if i is not None else None)
    done = [t for t in t_conv if t is not None]
    cold_periods = [summ[k]["periods"] for k in keep]
    out = dict(kind="warm", draws=len(ids), seconds_inference_and_load=t_ready, converged=len(done),
               schedule=sw.schedule, schedules=sw.schedules,
               seconds_to_last_convergence=max(done) if done else None,
               seconds_per_converged_discharge=(max(done) / len(ids)) if len(done) == len(ids) else None,
               mean_periods_warm=float(np.mean([c for c in conv if c > 0])) if done else None,
               median_periods_warm=float(np.median([c for c in conv if c > 0])) if done else None,
               mean_periods_cold=float(np.mean([c for c in cold_periods if c])),
               median_periods_cold=float(np.median([c for c in cold_periods if c])),
               first_window_distance_median=float(np.median(
                   [steady.distance(sw.windows[j][0], ref_prof[j]) for j in range(len(ids))])))
    np.savez(a.out, ids=np.array(ids), conv=np.array(conv),
             cold_conv=np.array([c if c else -1 for c in cold_periods]), tol=np.array(tols),
             t_conv=np.array([t if t is not None else -1.0 for t in t_conv]),
             steps_conv=np.array([s if s is not None else -1 for s in steps_conv]),
             dist0=np.array([steady.distance(sw.windows[j][0], ref_prof[j]) for j in range(len(ids))]))
    print(json.dumps(out), flush=True)


def cmd_plainset(a):
    """The plain method for the held-out draws: each draw alone in its own
    context (one discharge, cold start, the seed of its cold batched run, so
    the same discharge), stepped until it has converged to its cold run's
    reference under the same rule, or for --periods; the wall time of each.
    With --warm, only the draws that converged warm (the comparison's set)."""
    cold = np.load(a.cold)
    summ = cold_summary(cold)
    draws = SETS["heldout"]()
    keep = [k for k in range(len(cold["ids"])) if summ[k]["alive"]]
    if a.warm:
        w = np.load(a.warm)
        done = {int(i) for i, c in zip(w["ids"], w["conv"]) if c > 0}
        keep = [k for k in keep if int(cold["ids"][k]) in done]
    if a.ids:
        only = {int(i) for i in a.ids.split(",")}
        keep = [k for k in keep if int(cold["ids"][k]) in only]
    keep = keep[a.first:a.first + a.count] if a.count else keep[a.first:]
    ids, secs, per, steps = [], [], [], []
    for k in keep:
        i = int(cold["ids"][k])
        ref = steady.from_features(cold["y"][k])
        tol = summ[k]["tol"]
        cfg = warm.config(draws[i], weight=weight_of(draws[i], a), seed=1000 + i, capacity=a.capacity)
        sim = _sim([cfg])
        t0 = time.perf_counter()

        def stop(j, sw):
            return steady.converged_at(sw.windows[j], ref, tol=tol) is not None

        sw = Sweep(sim, [warm.steps_per_period(draws[i])], max_periods=a.periods, progress=0.0,
                   **_tuning(a)).run(stop=stop)
        wall = time.perf_counter() - t0
        c, p_ = convergence(sw.windows[0], ref, tol)
        ids.append(i)
        per.append(p_ if p_ is not None else -1)
        secs.append(sw.window_time[0][c] if c is not None else -1.0)
        steps.append(sw.window_step[0][c] if c is not None else -1)
        print(json.dumps(dict(draw=i, periods=per[-1], cold_periods=summ[k]["periods"], seconds=secs[-1],
                              wall=wall, counts=sim.counts(0)["count"])), flush=True)
        sim.close()
        np.savez(a.out, ids=np.array(ids), periods=np.array(per), seconds=np.array(secs), steps=np.array(steps))
    done = [s for s in secs if s > 0]
    print(json.dumps(dict(kind="plainset", draws=len(ids), converged=len(done), seconds=float(np.sum(done)),
                          seconds_per_converged_discharge=float(np.mean(done)) if done else None)), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="experiments")
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("plain")
    p.add_argument("--periods", type=int, default=300)
    p.add_argument("--weight-scale", type=float, default=1.0)
    p.add_argument("--weight-law", choices=["fixed", "f2"], default="fixed")
    p.add_argument("--out", required=True)
    p = sub.add_parser("sweep")
    p.add_argument("--set", choices=sorted(SETS), required=True)
    p.add_argument("--start", type=int, default=0)
    p.add_argument("--count", type=int, default=64)
    p.add_argument("--ids", default=None, help="comma-separated draw indices (instead of --start/--count)")
    p.add_argument("--batch", type=int, default=64)
    p.add_argument("--periods", type=int, default=300)
    p.add_argument("--weight-scale", type=float, default=1.0)
    p.add_argument("--weight-law", choices=["fixed", "f2"], default="fixed")
    p.add_argument("--capacity", type=int, default=1 << 20)
    p.add_argument("--out", required=True)
    p = sub.add_parser("train")
    p.add_argument("--data", nargs="+", required=True)
    p.add_argument("--steps", type=int, default=4000)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--batch", type=int, default=128)
    p.add_argument("--out", required=True)
    p = sub.add_parser("warm")
    p.add_argument("--model", required=True)
    p.add_argument("--cold", required=True)
    p.add_argument("--periods", type=int, default=300)
    p.add_argument("--weight-scale", type=float, default=1.0)
    p.add_argument("--weight-law", choices=["fixed", "f2"], default="fixed")
    p.add_argument("--capacity", type=int, default=1 << 20)
    p.add_argument("--out", required=True)
    p = sub.add_parser("plainset")
    p.add_argument("--cold", required=True)
    p.add_argument("--warm", default=None)
    p.add_argument("--ids", default=None, help="comma-separated draw indices (a subset of the kept draws)")
    p.add_argument("--first", type=int, default=0)
    p.add_argument("--count", type=int, default=0)
    p.add_argument("--periods", type=int, default=1200)
    p.add_argument("--weight-scale", type=float, default=1.0)
    p.add_argument("--weight-law", choices=["fixed", "f2"], default="fixed")
    p.add_argument("--capacity", type=int, default=1 << 20)
    p.add_argument("--out", required=True)
    for name in ("plain", "sweep", "warm", "plainset"):
        p = sub.choices[name]
        p.add_argument("--tune", action="store_true", help="autotune each batch's step schedule first")
        p.add_argument("--tune-cache", default=None, help="JSON cache of the autotuner's choices")
    a = ap.parse_args(argv)
    dict(plain=cmd_plain, sweep=cmd_sweep, train=cmd_train, warm=cmd_warm, plainset=cmd_plainset)[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
