"""Precision accounting: the error of each reported GPU result against the FP64
oracle (the GPU keeps particle state and the push in FP32 relative to the
cell, with FP64 only in the field solve, the density, energy and charge sums
and the time averages).

    python tests/precision_report.py [--quick]

prints one JSON line per quantity and a closing summary line.  Quantities:
  * one step of the full E x B box (8e6 particles): positions (in cells) and
    velocities (relative) from identical states;
  * the E x B box over 200 steps: mean drift velocity of each species and the
    kinetic energies, GPU against oracle (statistics of chaotic runs);
  * the Langmuir wave over 1000 steps: total-energy drift of each side, and
    the measured frequency against the kinetic root;
  * densities and charge of an argon RF state, and the charge balance;
  * the warm-start network: BF16 outputs and gradients against FP64;
  * swarm coefficients (Section 4): drift velocity, mean energy and rate
    coefficients from the same procedure (replicas with the same seeds,
    relaxation, sampling, thinning) on both sides, in combined standard
    errors over the replicas;
  * the electrical asymmetry effect (Section 3.3): from the GPU's state after
    a relaxation, both sides run the same RF periods; the self-bias of each
    phase and the mean ion impact energy at each electrode;
  * the electron cyclotron drift instability (Section 3.6): from the GPU's
    state during the growth, both sides run the same steps; the ion-density
    amplitude of the resonant mode and the dominant mode, and the field
    energy.

Statistical parity of time-averaged profiles at the argon RF configuration's
steady state and of sampled discharges of a batched sweep is a test of its
own (tests/test_gpu_steady_parity.py).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle                                   # noqa: E402
import workloads as W                           # noqa: E402
from gpu_helpers import to_oracle               # noqa: E402
from paper_2609_17151_amd import MLP, Sim       # noqa: E402


def emit(name, **kw):
    print(json.dumps(dict(quantity=name, **kw)), flush=True)


def exb_single_step(n_per_species):
    cfg = W.exb(n_per_species=n_per_species)
    sim = Sim(cfg)
    sim.step(5)
    o = to_oracle(sim, cfg)
    sim.step(1)
    o.step(1)
    dx = cfg["length"] / cfg["n_cells"]
    L = cfg["length"]
    for s, name in ((0, "electrons"), (1, "ions")):
        pg, po = sim.get_particles(s), o.get_particles(s)
        xg = (pg["cell"] + pg["off"].astype(np.float64)) * dx
        d = np.abs(xg - po["x"])
        d = np.minimum(d, L - d)
        dv = np.sqrt((pg["vx"] - po["vx"]) ** 2 + (pg["vy"] - po["vy"]) ** 2 + (pg["vz"] - po["vz"]) ** 2)
        v = np.sqrt(po["vx"] ** 2 + po["vy"] ** 2 + po["vz"] ** 2)
        vref = np.maximum(v, cfg["species"][s]["vth"])
        emit("exb_one_step_" + name, particles=int(len(xg)), max_dx_cells=float(d.max() / dx),
             rms_dx_cells=float(np.sqrt(np.mean((d / dx) ** 2))), max_rel_v=float(np.max(dv / vref)),
             rms_rel_v=float(np.sqrt(np.mean((dv / vref) ** 2))), bar="1e-6")
    dg, do = sim.density(), [o.density(s) for s in range(2)]
    emit("exb_one_step_density", max_rel=float(max(np.max(np.abs(dg[s] - do[s])) / np.max(do[s]) for s in range(2))),
         bar="1e-5")


def exb_run(n_per_species, steps):
    cfg = W.exb(n_per_species=n_per_species)
    sim = Sim(cfg)
    sim.set_diag(True)
    o = oracle.Oracle(cfg)
    sim.step(steps)
    o.step(steps)
    out = {}
    for s, name in ((0, "electrons"), (1, "ions")):
        pg, po = sim.get_particles(s), o.get_particles(s)
        mg, mo = float(np.mean(pg["vx"])), float(np.mean(po["vx"]))
        sd = float(np.std(po["vx"]) / math.sqrt(len(po["vx"])))
        out[name] = dict(mean_vx_gpu=mg, mean_vx_oracle=mo, diff_in_standard_errors=abs(mg - mo) / max(sd, 1e-300))
    keg, _ = sim.energy()
    keo, _ = o.energy()
    emit("exb_%d_steps" % steps, particles_per_species=n_per_species, **out,
         kinetic_energy_rel=[float(abs(a - b) / b) for a, b in zip(keg, keo)])


def langmuir_energy(steps):
    cfg = W.langmuir()
    sim = Sim(cfg)
    sim.set_diag(True)
    o = oracle.Oracle(cfg)
    eg, eo = [], []
    for _ in range(steps // 10):
        sim.step(10)
        o.step(10)
        kg, fg = sim.energy()
        ko, fo = o.energy()
        eg.append((float(sum(kg)), fg))
        eo.append((float(sum(ko)), fo))
    tg = np.array([a + b for a, b in eg])
    to = np.array([a + b for a, b in eo])
    fe_g = np.array([b for _, b in eg])
    fe_o = np.array([b for _, b in eo])
    emit("langmuir_total_energy", steps=steps, drift_gpu=float(np.max(np.abs(tg - tg[0])) / tg[0]),
         drift_oracle=float(np.max(np.abs(to - to[0])) / to[0]),
         field_energy_rel_rms=float(np.sqrt(np.mean((fe_g - fe_o) ** 2)) / np.sqrt(np.mean(fe_o ** 2))))


def argon_state():
    cfg, tabs = W.argon_rf(n_init=20000, capacity=200000), W.argon_tables()
    sim = Sim(cfg, tabs)
    sim.step(1600)
    o = to_oracle(sim, cfg, tabs)
    dg = sim.density()
    do = [o.density(s) for s in range(2)]
    q, qp = sim.charge()
    emit("argon_densities", max_rel=float(max(np.max(np.abs(dg[s] - do[s])) / np.max(do[s]) for s in range(2))),
         charge_balance_rel=float(abs(q - qp) / max(abs(qp), 1e-300)), bar="1e-5")


def network():
    from oracle import mlp as ref
    widths = W.WARM_WIDTHS
    p = W.mlp_init(widths, seed=11) + 0.01
    x, t = W.mlp_batch(256, widths[0], widths[-1], seed=12)
    net = MLP(widths, 256)
    net.set_params(p)
    y = net.forward(x).cpu().numpy()
    y_ref, _ = ref.forward(p.astype(np.float32).astype(np.float64), widths, x.astype(np.float32))
    loss, g = net.grad(x, t)
    loss_ref, g_ref = ref.loss_and_grad(p.astype(np.float32).astype(np.float64), widths, x.astype(np.float32),
                                        t.astype(np.float32))
    emit("network_bf16", output_rel_l2=float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)),
         loss_rel=float(abs(loss - loss_ref) / loss_ref),
         gradient_rel_l2=float(np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)),
         gradient_cosine=float(np.dot(g, g_ref) / (np.linalg.norm(g) * np.linalg.norm(g_ref))), bar="2e-2")


def _threads(fns):
    """Run oracle calls side by side (the C library runs without the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(len(fns)) as ex:
        return list(ex.map(lambda f: f(), fns))


def _host_threads():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _se_diff(g, o):
    """Difference of the replica means of g and o [replicas] in combined
    standard errors, and relative to the oracle's mean."""
    g, o = np.asarray(g, np.float64), np.asarray(o, np.float64)
    se = math.sqrt(g.var(ddof=1) / len(g) + o.var(ddof=1) / len(o))
    d = float(g.mean() - o.mean())
    return dict(gpu=float(g.mean()), oracle=float(o.mean()), diff_in_standard_errors=abs(d) / max(se, 1e-300),
                rel=abs(d) / max(abs(float(o.mean())), 1e-300))


def swarm_vs_oracle(en=(100.0, 500.0), replicas=4, n=20000, relax=8192, sample=8192, every=128):
    from paper_2609_17151_amd import swarm as SW
    sw = SW.Swarm(en, replicas=replicas, n=n)
    g = sw.run(relax, sample, every=every)
    nch = len(sw.tables)
    threads = max(1, _host_threads() // sw.B)

    def one(b):
        cfg = sw.cfgs[b]
        o = oracle.Oracle(cfg, sw.tables)
        o.set_threads(threads)
        rng = np.random.default_rng(7000 + b)

        def count():
            return len(o.get_particles(0)["id"])

        def thin():
            p = o.get_particles(0)
            if len(p["id"]) <= sw.control * n:
                return
            keep = np.sort(rng.choice(len(p["id"]), n, replace=False))
            o.set_particles(0, p["x"][keep], p["vx"][keep], p["vy"][keep], p["vz"][keep], p["id"][keep],
                            p["next_id"])

        for _ in range(max(1, relax // every)):
            o.step(every)
            thin()
        o.set_diag(True, 40.0)
        o.reset_avg()
        c0 = o.counters()["coll"][0][:nch].astype(np.float64)
        n_dt = 0.0
        for _ in range(max(1, sample // every)):
            nb = count()
            o.step(every)
            n_dt += math.sqrt(nb * count()) * every * sw.dt
            thin()
        a = o.avg()
        dens = a["density"][0]
        ex = cfg["e_ext"][0]
        W_ = -np.sign(ex) * np.sum(o.power(0)["flux"]) / np.sum(dens)
        eps = np.sum(dens * a["mean_energy"]) / np.sum(dens)
        rates = (o.counters()["coll"][0][:nch].astype(np.float64) - c0) / (sw.n_gas * n_dt)
        return W_, eps, rates

    res = _threads([lambda b=b: one(b) for b in range(sw.B)])
    per = g["per_replica"]
    for i, e in enumerate(en):
        bs = range(i * replicas, (i + 1) * replicas)
        row = dict(e_over_n_td=e, replicas=replicas, electrons=n, relax_steps=relax, sample_steps=sample,
                   W=_se_diff([per["W"][b] for b in bs], [res[b][0] for b in bs]),
                   mean_energy=_se_diff([per["energy"][b] for b in bs], [res[b][1] for b in bs]))
        for j, kind in enumerate(g["kinds"]):
            og = [res[b][2][j] for b in bs]
            if max(og) > 0.0:
                row["k_%s" % kind] = _se_diff([per["rates"][b][j] for b in bs], og)
        emit("swarm_coefficients", **row, bar="statistics")


def eae_vs_oracle(relax_periods=200, periods=3, weight=8e8):
    from paper_2609_17151_amd import eae
    cfgs = [eae.config(0.0, weight=weight), eae.config(0.5 * math.pi, weight=weight)]
    tabs = W.argon_tables()
    sim = Sim(cfgs, tabs)
    spp = int(round(1.0 / (cfgs[0]["v_freq"] * cfgs[0]["dt"])))
    sim.step(spp * relax_periods)
    orcs = []
    for b in range(2):
        o = to_oracle(sim, cfgs[b], tabs, batch=b)
        o.set_circuit(sim.circuit(b)[1])
        o.refresh_field()
        o.set_diag(True, 40.0)
        o.set_wall_edf(1, 600.0)
        o.set_threads(max(1, _host_threads() // 2))
        orcs.append(o)
    sim.set_diag(True, 40.0)
    sim.set_wall_edf(1, 600.0)
    counts = [sum(sim.counts(b)["count"]) for b in range(2)]

    def ion_means(edf):
        h, wdt = edf["counts"][1], edf["bin_width"][1]
        e = (np.arange(h.shape[1]) + 0.5) * wdt
        return [float((h[w] * e).sum() / max(h[w].sum(), 1.0)) for w in range(2)]

    bias_g, ion_g = [[], []], [[], []]
    for _ in range(periods):
        for b in range(2):
            sim.reset_avg(b)
        sim.step(spp)
        for b in range(2):
            bias_g[b].append(float(sim.avg(b)["phi"][0]))
            ion_g[b].append(ion_means(sim.wall_edf(b)))

    def run(o):
        bias, ion = [], []
        for _ in range(periods):
            o.reset_avg()
            o.step(spp)
            bias.append(float(o.avg()["phi"][0]))
            ion.append(ion_means(o.wall_edf()))
        return bias, ion

    res = _threads([lambda o=o: run(o) for o in orcs])
    for b, theta in enumerate((0, 90)):
        bo, io = res[b]
        ig, io_ = np.array(ion_g[b]), np.array(io)
        emit("eae_self_bias", theta_deg=theta, relax_periods=relax_periods, periods=periods,
             particles=int(counts[b]), self_bias=_se_diff(bias_g[b], bo),
             ion_mean_energy_powered=_se_diff(ig[:, 0], io_[:, 0]),
             ion_mean_energy_grounded=_se_diff(ig[:, 1], io_[:, 1]), bar="statistics")


def ecdi_vs_oracle(n=1_000_000, relax_us=0.8, chunks=8, every=500):
    cfg = W.ecdi(n_per_species=n)
    sim = Sim(cfg)
    sim.step(int(round(relax_us * 1e-6 / cfg["dt"])))
    o = to_oracle(sim, cfg)
    for s in range(2):
        o.set_axial(s, sim.axial(s))
    o.refresh_field()
    o.set_threads(_host_threads())
    m = 15                                  # the box holds 15 resonant wavelengths

    def modes(d):
        # amplitude of each spatial mode of the periodic density, over its mean
        return np.abs(np.fft.rfft(d - d.mean())) / (len(d) * d.mean())

    rows = []
    for k in range(chunks):
        sim.step(every)
        o.step(every)
        ag, ao = modes(sim.density()[1]), modes(o.density(1))
        _, feg = sim.energy()
        _, feo = o.energy()
        rows.append(dict(steps=(k + 1) * every, mode_gpu=int(np.argmax(ag[1:]) + 1),
                         mode_oracle=int(np.argmax(ao[1:]) + 1), amp_gpu=float(ag[m]), amp_oracle=float(ao[m]),
                         field_energy_rel=float(abs(feg - feo) / max(feo, 1e-300))))
    emit("ecdi_growth", particles_per_species=n, relax_us=relax_us, resonant_mode=m,
         amp_rel_max=max(abs(r["amp_gpu"] - r["amp_oracle"]) / r["amp_oracle"] for r in rows),
         field_energy_rel_max=max(r["field_energy_rel"] for r in rows), rows=rows, bar="statistics")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller E x B runs")
    ap.add_argument("--only", default=None,
                    help="comma-separated subset of exb,langmuir,argon,network,swarm,eae,ecdi")
    a = ap.parse_args(argv)
    want = set(a.only.split(",")) if a.only else None
    on = lambda k: want is None or k in want
    n = 500_000 if a.quick else 4_000_000
    if on("exb"):
        exb_single_step(n)
        exb_run(200_000 if a.quick else 1_000_000, 200)
    if on("langmuir"):
        langmuir_energy(1000)
    if on("argon"):
        argon_state()
    if on("network"):
        network()
    if on("swarm"):
        swarm_vs_oracle()
    if on("eae"):
        eae_vs_oracle()
    if on("ecdi"):
        ecdi_vs_oracle()
    emit("done")


if __name__ == "__main__":
    main()
