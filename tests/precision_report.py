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
  * the warm-start network: BF16 outputs and gradients against FP64.
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller E x B runs")
    a = ap.parse_args(argv)
    n = 500_000 if a.quick else 4_000_000
    exb_single_step(n)
    exb_run(200_000 if a.quick else 1_000_000, 200)
    langmuir_energy(1000)
    argon_state()
    network()
    emit("done")


if __name__ == "__main__":
    main()
