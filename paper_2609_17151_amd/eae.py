"""The electrical asymmetry effect (Section 3.3): a geometrically symmetric
argon discharge driven through a blocking capacitor by
V(t) = V0 [cos(2 pi f t + theta) + cos(4 pi f t)] develops a DC self-bias
that the phase theta alone controls.  Since V(t; 90 deg) = -V(t - T/4; 0),
the discharge at 90 degrees is the mirror image of the one at 0 degrees and
its self-bias is the opposite; the ion flux-energy distributions at the two
electrodes exchange.

    python -m paper_2609_17151_amd.eae --periods 1500 --out eae.npz

Both phases run as one batch.  Prints progress and one JSON line: the
self-bias (time mean of the driven electrode's potential) of each phase over
blocks of periods, and the mean and peak ion energies at both electrodes
over the last block.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import workloads as W


def config(theta, gap=0.067, n_cells=600, pressure_mtorr=20.0, v0=315.0, freq=13.56e6, cap=1e-8, weight=8e8,
           n_init=100_000, capacity=4_000_000, seed=31):
    cfg = W.argon_rf(gap=gap, n_cells=n_cells, pressure_mtorr=pressure_mtorr, v_amp=v0, n_init=n_init,
                     weight=weight, capacity=capacity, seed=seed)
    cfg.update(v_phase=theta, v_freq=freq, waveform=W.WAVE_TWO_HARMONIC, drive=W.DRIVE_CAPACITOR, cap=cap)
    return cfg


def main(argv=None):
    ap = argparse.ArgumentParser(prog="eae")
    ap.add_argument("--periods", type=int, default=1500)
    ap.add_argument("--block", type=int, default=100, help="periods per self-bias block")
    ap.add_argument("--weight", type=float, default=8e8)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    from . import Sim
    cfgs = [config(0.0, weight=a.weight), config(0.5 * math.pi, weight=a.weight)]
    sim = Sim(cfgs, W.argon_tables())
    spp = int(round(1.0 / (cfgs[0]["v_freq"] * cfgs[0]["dt"])))
    sim.set_diag(True, 40.0)
    sim.set_wall_edf(1, 600.0)
    t0 = time.time()
    blocks = []
    for blk in range(a.periods // a.block):
        for b in range(2):
            sim.reset_avg(b)
        sim.step(spp * a.block)
        eta = [float(sim.avg(b)["phi"][0]) for b in range(2)]
        n = [sum(sim.counts(b)["count"]) for b in range(2)]
        blocks.append(dict(periods=(blk + 1) * a.block, self_bias=eta, particles=n, flags=[sim.flags(b) for b in range(2)]))
        print("eae periods %d self-bias %.1f V / %.1f V particles %s %.0f s" %
              ((blk + 1) * a.block, eta[0], eta[1], n, time.time() - t0), flush=True)
    edf = [sim.wall_edf(b) for b in range(2)]
    ions = []
    for b in range(2):
        h, wdt = edf[b]["counts"][1], edf[b]["bin_width"][1]
        e = (np.arange(h.shape[1]) + 0.5) * wdt
        row = []
        for wall in range(2):
            c = h[wall]
            tot = c.sum()
            peak = float(e[np.nonzero(c)[0].max()]) if tot else 0.0
            row.append(dict(mean_eV=float((c * e).sum() / tot) if tot else 0.0, max_eV=peak, count=float(tot)))
        ions.append(row)
    np.savez(a.out, ion_edf=np.array([edf[b]["counts"][1] for b in range(2)]), bin_width=edf[0]["bin_width"][1],
             self_bias=np.array([blk["self_bias"] for blk in blocks]))
    last = blocks[-1]["self_bias"]
    print(json.dumps(dict(metric="eae_self_bias", theta_deg=[0, 90], self_bias_V=last,
                          asymmetry=(last[0] + last[1]) / (abs(last[0]) + abs(last[1]) + 1e-300),
                          ion_energy_powered_grounded=ions, blocks=blocks, steps_per_period=spp,
                          wall_s=time.time() - t0)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
