"""The E x B electron cyclotron drift instability box (Section 3.6): a
periodic azimuthal box of a whole number of resonant wavelengths
lambda_1 = 2 pi v_E / omega_ce, the paper's reference fields and density,
axial renewal after a virtual transit L_z, and the space-time spectrum of
the ion density.  The cyclotron resonance puts the dominant mode at the
box's number of resonant wavelengths.

    python -m paper_2609_17151_amd.ecdi --us 3 --every 128 --out ecdi.npz

Prints progress lines and one JSON line: the dominant mode and wavelength
over the last half of the record, and the run's wall time and rate.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

import workloads as W

from . import spectrum


def main(argv=None):
    ap = argparse.ArgumentParser(prog="ecdi")
    ap.add_argument("--us", type=float, default=3.0, help="simulated time, microseconds")
    ap.add_argument("--every", type=int, default=128, help="steps between density samples")
    ap.add_argument("--lambdas", type=int, default=15)
    ap.add_argument("--n", type=int, default=4_000_000, help="macro-particles per species")
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--density", type=float, default=1e17)
    ap.add_argument("--b", type=float, default=0.02)
    ap.add_argument("--lz", type=float, default=0.01)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    from . import Sim
    cfg = W.ecdi(n_lambda=a.lambdas, n_cells=a.cells, n_per_species=a.n, density=a.density, b_field=a.b,
                 lz=a.lz)
    sim = Sim(cfg)
    dt = cfg["dt"]
    count = max(2, int(round(a.us * 1e-6 / (dt * a.every))))
    t0 = time.time()
    last = [t0]

    def progress(i):
        now = time.time()
        if now - last[0] > 20.0:
            last[0] = now
            print("ecdi sample %d/%d t=%.3f us %.0f s" % (i + 1, count, (i + 1) * a.every * dt * 1e6, now - t0),
                  flush=True)

    hist = spectrum.record(sim, 1, a.every, count, progress=progress)
    sim.sync()
    wall = time.time() - t0
    half = hist[count // 2:]
    m, lam = spectrum.dominant_mode(half, cfg["length"], a.every * dt)
    # dominant mode of each tenth of the record: growth and saturation
    tenths = [spectrum.dominant_mode(hist[i * count // 10:(i + 1) * count // 10], cfg["length"])[0]
              for i in range(10)]
    amp = [float(np.std(hist[i * count // 10:(i + 1) * count // 10]) / np.mean(hist)) for i in range(10)]
    steps = count * a.every
    n_tot = sum(sim.counts()["count"])
    out = dict(metric="ecdi_dominant_mode", lambdas=a.lambdas, dominant_mode=m, wavelength_m=lam,
               lambda1_m=W.lambda1(b_field=a.b), mode_by_tenth=tenths, rel_fluct_by_tenth=amp,
               renewed=[int(v) for v in sim.renewed()], simulated_us=steps * dt * 1e6, steps=steps,
               wall_s=wall, particle_steps_per_s=n_tot * steps / wall)
    np.savez(a.out, ion_density=hist.astype(np.float32), length=cfg["length"], dt_sample=a.every * dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
