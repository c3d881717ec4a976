"""Swarm mode (Section 4): electrons in a gas under a uniform field, with no
Poisson solve and no ions, give the transport and rate coefficients of the
gas as functions of E/N; the error bars come from independent replicas.

Each (E/N, replica) pair is one discharge of a single context: electrons
only, periodic, field_solve = 0, the field imposed along x.  Ionization
adds electrons (the ion is not followed); when a replica has grown past
`control` times its initial count it is thinned back to about that count on
the device (pic_thin: each electron kept with the same probability, by a
Philox draw keyed by its id and the step; the order of the survivors is
kept), which leaves every per-electron average unchanged.

Coefficients over a sampling window that follows a relaxation:
  * flux drift velocity W = <v_x> along the electrons' drift (-E direction);
  * mean energy <eps> (eV);
  * rate coefficient of each process k_j = C_j / (N_gas integral N dt), C_j
    the real collisions of process j, N the electrons present;
  * the energy distribution of the electrons (every cell is bulk in a
    periodic box), normalised to unit area in eV.
Diffusion coefficients are not measured: a 1D3V swarm keeps no transverse
position, and the periodic box wraps the longitudinal one.
"""
from __future__ import annotations

import math

import numpy as np

import workloads as W

from . import EEPF_BINS

TD = 1e-21          # 1 Townsend in V m^2


def electron_tables(tables):
    """The processes of species 0 (electrons) of a set of tables."""
    return [dict(t) for t in tables if t["species"] == 0]


def numax_estimate(tables, n_gas):
    """Largest total collision frequency n_g sum_j sigma_j v over the table
    energies (the library adds its own margin)."""
    e = np.unique(np.concatenate([np.asarray(t["energy"], np.float64) for t in tables]))
    tot = np.zeros_like(e)
    for t in tables:
        s = np.interp(np.log(e), np.log(t["energy"]), t["sigma"])
        s[e < t["threshold"]] = 0.0
        tot += s
    v = np.sqrt(2.0 * e * W.E_CHARGE / W.M_ELECTRON)
    return float(np.max(n_gas * tot * v))


def config(e_over_n_td, n_gas, n, dt, seed, te_ev=1.0, capacity=None, gas_mass=W.AR_MASS, gas_temp=300.0):
    """One swarm replica: electrons only, the field E = (E/N) N_gas along +x."""
    vte = math.sqrt(te_ev * W.E_CHARGE / W.M_ELECTRON)
    cap = capacity if capacity else 4 * n
    el = W.species(-W.E_CHARGE, W.M_ELECTRON, 1.0, n, vte, capacity=cap, load=W.LOAD_RANDOM)
    e_field = e_over_n_td * TD * n_gas
    return W.base_config(n_cells=16, bc=0, field_solve=0, length=1.0, dt=dt, eps0=W.EPS0, e_unit=W.E_CHARGE,
                         e_ext=[e_field, 0.0, 0.0], gas_density=n_gas, gas_temp=gas_temp, gas_mass=gas_mass,
                         seed=seed, species=[el])


class Swarm:
    """Replicas of electron swarms at several E/N in one context."""

    def __init__(self, e_over_n_td, replicas=8, n=100_000, tables=None, n_gas=3.22e22, dt=None, seed=1,
                 nu_dt=0.05, te_ev=1.0, control=2.0, gas_mass=W.AR_MASS, gas_temp=300.0, stream=None):
        from . import Sim
        self.tables = electron_tables(tables if tables is not None else W.argon_tables())
        self.en = [float(x) for x in e_over_n_td]
        self.R = int(replicas)
        self.n0 = int(n)
        self.n_gas = float(n_gas)
        self.dt = dt if dt else nu_dt / numax_estimate(self.tables, n_gas)
        self.control = float(control)
        self.cfgs = [config(en, n_gas, n, self.dt, seed + 1000 * i + r, te_ev=te_ev,
                            capacity=int(math.ceil(control * n * 4)) + 4096, gas_mass=gas_mass,
                            gas_temp=gas_temp)
                     for i, en in enumerate(self.en) for r in range(self.R)]
        self.sim = Sim(self.cfgs, self.tables, stream=stream)
        self.B = len(self.cfgs)
        self.thinned = 0                # thinning rounds (every replica at once)

    def _thin(self):
        """Thin every replica that has outgrown control x its initial count
        back to about that count, on the device, with no host round trip."""
        self.sim.thin(0, int(self.control * self.n0), self.n0)
        self.thinned += 1

    def run(self, relax_steps, sample_steps, every=128, eepf_emax=40.0, progress=None):
        """Relax, then sample; returns a dict of per-(E/N) means and errors
        (standard error over replicas) and the per-replica values.  Replicas
        are thinned every `every` steps: at 1000 Td in argon the population
        doubles in about 250 steps, and the store holds 4 x control x the
        initial count."""
        sim = self.sim
        chunks = max(1, relax_steps // every)
        for i in range(chunks):
            sim.step(every)
            self._thin()
            if progress:
                progress("relax", i + 1, chunks)
        sim.set_diag(True, eepf_emax)
        for b in range(self.B):
            sim.reset_avg(b)
        c0 = [sim.coll(b) for b in range(self.B)]
        n_dt = np.zeros(self.B)
        chunks = max(1, sample_steps // every)
        for i in range(chunks):
            n_before = np.array([sim.counts(b)["count"][0] for b in range(self.B)], np.float64)
            sim.step(every)
            n_after = np.array([sim.counts(b)["count"][0] for b in range(self.B)], np.float64)
            # electrons present over the chunk: geometric mean of its ends
            n_dt += np.sqrt(n_before * n_after) * every * self.dt
            self._thin()
            if progress:
                progress("sample", i + 1, chunks)
        nch = len(self.tables)
        per = dict(W=np.zeros(self.B), energy=np.zeros(self.B), rates=np.zeros((self.B, nch)),
                   eepf=np.zeros((self.B, EEPF_BINS)))
        for b in range(self.B):
            a = sim.avg(b)
            pw = sim.power(b)
            n = a["density"][0]
            ex = self.cfgs[b]["e_ext"][0]
            # flux over density; the electrons drift against E
            per["W"][b] = -np.sign(ex) * np.sum(pw["flux"][0]) / np.sum(n)
            per["energy"][b] = np.sum(n * a["mean_energy"]) / np.sum(n)
            c1 = sim.coll(b)
            dc = np.array(c1["coll"][0][:nch], np.float64) - np.array(c0[b]["coll"][0][:nch], np.float64)
            per["rates"][b] = dc / (self.n_gas * n_dt[b])
            h = sim.eepf(b)
            tot = h["bulk"].sum()
            per["eepf"][b] = h["bulk"] / (tot * h["bin_width"]) if tot > 0 else 0.0
        out = dict(e_over_n_td=np.array(self.en), dt=self.dt, replicas=self.R, thinned=self.thinned,
                   per_replica=per, kinds=[t["kind"] for t in self.tables])
        for k in ("W", "energy", "rates", "eepf"):
            v = per[k].reshape((len(self.en), self.R) + per[k].shape[1:])
            out[k] = v.mean(axis=1)
            out[k + "_err"] = v.std(axis=1, ddof=1) / math.sqrt(self.R) if self.R > 1 else np.zeros_like(out[k])
        return out



def main(argv=None):
    """python -m paper_2609_17151_amd.swarm --en 50,100,300,1000 --out swarm.npz"""
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser(prog="swarm")
    ap.add_argument("--en", default="50,100,200,500,1000", help="E/N values in Td")
    ap.add_argument("--replicas", type=int, default=8)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--relax", type=int, default=65536)
    ap.add_argument("--sample", type=int, default=32768)
    ap.add_argument("--every", type=int, default=128)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    en = [float(x) for x in a.en.split(",")]
    t0 = time.time()
    sw = Swarm(en, replicas=a.replicas, n=a.n)
    last = [t0]

    def progress(stage, i, n):
        if time.time() - last[0] > 20.0:
            last[0] = time.time()
            print("swarm %s %d/%d %.0f s" % (stage, i, n, last[0] - t0), flush=True)

    out = sw.run(a.relax, a.sample, every=a.every, progress=progress)
    sw.sim.sync()
    wall = time.time() - t0
    np.savez(a.out, **{k: np.asarray(v) for k, v in out.items() if k != "per_replica"})
    rows = [dict(e_over_n_td=en[i], W=float(out["W"][i]), W_err=float(out["W_err"][i]),
                 energy_eV=float(out["energy"][i]), energy_err=float(out["energy_err"][i]),
                 rates=[float(x) for x in out["rates"][i]], rates_err=[float(x) for x in out["rates_err"][i]])
            for i in range(len(en))]
    print(json.dumps(dict(metric="swarm_coefficients", kinds=out["kinds"], dt=out["dt"], replicas=a.replicas,
                          electrons_per_replica=a.n, thinned=out["thinned"], wall_s=wall, rows=rows)), flush=True)


if __name__ == "__main__":
    main()
