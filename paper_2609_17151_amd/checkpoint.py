"""Checkpoint files: save a context's physical state to disk and resume it,
here or on another machine (Section 1: runs can be stopped and continued).

What a step needs is the particles in canonical order (cell, offset,
velocities, ids), each species' next id, the step index, the configuration
and the cross-section tables.  Random draws are keyed by (seed, id, step) and
the deposit sums are exact integers, so a run resumed from a checkpoint
continues bit for bit as the uninterrupted run would (the field is recomputed
from the particles and equals the one the run held).  With axial renewal
the axial displacements are kept too, and with an external circuit the
charge of the driven electrode's conductor.  Not kept: counters, time averages
and distributions (they restart from zero), the diagnostic and tile
settings, and graphs.  All discharges of a context share one step index
on resume; a retired discharge is restored retired.

Format: one ``.npz`` file (numpy arrays only, readable with
``allow_pickle=False``): ``format``, ``configs`` and ``tables`` as JSON
strings, ``steps`` [B], ``next_id`` [B, S], ``retired`` [B], the table
arrays ``t{i}_energy`` / ``t{i}_sigma``, and per discharge and species
``b{b}_s{s}_{cell,off,vx,vy,vz,id}`` (and ``b{b}_s{s}_z`` with renewal),
``circuit`` [B] (NaN where the electrode is driven by a voltage).
"""
from __future__ import annotations

import json
import os

import numpy as np

FORMAT = "pic-mi355x-checkpoint-1"
FIELDS = ("cell", "off", "vx", "vy", "vz", "id")


def _has_circuit(cfg):
    return cfg["bc"] == 1 and cfg["field_solve"] and cfg.get("drive", 0) != 0


def save(sim, path):
    """Write the state of every discharge of `sim` to `path` (.npz).  Waits for
    queued work; compacts the particle store first (order unchanged)."""
    B, S = sim.B, sim.S
    arrays = {}
    steps = np.zeros(B, np.int64)
    next_id = np.zeros((B, S), np.int64)
    for b in range(B):
        steps[b] = sim.counts(b)["step"]
        for s in range(S):
            p = sim.get_particles(s, b)
            next_id[b, s] = p["next_id"]
            for k in FIELDS:
                arrays["b%d_s%d_%s" % (b, s, k)] = p[k]
            if sim.cfgs[b].get("renew_lz", 0.0) > 0.0:
                arrays["b%d_s%d_z" % (b, s)] = sim.axial(s, b)
    live = [b for b in range(B) if b not in sim.retired]
    if len({int(steps[b]) for b in live}) > 1:
        raise ValueError("discharges at different steps cannot share one resumed step index")
    tabs = []
    for i, t in enumerate(sim.tables):
        tabs.append(dict(species=t["species"], kind=t["kind"], threshold=t["threshold"], batch=t.get("batch", -1)))
        arrays["t%d_energy" % i] = np.asarray(t["energy"], np.float64)
        arrays["t%d_sigma" % i] = np.asarray(t["sigma"], np.float64)
    arrays["format"] = np.array(FORMAT)
    arrays["configs"] = np.array(json.dumps(sim.cfgs))
    arrays["tables"] = np.array(json.dumps(tabs))
    arrays["steps"] = steps
    arrays["next_id"] = next_id
    arrays["retired"] = np.array([b in sim.retired for b in range(B)])
    arrays["circuit"] = np.array([sim.circuit(b)[1] if _has_circuit(sim.cfgs[b]) else np.nan for b in range(B)])
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def read(path):
    """The checkpoint's contents as plain Python and numpy objects."""
    with np.load(path, allow_pickle=False) as z:
        if str(z["format"]) != FORMAT:
            raise ValueError("%s is not a checkpoint of this library (format %r)" % (path, str(z["format"])))
        cfgs = json.loads(str(z["configs"]))
        tabs = json.loads(str(z["tables"]))
        for i, t in enumerate(tabs):
            t["energy"] = z["t%d_energy" % i]
            t["sigma"] = z["t%d_sigma" % i]
        B, S = len(cfgs), len(cfgs[0]["species"])
        parts = [[{k: z[f] for k in FIELDS + ("z",) for f in ["b%d_s%d_%s" % (b, s, k)] if f in z.files}
                  for s in range(S)] for b in range(B)]
        circ = z["circuit"].copy() if "circuit" in z.files else np.full(B, np.nan)
        return dict(configs=cfgs, tables=tabs, steps=z["steps"].copy(), next_id=z["next_id"].copy(),
                    retired=z["retired"].copy(), particles=parts, circuit=circ)


def load(path, stream=None, make_sim=None):
    """A new context holding the checkpoint's state, ready to step.  The
    context is created with no particles loaded, then every species of every
    discharge is set (which re-deposits the charge and re-solves the field at
    the saved step)."""
    c = read(path)
    cfgs = []
    for cfg in c["configs"]:
        cfg = json.loads(json.dumps(cfg))
        for sp in cfg["species"]:
            sp["load"] = 2                   # PIC_LOAD_NONE: the particles come from the file
        cfgs.append(cfg)
    if make_sim is None:
        from . import Sim

        def make_sim(cfgs, tables):
            return Sim(cfgs, tables, stream=stream)
    sim = make_sim(cfgs, c["tables"])
    live = [b for b in range(len(cfgs)) if not c["retired"][b]]
    step = int(c["steps"][live[0]]) if live else int(c["steps"][0])
    for b in range(len(cfgs)):
        for s in range(len(cfgs[b]["species"])):
            p = c["particles"][b][s]
            sim.set_particles(s, p["cell"], p["off"], p["vx"], p["vy"], p["vz"], p["id"],
                              int(c["next_id"][b, s]), step, batch=b)
            if "z" in p:
                sim.set_axial(s, p["z"], batch=b)
    for b in range(len(cfgs)):
        if np.isfinite(c["circuit"][b]):
            sim.set_circuit(float(c["circuit"][b]), batch=b)
        if c["retired"][b]:
            sim.retire(b)
    # the saved configurations (with their load modes) stay the context's record
    sim.cfgs = c["configs"]
    return sim
