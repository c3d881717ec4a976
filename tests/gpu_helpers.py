"""Shared helpers of the GPU parity tests: move a GPU state into the oracle and
compare states element by element."""
import numpy as np

import oracle
import workloads as W


def dx_of(cfg):
    return cfg["length"] / cfg["n_cells"]


def gpu_positions(p, cfg):
    """FP64 positions of GPU particles: x = (cell + off) dx."""
    return (p["cell"].astype(np.float64) + p["off"].astype(np.float64)) * dx_of(cfg)


def to_oracle(sim, cfg, tables=(), batch=0):
    """An oracle holding exactly the GPU's current state (positions from
    (cell, off), FP32 velocities widened to FP64, ids, next ids, step)."""
    o = oracle.Oracle(cfg, tables, load=False)
    c = sim.counts(batch)
    for s in range(len(cfg["species"])):
        p = sim.get_particles(s, batch)
        x = gpu_positions(p, cfg)
        x = np.where(x >= cfg["length"], x - cfg["length"], x)
        o.set_particles(s, x, p["vx"].astype(np.float64), p["vy"].astype(np.float64),
                        p["vz"].astype(np.float64), p["id"], p["next_id"])
    o.set_step(c["step"])
    o.refresh_field()
    return o


def ties(x_orc, cfg):
    """Particles whose oracle position lies within 4 binary32 ulps of a cell
    edge: their cell index may legitimately differ."""
    xi = x_orc / dx_of(cfg)
    ulp = np.spacing(np.float32(np.maximum(np.abs(xi), 1.0))).astype(np.float64)
    return np.abs(xi - np.rint(xi)) <= 4 * ulp


def compare_species(pg, po, cfg, vscale):
    """Element-wise comparison of one species (same canonical order expected).
    Returns a dict of the worst deviations and mismatch counts."""
    L = cfg["length"]
    dx = dx_of(cfg)
    xg = gpu_positions(pg, cfg)
    xo = po["x"]
    dxp = np.abs(xg - xo)
    if cfg["bc"] == 0:
        dxp = np.minimum(dxp, L - dxp)
    cell_o = np.floor(xo / dx).astype(np.int64)
    if cfg["bc"] == 0:
        cell_o %= cfg["n_cells"]
    cell_mismatch = (pg["cell"].astype(np.int64) != cell_o) & ~ties(xo, cfg)
    dv = np.sqrt((pg["vx"] - po["vx"]) ** 2 + (pg["vy"] - po["vy"]) ** 2 + (pg["vz"] - po["vz"]) ** 2)
    vref = np.maximum(np.sqrt(po["vx"] ** 2 + po["vy"] ** 2 + po["vz"] ** 2), vscale)
    rel_v = dv / vref
    return dict(max_dx_over_L=float(dxp.max() / L) if len(dxp) else 0.0,
                max_dx_over_dx=float(dxp.max() / dx) if len(dxp) else 0.0,
                max_rel_v=float(rel_v.max()) if len(rel_v) else 0.0,
                cell_mismatch=int(cell_mismatch.sum()),
                id_equal=bool(np.array_equal(pg["id"], po["id"])),
                rel_v=rel_v, dx=dxp)


def small_argon(n_init=20000, seed=2, n_cells=400, weight=None):
    cfg = W.argon_rf(n_init=n_init, seed=seed, n_cells=n_cells,
                     weight=weight if weight else 6.0e13 / n_init * 0.5,
                     capacity=8 * n_init)
    return cfg, W.argon_tables()
