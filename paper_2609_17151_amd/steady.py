"""Periodic steady state of RF discharges: window profiles and the rule that
decides when a run has converged.

A window is a whole number of RF periods over which the library accumulates
the time-averaged electron density, ion density and electron mean energy at
the mesh nodes.  Every profile is resampled to NPTS points evenly spread over
x / gap, so discharges with different meshes compare point by point.

Converged: the reference state of a discharge is the mean of its windows over
a late span of a cold run (the last 50 periods); a run has converged at the
first window after which NRUN consecutive windows all lie within a relative
L2 distance of the reference, in each of the three profiles.  The distance
allowed is 2 % or, when a window's own statistical scatter is larger, three
times that scatter (the RMS distance of the reference span's windows to their
mean), as profiles are held to 2 % or the run's statistical error.
"""
from __future__ import annotations

import numpy as np

NPTS = 256
TOL = 0.02
NRUN = 10
N_FLOOR = 1e12          # m^-3, added before taking log10 of a density


def resample(y, npts=NPTS):
    """Node values on a uniform mesh over [0, gap] -> npts points over x / gap."""
    y = np.asarray(y, dtype=np.float64)
    return np.interp(np.linspace(0.0, 1.0, npts), np.linspace(0.0, 1.0, y.size), y)


def window(sim, batch=0, electron=0, ion=1):
    """The [3, NPTS] profiles (n_e, n_i, mean electron energy in eV) accumulated
    since the last reset of discharge `batch`; then clears the accumulators.
    Latched device conditions are not raised here: the caller reads them
    with the counts."""
    a = sim.avg(batch, check=False)
    out = np.stack([resample(a["density"][electron]), resample(a["density"][ion]),
                    resample(a["mean_energy"])])
    sim.reset_avg(batch, check=False)
    return out


def distance(w, ref):
    """Largest relative L2 distance over the three profiles."""
    w, ref = np.asarray(w), np.asarray(ref)
    out = 0.0
    for k in range(ref.shape[0]):
        nr = float(np.linalg.norm(ref[k]))
        nd = float(np.linalg.norm(w[k] - ref[k]))
        out = max(out, nd / nr if nr > 0.0 else (0.0 if nd == 0.0 else float("inf")))
    return out


def noise_tolerance(dists, span_windows=10, k=3.0, floor=TOL):
    """Allowed distance: max(floor, k x RMS of the last `span_windows`
    distances to the reference), the windows that make up the reference."""
    d = np.asarray(dists, dtype=np.float64)
    d = d[np.isfinite(d)][-span_windows:]
    if d.size == 0:
        return floor
    return max(floor, k * float(np.sqrt(np.mean(d * d))))


def converged_at(windows, ref, tol=TOL, nrun=NRUN):
    """Index of the first window from which `nrun` consecutive windows are all
    within `tol` of `ref`, or None."""
    ok = [distance(w, ref) <= tol for w in windows]
    for i in range(len(ok) - nrun + 1):
        if all(ok[i:i + nrun]):
            return i
    return None


def to_features(windows_mean):
    """Network targets of a [3, NPTS] state: log10 densities (with a floor) and
    the mean energy in eV, flattened to 3 * NPTS values."""
    s = np.asarray(windows_mean, dtype=np.float64)
    return np.concatenate([np.log10(s[0] + N_FLOOR), np.log10(s[1] + N_FLOOR), s[2]])


def from_features(f):
    """Inverse of to_features: [3, NPTS] (n_e, n_i in m^-3, energy in eV)."""
    f = np.asarray(f, dtype=np.float64).reshape(3, -1)
    return np.stack([np.maximum(10.0 ** f[0] - N_FLOOR, 0.0), np.maximum(10.0 ** f[1] - N_FLOOR, 0.0),
                     np.maximum(f[2], 0.0)])
