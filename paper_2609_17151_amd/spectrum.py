"""Space-time spectra of a periodic box (Section 3.6: the two-dimensional
spectrum of the ion density and its dominant wavelength).

A history is a [T, N] array of a field sampled at N nodes of a periodic mesh
every `dt_sample` seconds.  Its spectrum is |FFT_t FFT_x (f - mean)|^2 over
(omega, k); the dominant mode is the spatial mode m = k L / 2 pi that holds
the most power summed over frequency.
"""
from __future__ import annotations

import numpy as np


def record(sim, species, every, count, batch=0, progress=None):
    """Density of `species` at the nodes after every `every` steps, `count`
    times: a [count, N] history (m^-3).  `progress(i)` is called after each
    sample when given."""
    out = np.zeros((count, sim.n_nodes[batch]))
    for i in range(count):
        sim.step(every)
        out[i] = sim.density(batch)[species]
        if progress:
            progress(i)
    return out


def spectrum(history, length, dt_sample):
    """(power[omega, m], m, omega): the power of the fluctuation f - <f> per
    spatial mode m = 0 .. N/2 and angular frequency omega (rad/s), both
    halves of the frequency axis kept (the sign of omega gives the direction
    of propagation for m > 0)."""
    h = np.asarray(history, dtype=np.float64)
    T, N = h.shape
    f = h - h.mean()
    F = np.fft.fft(np.fft.rfft(f, axis=1), axis=0)
    P = np.abs(F) ** 2 / (T * N) ** 2
    m = np.arange(P.shape[1])
    omega = 2.0 * np.pi * np.fft.fftfreq(T, d=dt_sample)
    order = np.argsort(omega)
    return P[order], m, omega[order]


def dominant_mode(history, length, dt_sample=1.0):
    """The spatial mode (m >= 1) with the most power summed over frequency,
    and its wavelength L / m."""
    P, m, _ = spectrum(history, length, dt_sample)
    pm = P.sum(axis=0)
    pm[0] = 0.0
    k = int(np.argmax(pm))
    return k, length / k if k else np.inf


def power_near(P, m, omega, curve, length, width=0.2):
    """Fraction of the fluctuation power (m >= 1) within a relative band
    |omega - curve(k)| <= width |curve(k)| of a dispersion relation
    omega = curve(k), k = 2 pi m / L (both signs of omega accepted)."""
    k = 2.0 * np.pi * m / length
    w = np.abs(np.asarray(curve(k), dtype=np.float64))
    near = np.abs(np.abs(omega)[:, None] - w[None, :]) <= width * np.maximum(w[None, :], 1e-300)
    near[:, 0] = False
    tot = P[:, 1:].sum()
    return float(P[near].sum() / tot) if tot > 0 else 0.0
