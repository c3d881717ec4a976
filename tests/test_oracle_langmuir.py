"""Langmuir-wave pins of the oracle (Section 3.1, Figure 3).

The reference is the exact kinetic dispersion relation of a Maxwellian plasma,
1 + (1 + zeta Z(zeta)) / (k lambda_D)^2 = 0, zeta = omega / (sqrt(2) k v_th),
solved here with the Faddeeva function, plus the values the paper prints for
its worked example (golden fixture).  Mode-1 field histories from runs seeded
with +eps and -eps (same seed) are differenced to cancel the part of the
thermal noise that is even in eps, then averaged over seeds and fitted with
A exp(gamma t) cos(omega t + p).
"""
import json
import math
import multiprocessing as mp
import os

import numpy as np
from scipy.optimize import curve_fit, fsolve
from scipy.special import wofz

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kinetic_root(k):
    def f(z):
        w = z[0] + 1j * z[1]
        zeta = w / (math.sqrt(2) * k)
        d = 1 + (1 + zeta * 1j * math.sqrt(math.pi) * wofz(zeta)) / k ** 2
        return [d.real, d.imag]
    r = fsolve(f, [math.sqrt(1 + 3 * k * k), -0.05], xtol=1e-13)
    return r[0], r[1]


def _mode1_series(args):
    k, eps, n, steps, seed = args
    cfg = W.langmuir(k_lambda=k, eps=eps, n_particles=n, seed=seed)
    o = oracle.Oracle(cfg)
    L, nn = cfg["length"], o.n_nodes
    s = np.sin(2 * np.pi * np.arange(nn) / nn)
    out = np.empty(steps)
    for i in range(steps):
        o.step(1)
        out[i] = 2.0 / nn * np.dot(o.field()[2], s)
    return out


def measure(k, eps, n, steps, seeds, window):
    jobs = [(k, sgn * eps, n, steps, sd) for sd in seeds for sgn in (1, -1)]
    procs = min(len(jobs), os.cpu_count() or 1, 8)
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_mode1_series, jobs)
    sig = np.mean([0.5 * (res[2 * i] - res[2 * i + 1]) for i in range(len(seeds))], axis=0)
    t = (np.arange(steps) + 1) * 0.1
    m = (t >= window[0]) & (t <= window[1])
    model = lambda t, A, g, w, p: A * np.exp(g * t) * np.cos(w * t + p)
    p, _ = curve_fit(model, t[m], sig[m], p0=[sig[m][0], -0.05, math.sqrt(1 + 3 * k * k), 0.0],
                     maxfev=20000)
    return p[2], p[1]


def test_kinetic_roots_match_known_values():
    # Independent check of the root finder itself (values in the text: the
    # 0.38 case is 5 % above Bohm-Gross; asymptotic formula 0.081 vs exact 0.053).
    w, g = kinetic_root(0.38)
    assert abs(w / math.sqrt(1 + 3 * 0.38 ** 2) - 1 - 0.05) < 0.005
    assert abs(-g - 0.053) < 0.001
    w, g = kinetic_root(0.1)
    assert abs(w / math.sqrt(1.03) - 1) < 0.001


def test_landau_paper_worked_example():
    gold = json.load(open(os.path.join(GOLDEN, "langmuir_paper_example.json")))
    k, eps = gold["k_lambda_d"], gold["seed_fraction"]
    w, g = measure(k, eps, 1 << 20, 160, [1, 2, 3, 4], (4.0, 16.0))
    wk, gk = kinetic_root(k)
    assert abs(g / gk - 1) < 0.05
    assert abs(-g / gold["gamma_over_omega_pe"] - 1) < 0.05
    assert abs(w / wk - 1) < 0.01
    above_bg = w / math.sqrt(1 + 3 * k * k) - 1
    assert abs(above_bg - gold["omega_above_bohm_gross"]) < 0.01
    assert abs(wk / k - gold["phase_velocity_over_vth"]) < 0.05


def test_landau_linear_regime():
    # k lambda_D = 0.5 with a 0.5 % seed: gamma / omega_bounce ~ 2, so the
    # decay is linear Landau damping over the whole window.
    w, g = measure(0.5, 0.005, 1 << 20, 130, [1, 2, 3, 4], (2.0, 12.0))
    wk, gk = kinetic_root(0.5)
    assert abs(g / gk - 1) < 0.05
    assert abs(w / wk - 1) < 0.01


def test_langmuir_config_frequency_and_damping():
    # The Langmuir configuration (k lambda_D = 0.3, 1 % seed, 128 cells):
    # frequency within 1 % of the kinetic root (which is 2.9 % above
    # Bohm-Gross).  Its seed is in the trapping regime (bounce frequency
    # sqrt(eps) omega_pe = 0.1 against gamma = 0.0126), so the decay is only
    # approximately the linear rate: 10 % here; the 5 % bar is held by the
    # linear-regime and worked-example tests above.
    w, g = measure(0.3, 0.01, 1 << 18, 400, list(range(1, 9)), (5.0, 40.0))
    wk, gk = kinetic_root(0.3)
    assert abs(w / wk - 1) < 0.01
    assert abs(g / gk - 1) < 0.10


def test_bohm_gross_long_wavelength():
    # k lambda_D = 0.1: kinetic and Bohm-Gross frequencies agree to 0.03 %.
    w, _ = measure(0.1, 0.01, 1 << 16, 400, [1, 2], (3.0, 40.0))
    assert abs(w / math.sqrt(1 + 3 * 0.01) - 1) < 0.01


def test_total_energy_conserved_collisionless():
    cfg = W.langmuir()
    o = oracle.Oracle(cfg)
    tot = []
    for _ in range(300):
        fe = o.energy()[1]                 # E^n
        o.step(1)
        ke = o.energy()[0].sum()           # time-centred kinetic energy at n
        tot.append(ke + fe)
    tot = np.array(tot)
    assert np.ptp(tot) / tot[0] < 2e-4
