"""Pins of the swarm setting (Section 4: electrons only, no Poisson solve) in
the oracle: the steady drift and mean energy of the Maxwell model (constant
collision frequency) in closed form for the discrete scheme, and the growth
of an ionizing swarm whose ions are not followed.

Closed forms.  With a collision probability p per step, a kick a dt per
step and elastic scattering that keeps, on average, the fraction
f(beta) = (1/2) int_{-1}^{1} c sqrt(1 - beta (1 - c)) dc of the incident
velocity (beta = 2m/M, isotropic c = cos chi), the stored velocity after the
collision stage has the mean W_s = q a dt / (1 - q), q = 1 - p (1 - f).  The
energy before the collision stage satisfies gain = loss,
m a dt (W_s + a dt / 2) = p beta eps_pre, and the time-centred energy the
oracle reports is eps_pre (1 - p beta / 2).  For beta -> 0 and dt -> 0 these
are eE/(m nu) and M W^2 / 2."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W


def test_maxwell_model_drift_and_energy_closed_forms():
    E, nu0, dt, mr, n = 1e3, 1e9, 2e-11, 20.0, 10000
    cfg, tabs = W.maxwell_swarm(e_field=-E, nu0=nu0, n_particles=n, gas_mass=W.M_ELECTRON * mr, dt=dt,
                                te_ev=1.0)
    o = oracle.Oracle(cfg, tabs)
    numax, _ = o.numax(0)
    p = (1.0 - math.exp(-numax * dt)) * nu0 / numax
    beta = 2.0 / mr
    f = 0.5 * integrate.quad(lambda c: c * math.sqrt(1.0 - beta * (1.0 - c)), -1.0, 1.0)[0]
    a = W.E_CHARGE * E / W.M_ELECTRON
    q = 1.0 - p * (1.0 - f)
    ws = q * a * dt / (1.0 - q)
    eps_pre = W.M_ELECTRON * a * dt * (ws + 0.5 * a * dt) / (p * beta)
    eps_c = eps_pre * (1.0 - 0.5 * p * beta) / W.E_CHARGE
    o.step(3000)                        # six energy relaxation times M / (2 m nu)
    vx, ke = [], []
    for _ in range(60):
        o.step(50)
        k, _ = o.energy()
        vx.append(o.get_particles(0)["vx"].mean())
        ke.append(k[0] / (cfg["species"][0]["weight"] * n) / W.E_CHARGE)
    assert np.mean(vx) == pytest.approx(ws, rel=0.01)
    assert np.mean(ke) == pytest.approx(eps_c, rel=0.01)
    # the continuum limits, for scale: within a few per cent at this beta, nu dt
    assert ws == pytest.approx(W.E_CHARGE * E / (W.M_ELECTRON * nu0), rel=0.03)
    assert eps_c == pytest.approx(0.5 * mr * W.M_ELECTRON * ws ** 2 / W.E_CHARGE, rel=0.03)


def test_ionizing_swarm_grows_at_the_ionization_probability():
    # every collision is ionization or elastic at constant frequencies, with
    # no threshold: each electron ionizes with probability
    # p_iz = (1 - exp(-nu_max dt)) nu_iz / nu_max per step, and no ion appears
    nu_el, nu_iz, dt, n, steps = 4e8, 1e8, 1e-10, 20000, 40
    ng = 1e22
    cfg, _ = W.maxwell_swarm(e_field=0.0, nu0=1.0, n_particles=n, dt=dt, te_ev=1.0)
    cfg["species"][0]["capacity"] = 4 * n
    e = np.logspace(-6, 4, 2000)
    v = np.sqrt(2.0 * e * W.E_CHARGE / W.M_ELECTRON)
    tabs = [dict(species=0, kind=W.XS_ELASTIC, threshold=0.0, energy=e, sigma=nu_el / (ng * v)),
            dict(species=0, kind=W.XS_IONIZATION, threshold=0.0, energy=e, sigma=nu_iz / (ng * v))]
    o = oracle.Oracle(cfg, tabs)
    numax, _ = o.numax(0)
    p_iz = (1.0 - math.exp(-numax * dt)) * nu_iz / numax
    o.step(steps)
    c = o.counters()
    n_end = len(o.get_particles(0)["x"])
    assert n_end == n + c["coll"][0][1]          # one electron per ionization
    expect = n * (1.0 + p_iz) ** steps
    # the sum of the binomial increments: variance below the Poisson bound
    assert abs(n_end - expect) <= 5.0 * math.sqrt(expect - n)


def test_ionization_accepted_with_electrons_only():
    cfg, _ = W.maxwell_swarm(n_particles=100)
    o = oracle.Oracle(cfg, load=False)
    t = W.argon_tables(n=50)[2]
    o.load_xsec(0, W.XS_IONIZATION, t["threshold"], t["energy"], t["sigma"])
