"""Pins of the oracle's axial renewal (Section 3.6 follows Lafleur, Baalrud
and Chabert: particles are renewed after a virtual axial transit L_z).

Free flight gives the renewal step of each particle in closed form, the
renewed velocities are the Box-Muller normals of the particle's own Philox
draw, and an ion starting at rest in the axial field reaches L_z after the
discrete transit time of the leapfrog, N = ceil(sqrt(2 L_z / (a dt^2)))."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W


def _box_muller(ua, ub):
    r = math.sqrt(-2.0 * math.log(ua))
    return r * math.cos(2.0 * math.pi * ub), r * math.sin(2.0 * math.pi * ub)


def _cfg(n, lz, vth=1.0, drift=(0.0, 0.0, 0.0), dt=0.1, e_ext=(0.0, 0.0, 0.0), charge=-1.0, mass=1.0, seed=9):
    sp = W.species(charge, mass, 1.0, 0, vth, capacity=n, drift=drift, load=W.LOAD_NONE)
    return W.base_config(n_cells=16, bc=0, field_solve=0, length=1.0, dt=dt, e_ext=list(e_ext),
                         species=[sp], renew_lz=lz, seed=seed)


def test_free_flight_renewal_step_and_velocities():
    # particle j moves along z only, at a speed with L_z / (|vz| dt) = k_j + 1/2,
    # so its first renewal comes at the end of step k_j + 1 (index k_j)
    lz, dt, n = 0.3, 0.1, 12
    k = np.arange(1, n + 1)
    vz = lz / ((k + 0.5) * dt) * np.where(k % 2 == 0, 1.0, -1.0)
    # renewed velocities are slow (no second renewal within the run)
    cfg = _cfg(n, lz, vth=0.02, drift=(0.01, -0.02, 0.03), dt=dt)
    o = oracle.Oracle(cfg, load=False)
    x = (np.arange(n) + 0.5) / n
    ids = np.arange(100, 100 + n, dtype=np.uint32)
    o.set_particles(0, x, np.zeros(n), np.zeros(n), vz, ids)
    steps = 7
    o.step(steps)
    c = o.counters()
    hit = k + 1 <= steps
    assert c["renewed"][0] == hit.sum()
    p = o.get_particles(0)
    z = o.axial(0)
    seed = cfg["seed"]
    for j in range(n):
        if not hit[j]:
            assert p["vz"][j] == vz[j] and p["vx"][j] == 0.0
            assert z[j] == pytest.approx(steps * vz[j] * dt, rel=1e-12)
            continue
        r = oracle.philox([int(ids[j]), int(k[j]), 6, 0], [seed & 0xffffffff, seed >> 32])
        g0, g1 = _box_muller(oracle.u01(r[0]), oracle.u01(r[1]))
        g2, _ = _box_muller(oracle.u01(r[2]), oracle.u01(r[3]))
        want = np.array([0.01 + 0.02 * g0, -0.02 + 0.02 * g1, 0.03 + 0.02 * g2])
        # renewed at the end of step index k_j, then free flight with the new velocity
        np.testing.assert_allclose([p["vx"][j], p["vy"][j], p["vz"][j]], want, rtol=1e-13, atol=1e-15)
        assert z[j] == pytest.approx((steps - k[j] - 1) * want[2] * dt, abs=1e-13)
    # positions never move along x before a renewal, and move with the new vx after
    xs = (x + np.where(hit, (steps - k - 1) * p["vx"] * dt, 0.0)) % 1.0
    np.testing.assert_allclose(p["x"], xs, atol=1e-12)


def test_renewed_velocities_follow_the_initial_distribution():
    # an axial length far below one step's displacement renews every particle
    # every step: the velocities are draws of the loaded Maxwellian with drift
    n, vth, drift = 20000, 2.0, (1.5, 0.0, -0.5)
    cfg = _cfg(n, 1e-9, vth=vth, drift=drift)
    o = oracle.Oracle(cfg, load=False)
    rng = np.random.default_rng(1)
    o.set_particles(0, rng.random(n), np.zeros(n), np.zeros(n), np.full(n, 5.0), np.arange(n))
    o.step(2)
    assert o.counters()["renewed"][0] == 2 * n
    p = o.get_particles(0)
    for comp, d in zip(("vx", "vy", "vz"), drift):
        assert stats.kstest((p[comp] - d) / vth, "norm").pvalue > 1e-4
    assert np.all(o.axial(0) == 0.0)


def test_ion_transit_time_in_the_axial_field():
    # from rest with the leapfrog start, v^{n+1/2} = a dt (n + 1/2), so after
    # N steps z = a dt^2 N^2 / 2: the first renewal is at N = ceil(sqrt(2 L_z / (a dt^2)))
    q, m, e, dt, lz, n = 1.0, 40.0, 3.0, 0.05, 0.37, 64
    a = q * e / m
    nstar = math.ceil(math.sqrt(2 * lz / (a * dt * dt)))
    assert abs(math.sqrt(2 * lz / (a * dt * dt)) - round(math.sqrt(2 * lz / (a * dt * dt)))) > 0.05
    sp = W.species(q, m, 1.0, n, 0.0, capacity=n, load=W.LOAD_STRATIFIED)
    cfg = W.base_config(n_cells=16, bc=0, field_solve=0, length=1.0, dt=dt, e_ext=[0.0, 0.0, e],
                        species=[sp], renew_lz=lz, seed=4)
    o = oracle.Oracle(cfg)
    o.step(nstar - 1)
    assert o.counters()["renewed"][0] == 0
    z = o.axial(0)
    np.testing.assert_allclose(z, a * dt * dt * (nstar - 1) ** 2 / 2, rtol=1e-12)
    o.step(1)
    assert o.counters()["renewed"][0] == n
    assert np.all(o.get_particles(0)["vz"] == 0.0) and np.all(o.axial(0) == 0.0)


def test_no_renewal_when_off_and_resets():
    cfg = _cfg(8, 0.0)
    o = oracle.Oracle(cfg, load=False)
    o.set_particles(0, np.linspace(0.05, 0.95, 8), np.zeros(8), np.zeros(8), np.full(8, 100.0), np.arange(8))
    o.step(5)
    assert o.counters()["renewed"][0] == 0
    assert np.all(o.axial(0) == 0.0)              # not tracked without renewal
    o.set_axial(0, np.full(8, 0.25))
    assert np.all(o.axial(0) == 0.25)
    p = o.get_particles(0)
    o.set_particles(0, p["x"], p["vx"], p["vy"], p["vz"], p["id"])
    assert np.all(o.axial(0) == 0.0)
    with pytest.raises(oracle.OracleError):
        o.set_axial(0, np.zeros(3))
    with pytest.raises(oracle.OracleError):
        oracle.Oracle(_cfg(8, -1.0), load=False)
