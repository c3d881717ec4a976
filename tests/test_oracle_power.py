"""Pins of the power decomposition (Section 1 lists the power terms; the
reading is the species' momentum balance m dGamma/dt + d(m n <vx^2>)/dx =
q n E + R times its mean velocity u = Gamma / n: the field's power q Gamma E
splits into an inertia term u (m dGamma/dt + d(m Gamma^2 / n)/dx), a
pressure term u dp/dx, p = m (n <vx^2> - Gamma^2 / n), and the ohmic rest
-u R, the momentum collisions take).

Exact: a cold lattice plasma accelerated by a uniform imposed field, no
collisions, no field solve: the density stays uniform and p = 0, so all the
power goes into inertia; the power itself is q n v E at the velocities of
the sampled steps.  Statistical: the Maxwell-model swarm at its steady drift
in a periodic box, where dGamma/dt averages out and the gradient terms
vanish summed over the box, so the ohmic term carries the field's power."""
import numpy as np

import oracle
import workloads as W


def test_uniform_acceleration_is_all_inertia():
    nc, per, L, dt, e0, v0 = 16, 8, 1.0, 0.01, 0.5, 0.37
    n = nc * per
    sp = W.species(-1.0, 1.0, 1.0, 0, 0.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=nc, bc=0, field_solve=0, length=L, dt=dt, e_ext=[e0, 0.0, 0.0], species=[sp],
                        seed=3)
    o = oracle.Oracle(cfg, load=False)
    x = (np.arange(n) + 0.5) * L / n
    o.set_particles(0, x, np.full(n, v0), np.zeros(n), np.zeros(n), np.arange(n))
    o.set_diag(True)
    o.step(1)                       # stores the flux the first derivative needs
    o.reset_avg()
    k = 20
    o.step(k)
    p = o.power(0)
    a = -1.0 * e0 / 1.0             # q E / m
    dens = n * 1.0 / L              # weight per macro 1
    vbar = v0 + a * dt * np.mean(np.arange(2, k + 2))
    np.testing.assert_allclose(p["power"], -1.0 * dens * vbar * e0, rtol=1e-12)
    scale = np.max(np.abs(p["power"]))
    np.testing.assert_allclose(p["inertia"], p["power"], rtol=0, atol=1e-10 * scale)
    assert np.max(np.abs(p["pressure"])) <= 1e-10 * scale
    assert np.max(np.abs(p["ohmic"])) <= 1e-10 * scale
    # the terms close on the field's power by construction
    np.testing.assert_allclose(p["inertia"] + p["pressure"] + p["ohmic"], p["power"], rtol=1e-14, atol=1e-14 * scale)


def test_first_sample_without_a_previous_flux_has_no_time_derivative():
    nc, per, L, dt, e0 = 8, 4, 1.0, 0.01, 0.5
    n = nc * per
    sp = W.species(-1.0, 1.0, 1.0, 0, 0.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=nc, bc=0, field_solve=0, length=L, dt=dt, e_ext=[e0, 0.0, 0.0], species=[sp])
    o = oracle.Oracle(cfg, load=False)
    o.set_particles(0, (np.arange(n) + 0.5) * L / n, np.full(n, 0.2), np.zeros(n), np.zeros(n), np.arange(n))
    o.step(3)                       # not sampled
    o.set_diag(True)
    o.step(1)
    p = o.power(0)
    assert np.max(np.abs(p["inertia"])) <= 1e-12 * np.max(np.abs(p["power"]))
    assert np.max(np.abs(p["ohmic"] - p["power"])) <= 1e-12 * np.max(np.abs(p["power"]))


def test_maxwell_swarm_power_is_ohmic():
    E, nu0, dt, n = 1e3, 1e9, 2e-11, 20000
    cfg, tabs = W.maxwell_swarm(e_field=-E, nu0=nu0, n_particles=n, gas_mass=W.M_ELECTRON * 20.0, dt=dt,
                                te_ev=1.0, n_cells=16)
    o = oracle.Oracle(cfg, tabs)
    o.set_threads(4)
    o.step(3000)                    # steady drift and energy
    o.set_diag(True)
    o.step(1)
    o.reset_avg()
    o.step(3000)
    p = o.power(0)
    total = p["power"].sum()
    assert total > 0.0              # the field heats the swarm
    assert abs(p["inertia"].sum()) <= 0.03 * total, p["inertia"].sum() / total
    assert abs(p["pressure"].sum()) <= 0.03 * total, p["pressure"].sum() / total
    assert abs(p["ohmic"].sum() / total - 1.0) <= 0.04, p["ohmic"].sum() / total
