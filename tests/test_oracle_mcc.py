"""Pins of the oracle's null-collision Monte Carlo, walls and secondary emission.

Reference values are binomial expectations from the tabulated cross sections,
the Maxwell-model drift closed form, energy bookkeeping identities, thermal
equilibrium, and the secondary-emission yield.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

E = W.E_CHARGE
ME = W.M_ELECTRON


def _z(n):
    return np.zeros(n)


def _monoenergetic(n, eps_ev, seed=0, mass=ME):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    v = math.sqrt(2 * eps_ev * E / mass)
    return v * d


def _argon_electron_box(n, eps_ev, seed=0):
    cfg = W.argon_rf(n_init=0)
    cfg["bc"] = 0
    cfg["field_solve"] = 0
    cfg["see_gamma"] = 0.0
    for sp in cfg["species"]:
        sp["capacity"] = 2 * n
        sp["load"] = W.LOAD_NONE
    o = oracle.Oracle(cfg, W.argon_tables(), load=False)
    v = _monoenergetic(n, eps_ev, seed)
    x = np.random.default_rng(seed + 1).uniform(0, cfg["length"], n)
    o.set_particles(0, x, v[0], v[1], v[2], np.arange(n))
    o.refresh_field()
    return o, cfg


def _sigma_analytic(eps):
    el = 1e-19 * (1 - 0.9 * math.exp(-math.log(eps / 0.3) ** 2 / 0.5)) / (1 + eps / 30)
    f = lambda th, a: 0.0 if eps <= th else a * (eps / th - 1) / (eps / th) ** 2
    return [el, f(11.5, 4e-20), f(15.8, 12e-20)]


def test_candidate_fraction_and_channel_frequencies():
    n = 400_000
    eps = 20.0
    o, cfg = _argon_electron_box(n, eps)
    numax, t32 = o.numax(0)
    pnull = 1 - math.exp(-numax * cfg["dt"])
    assert abs(t32 - math.floor(pnull * 2 ** 32)) <= 1
    o.step(1)
    c = o.counters()
    cand = c["candidates"][0]
    mu = n * t32 / 2 ** 32
    assert abs(cand - mu) < 5 * math.sqrt(mu)
    v = math.sqrt(2 * eps * E / ME)
    for k, s in enumerate(_sigma_analytic(eps)):
        p = cfg["gas_density"] * s * v / numax
        mu = cand * p
        assert abs(c["coll"][0][k] - mu) < 5 * math.sqrt(mu * (1 - p)) + 1, k
    assert c["violations"][0] == 0


def test_numax_bounds_collision_frequency():
    # nu_max is an upper bound of n_g sum sigma v over the table range.
    o, cfg = _argon_electron_box(10, 1.0)
    numax, _ = o.numax(0)
    tabs = W.argon_tables()[:3]
    e = np.logspace(-2, 3, 20001)
    tot = sum(np.interp(np.log(e), np.log(t["energy"]), t["sigma"]) *
              (e >= t["threshold"]) for t in tabs)
    nu = cfg["gas_density"] * tot * np.sqrt(2 * e * E / ME)
    assert nu.max() < numax <= 1.06 * nu.max()


def test_no_inelastic_below_threshold():
    o, _ = _argon_electron_box(200_000, 11.0)
    o.step(1)
    c = o.counters()
    assert c["coll"][0][0] > 0 and c["coll"][0][1] == 0 and c["coll"][0][2] == 0


def test_excitation_removes_threshold_energy():
    n = 200_000
    o, _ = _argon_electron_box(n, 13.0, seed=3)
    o.step(1)
    p = o.get_particles(0)
    eps = 0.5 * ME * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2) / E
    c = o.counters()
    exc = np.abs(eps - 1.5) < 1e-9
    assert exc.sum() == c["coll"][0][1] > 0


def test_ionization_energy_bookkeeping_and_pairs():
    n = 200_000
    eps0 = 50.0
    o, cfg = _argon_electron_box(n, eps0, seed=4)
    o.step(1)
    c = o.counters()
    pe, pi = o.get_particles(0), o.get_particles(1)
    nion = c["coll"][0][2]
    assert nion > 0
    assert len(pe["x"]) == n + nion and len(pi["x"]) == nion        # pairs, in order
    assert np.array_equal(pe["id"][n:], np.arange(n, n + nion))
    assert np.array_equal(pi["id"], np.arange(nion))
    assert np.array_equal(pe["x"][n:], pi["x"])                       # born together
    eps = 0.5 * ME * (pe["vx"] ** 2 + pe["vy"] ** 2 + pe["vz"] ** 2) / E
    parents = np.nonzero(eps[:n] <= eps0 - 15.8 + 1e-9)[0]
    assert len(parents) == nion
    assert np.max(np.abs(eps[parents] + eps[n:] - (eps0 - 15.8))) < 1e-11 * eps0
    # born ions are thermal at T_g
    kt = W.K_BOLTZMANN * cfg["gas_temp"]
    ke = 0.5 * cfg["gas_mass"] * (pi["vx"] ** 2 + pi["vy"] ** 2 + pi["vz"] ** 2)
    assert abs(ke.mean() / (1.5 * kt) - 1) < 6 * math.sqrt(2 / 3 / nion)


def test_maxwell_model_drift_and_free_flight_law():
    # Constant collision frequency nu0 with an infinitely heavy target: the
    # drift is the Maxwell-model value eE/(m nu0); with one collision test per
    # step the stored (post-collision) mean is a dt / (exp(nu0 dt) - 1).
    nu0, efield, dt = 1e9, -1e3, 1e-11
    cfg, tabs = W.maxwell_swarm(e_field=efield, nu0=nu0, n_particles=50_000, dt=dt)
    o = oracle.Oracle(cfg, tabs)
    a = -E * efield / ME                       # electron acceleration (> 0)
    o.step(500)
    c0 = o.counters()
    vs = []
    for _ in range(30):
        o.step(50)
        vs.append(o.get_particles(0)["vx"].mean())
    w_discrete = a * dt / math.expm1(nu0 * dt)
    w_maxwell = a / nu0
    assert abs(np.mean(vs) / w_discrete - 1) < 0.01
    assert abs(w_discrete / w_maxwell - 1) < 0.006
    c1 = o.counters()
    real = c1["coll"][0][0] - c0["coll"][0][0]
    p = -math.expm1(-nu0 * dt)
    mu = 50_000 * 1500 * p
    assert abs(real - mu) < 5 * math.sqrt(mu)
    assert c1["violations"][0] == 0


@pytest.mark.parametrize("kind", [W.XS_ION_CX, W.XS_ION_ISO])
def test_ion_thermalisation(kind):
    # Ions colliding with a 300 K neutral gas relax to its Maxwellian,
    # mean energy (3/2) k T_g.
    n = 10_000
    ng = 3e23
    sp = W.species(E, W.AR_MASS, 1.0, 0, 1.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=16, bc=0, field_solve=0, length=0.01, dt=1e-10,
                        eps0=W.EPS0, e_unit=E, gas_density=ng, gas_temp=300.0,
                        gas_mass=W.AR_MASS, species=[sp], seed=9)
    e = np.logspace(-3, 1, 200)       # table top sets g_max, hence nu_max
    o = oracle.Oracle(cfg, [dict(species=0, kind=kind, threshold=0.0, energy=e,
                                 sigma=np.full(200, 5e-19))], load=False)
    v = _monoenergetic(n, 0.5, seed=5, mass=W.AR_MASS)
    o.set_particles(0, np.random.default_rng(6).uniform(0, 0.01, n), v[0], v[1], v[2],
                    np.arange(n))
    o.refresh_field()
    o.step(1500 if kind == W.XS_ION_CX else 3500)
    p = o.get_particles(0)
    ke = 0.5 * W.AR_MASS * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2)
    kt = W.K_BOLTZMANN * 300.0
    assert abs(ke.mean() / (1.5 * kt) - 1) < 0.04
    assert abs(p["vx"].mean()) < 5 * math.sqrt(kt / W.AR_MASS / n)


def test_secondary_emission_yield_and_kinematics():
    n = 100_000
    gamma = 0.1
    cfg = W.argon_rf(n_init=0, see_gamma=gamma)
    cfg["field_solve"] = 0
    for sp in cfg["species"]:
        sp["capacity"] = 2 * n
        sp["load"] = W.LOAD_NONE
    o = oracle.Oracle(cfg, load=False)
    L, dt = cfg["length"], cfg["dt"]
    # ions next to both walls, moving out fast enough to leave in one step
    half = n // 2
    x = np.r_[np.full(half, 1e-7), np.full(n - half, L - 1e-7)]
    vx = np.r_[np.full(half, -1e4), np.full(n - half, 1e4)]
    o.set_particles(1, x, vx, _z(n), _z(n), np.arange(n))
    o.refresh_field()
    o.step(1)
    c = o.counters()
    assert c["absorbed"][1].tolist() == [half, n - half]
    em = c["see_emitted"]
    for w, na in ((0, half), (1, n - half)):
        assert abs(em[w] - gamma * na) < 5 * math.sqrt(na * gamma * (1 - gamma))
    pe = o.get_particles(0)
    assert len(pe["x"]) == em.sum()
    vsee = math.sqrt(1.0 * E / ME)
    left = pe["x"] < L / 2
    assert np.all(pe["vx"][left] > 0) and np.all(pe["vx"][~left] < 0)
    assert np.all(pe["x"][left] <= pe["vx"][left] * dt)
    assert np.all(L - pe["x"][~left] <= -pe["vx"][~left] * dt)
    # normal speeds: flux-weighted half-Maxwellian, mean v_see sqrt(pi/2)
    s = np.abs(pe["vx"])
    assert abs(s.mean() / (vsee * math.sqrt(math.pi / 2)) - 1) < 5 * 0.52 / math.sqrt(len(s))
    assert abs(pe["vy"].std() / vsee - 1) < 0.05


def test_particle_count_bookkeeping_bounded():
    # Counts are integer-exact: N(n+1) = N(n) - absorbed + born; ionization
    # makes pairs, so N_e - N_i changes only by wall losses and emission.
    cfg = W.argon_rf(n_init=20000, weight=1e9)
    o = oracle.Oracle(cfg, W.argon_tables())
    ne0, ni0 = len(o.get_particles(0)["x"]), len(o.get_particles(1)["x"])
    o.step(200)
    c = o.counters()
    ne, ni = len(o.get_particles(0)["x"]), len(o.get_particles(1)["x"])
    nionz = c["coll"][0][2]
    assert ne == ne0 - c["absorbed"][0].sum() + nionz + c["see_emitted"].sum()
    assert ni == ni0 - c["absorbed"][1].sum() + nionz
    assert c["dropped"] == 0
