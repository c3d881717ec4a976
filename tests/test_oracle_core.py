"""Pins of the FP64 oracle: random numbers, push, mesh weighting and field.

Each check compares the oracle with something it does not compute itself:
published known-answer values, closed forms of the discrete scheme, exact
invariants, or textbook limits.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as W


# ---------------------------------------------------------------- Philox ----
def test_philox_known_answers():
    # Salmon et al. (SC'11) Philox4x32-10 known-answer vectors.
    assert [hex(v) for v in oracle.philox([0, 0, 0, 0], [0, 0])] == \
        ["0x6627e8d5", "0xe169c58d", "0xbc57ac4c", "0x9b00dbd8"]
    assert [hex(v) for v in oracle.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)] == \
        ["0x408f276d", "0x41c83b0e", "0xa20bc7c6", "0x6d5451fd"]


def test_uniform_map_is_exact_and_open():
    for x in (0, 1, 511, 512, 0x7FFFFFFF, 0xFFFFFFFF, 0xDEADBEEF):
        u = oracle.u01(x)
        assert 0.0 < u < 1.0
        k = u * 2 ** 24
        assert k == int(k) and int(k) % 2 == 1           # odd multiple of 2^-24
        assert np.float32(u) == u                         # exact in binary32
    assert oracle.u01(0) == 2.0 ** -24
    assert oracle.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24


def test_philox_uniforms_pass_ks():
    u = np.array([oracle.u01(oracle.philox([i, 7, 3, 0], [11, 13])[j])
                  for i in range(2500) for j in range(4)])
    assert stats.kstest(u, "uniform").pvalue > 1e-3


# ---------------------------------------------------------------- Boris -----
def test_boris_rotation_angle_and_speed():
    # With E = 0 the Boris step is a rotation by exactly 2 atan(w_c dt / 2).
    qm, b, dt = -1.7, 0.9, 0.37
    v0 = np.array([0.3, -1.1, 0.5])
    v = oracle.boris(v0, [0, 0, 0], [0, 0, b], qm, dt)
    theta = 2 * math.atan(abs(qm * b) * dt / 2)
    vp0, vp1 = v0[:2], v[:2]
    cosang = vp0 @ vp1 / (np.linalg.norm(vp0) * np.linalg.norm(vp1))
    assert abs(math.acos(cosang) - theta) < 1e-12
    assert v[2] == v0[2]                                  # parallel part untouched
    # electrons (q<0) gyrate counter-clockwise about +z
    assert np.cross(np.r_[vp0, 0], np.r_[vp1, 0])[2] > 0
    for _ in range(20000):
        v = oracle.boris(v, [0, 0, 0], [0.2, -0.4, b], qm, dt)
    assert abs(np.linalg.norm(v) - np.linalg.norm(v0)) < 1e-13 * np.linalg.norm(v0) * 50


def test_boris_pure_electric_kick():
    v = oracle.boris([0.1, 0.2, 0.3], [2.0, -1.0, 0.5], [0, 0, 0], 3.0, 0.25)
    assert np.allclose(v, [0.1 + 1.5, 0.2 - 0.75, 0.3 + 0.375], rtol=0, atol=1e-15)


def _orbit_cfg(qm_sign=-1.0, mass=1.0, bz=1.0, dt=0.1, e_ext=(0, 0, 0)):
    sp = W.species(qm_sign, mass, 1.0, 1, 1.0, capacity=1, load=W.LOAD_NONE)
    return W.base_config(n_cells=64, bc=0, field_solve=0, length=1000.0, dt=dt,
                         eps0=1.0, b_ext=[0, 0, bz], e_ext=list(e_ext), species=[sp])


def _track(cfg, x0, v, steps):
    o = oracle.Oracle(cfg, load=False)
    o.set_particles(0, [x0], [v[0]], [v[1]], [v[2]], [0])
    o.refresh_field()
    xs = [x0]
    for _ in range(steps):
        o.step(1)
        xs.append(o.get_particles(0)["x"][0])
    return np.array(xs), o


def test_gyration_is_discrete_circle():
    # x_n = x_c + r_d cos(n theta + a), r_d = |v_perp| dt / (2 sin(theta/2)).
    dt, vperp = 0.1, 2.0
    cfg = _orbit_cfg(dt=dt)
    xs, _ = _track(cfg, 500.0, [vperp, 0.0, 0.3], 400)
    theta = 2 * math.atan(dt / 2)
    c = 2 * math.cos(theta)
    rec = xs[2:] - c * xs[1:-1] + xs[:-2]                 # = (2 - 2cos th) x_c
    xc = rec / (2 - c)
    assert np.ptp(xc) < 1e-9
    xcm = xc.mean()
    r = np.sqrt((xs[1:-1] - xcm) ** 2 + ((xs[2:] - xs[:-2]) / (2 * math.sin(theta))) ** 2)
    r_d = vperp * dt / (2 * math.sin(theta / 2))
    assert np.max(np.abs(r - r_d)) < 1e-9 * r_d


def test_gyroradius_ratio_sqrt_mass_ratio():
    # Equal energy, same B: r_ion / r_e -> sqrt(M/m) (single-particle module).
    M = 400.0
    dt = 1e-3
    radii = []
    for q, m in ((-1.0, 1.0), (1.0, M)):
        v = math.sqrt(2 * 1.0 / m)          # same kinetic energy
        cfg = _orbit_cfg(qm_sign=q, mass=m, dt=dt)
        xs, _ = _track(cfg, 500.0, [v, 0.0, 0.0], 60 if m == 1.0 else 60)
        theta = 2 * math.atan(abs(q / m) * dt / 2)
        r = math.hypot(xs[1] - xs[0], 0) / (2 * math.sin(theta / 2))   # chord |v| dt
        radii.append(r)
    assert abs(radii[1] / radii[0] - math.sqrt(M)) < 1e-5 * math.sqrt(M)


def test_exb_drift_fixed_point_and_average():
    # E x B / B^2 = (0, E, 0) x (0, 0, B) / B^2 = (E/B, 0, 0).
    e, b = 0.7, 1.3
    ve = e / b
    k = 40                                        # steps per discrete gyration
    dt = 2.0 / b * math.tan(math.pi / k)          # theta = 2 pi / k exactly
    cfg = _orbit_cfg(bz=b, dt=dt, e_ext=(0, e, 0))
    cfg["species"][0]["charge"] = -1.0
    # fixed point: v = v_E stays v_E
    o = oracle.Oracle(cfg, load=False)
    o.set_particles(0, [10.0], [ve], [0.0], [0.0], [0])
    o.refresh_field()
    o.step(200)
    p = o.get_particles(0)
    assert abs(p["vx"][0] - ve) < 1e-13 and abs(p["vy"][0]) < 1e-13
    assert abs(p["x"][0] - (10.0 + 200 * dt * ve)) < 1e-9
    # perturbed: the mean over k steps of v_x equals v_E
    xs, _ = _track(cfg, 10.0, [ve + 0.9, -0.4, 0.2], 3 * k)
    vx = np.diff(xs) / dt
    for j in range(3):
        assert abs(vx[j * k:(j + 1) * k].mean() - ve) < 1e-10


# ---------------------------------------------------------------- field -----
def _field_oracle(bc, n_cells=50, length=2.0, eps0=1.3, v_amp=0.0, v_phase=0.0):
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=n_cells, bc=bc, length=length, dt=0.1, eps0=eps0,
                        v_amp=v_amp, v_freq=1.0, v_phase=v_phase, species=[sp])
    return oracle.Oracle(cfg, load=False), cfg


def test_dirichlet_uniform_charge_closed_form():
    V = 3.5
    o, cfg = _field_oracle(1, v_amp=V, v_phase=math.pi / 2)     # phi(0, t=0) = V
    L, eps0 = cfg["length"], cfg["eps0"]
    x = np.linspace(0, L, o.n_nodes)
    rho0 = 0.8
    phi, ef = o.poisson(0.0, np.full(o.n_nodes, rho0))
    phi_exact = rho0 * x * (L - x) / (2 * eps0) + V * (1 - x / L)
    e_exact = -rho0 * (L - 2 * x) / (2 * eps0) + V / L
    assert np.max(np.abs(phi - phi_exact)) < 1e-12 * np.max(np.abs(phi_exact))
    assert np.max(np.abs(ef - e_exact)) < 1e-11 * np.max(np.abs(e_exact))   # walls too


def test_dirichlet_drive_follows_sine():
    o, cfg = _field_oracle(1, v_amp=2.0)
    for t in (0.1, 0.3, 0.77):
        phi, _ = o.poisson(t, np.zeros(o.n_nodes))
        assert abs(phi[0] - 2.0 * math.sin(2 * math.pi * t)) < 1e-14
        assert phi[-1] == 0.0


@pytest.mark.parametrize("mode", [1, 3, 7])
def test_periodic_mode_closed_form(mode):
    o, cfg = _field_oracle(0, n_cells=64)
    L, eps0, n = cfg["length"], cfg["eps0"], o.n_nodes
    dx = L / n
    x = np.arange(n) * dx
    k = 2 * math.pi * mode / L
    K2 = 4 / dx ** 2 * math.sin(k * dx / 2) ** 2
    rho = 0.6 * np.cos(k * x) + 5.0                       # mean is removed
    phi, ef = o.poisson(0.0, rho)
    assert np.max(np.abs(phi - 0.6 * np.cos(k * x) / (eps0 * K2))) < 1e-11
    e_exact = 0.6 / (eps0 * K2) * np.sin(k * x) * math.sin(k * dx) / dx
    assert np.max(np.abs(ef - e_exact)) < 1e-11
    assert abs(phi.mean()) < 1e-13


def test_poisson_stencil_random_charge():
    for bc in (0, 1):
        o, cfg = _field_oracle(bc, n_cells=77, v_amp=1.0, v_phase=0.3)
        rng = np.random.default_rng(5)
        rho = rng.normal(size=o.n_nodes)
        phi, _ = o.poisson(0.0, rho)
        dx = cfg["length"] / cfg["n_cells"]
        if bc == 1:
            lap = (phi[:-2] - 2 * phi[1:-1] + phi[2:]) / dx ** 2
            assert np.max(np.abs(-lap * cfg["eps0"] - rho[1:-1])) < 1e-9
            assert phi[0] == pytest.approx(math.sin(0.3)) and phi[-1] == 0.0
        else:
            lap = (np.roll(phi, 1) - 2 * phi + np.roll(phi, -1)) / dx ** 2
            assert np.max(np.abs(-lap * cfg["eps0"] - (rho - rho.mean()))) < 1e-9


# ------------------------------------------------------------- weighting ----
@pytest.mark.parametrize("bc", [0, 1])
def test_lone_particle_cic(bc):
    o, cfg = _field_oracle(bc, n_cells=10, length=1.0, eps0=1.0)
    dx = 0.1
    for c, f in ((3, 0.25), (9, 0.625), (0, 0.0), (5, 0.5)):
        o.set_particles(0, [(c + f) * dx], [0.0], [0.0], [0.0], [0])
        o.refresh_field()
        n = o.density(0)
        vol = np.full(o.n_nodes, dx)
        if bc == 1:
            vol[0] = vol[-1] = dx / 2
        s = n * vol                                   # weight 1
        expect = np.zeros(o.n_nodes)
        expect[c] += 1 - f
        expect[(c + 1) % o.n_nodes if bc == 0 else c + 1] += f
        assert np.allclose(s, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("bc", [0, 1])
def test_lattice_loads_uniform_density(bc):
    # Partition of unity: a lattice of particles gives exactly uniform density,
    # wall nodes included (half volume).
    sp = W.species(-1.0, 1.0, 0.5, 800, 1.0, capacity=800, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=40, bc=bc, length=4.0, dt=0.1, eps0=1.0, species=[sp])
    o = oracle.Oracle(cfg, load=False)
    N = 800
    x = (np.arange(N) + 0.5) * 4.0 / N
    o.set_particles(0, x, np.zeros(N), np.zeros(N), np.zeros(N), np.arange(N))
    o.refresh_field()
    n = o.density(0)
    assert np.max(np.abs(n - 0.5 * N / 4.0)) < 1e-12 * 100


def test_charge_conservation_periodic_random():
    cfg = W.exb(n_per_species=5000, n_cells=64)
    o = oracle.Oracle(cfg)
    rho, _, _ = o.field()
    dx = cfg["length"] / cfg["n_cells"]
    total = sum(sp["charge"] * sp["weight"] * sp["n_init"] for sp in cfg["species"])
    assert abs(rho.sum() * dx - total) <= 1e-12 * abs(cfg["species"][0]["charge"] *
                                                        cfg["species"][0]["weight"] * 5000)
    for k in range(2):
        n = o.density(k)
        assert abs(n.sum() * dx - cfg["species"][k]["weight"] * 5000) < 1e-9 * 5000 * \
            cfg["species"][k]["weight"]


# ---------------------------------------------------------------- loading ---
def test_stratified_loading_one_particle_per_stratum():
    cfg = W.langmuir(eps=0.0, n_particles=4096)
    o = oracle.Oracle(cfg)
    x = o.get_particles(0)["x"]
    L = cfg["length"]
    j = np.floor(x / (L / 4096)).astype(int)
    assert np.array_equal(j, np.arange(4096))


def test_loaded_velocities_are_maxwellian():
    cfg = W.exb(n_per_species=20000, n_cells=32)
    cfg["species"][0]["vth"] = 1.0
    cfg["species"][0]["drift"] = [0.25, 0.0, -0.5]
    cfg["e_ext"] = [0, 0, 0]
    cfg["b_ext"] = [0, 0, 0]
    cfg["field_solve"] = 0          # v^{-1/2} = v^0 when no force acts
    o = oracle.Oracle(cfg)
    p = o.get_particles(0)
    for comp, d in (("vx", 0.25), ("vy", 0.0), ("vz", -0.5)):
        g = p[comp] - d
        assert stats.kstest(g, "norm").pvalue > 1e-3
        assert abs(g.mean()) < 5 / math.sqrt(20000)
        assert abs(g.var() - 1.0) < 5 * math.sqrt(2 / 20000)


def test_perturbed_loading_mode_amplitude():
    cfg = W.langmuir()                   # 1 % at mode 1, stratified
    o = oracle.Oracle(cfg)
    n = o.density(0)
    L = cfg["length"]
    x = np.arange(o.n_nodes) * L / o.n_nodes
    amp = 2 / o.n_nodes * np.sum(n * np.cos(2 * np.pi * x / L))
    assert abs(amp - 0.01) < 5e-4


def test_moments_of_a_drifting_beam():
    """A cold beam of velocity vd: flux n vd and momentum flux n vd^2 at every
    node (n the deposited density there), and volume integrals w N vd and
    w N vd^2 (half-cell volumes at walls)."""
    import oracle as O
    for bc in (0, 1):
        n, L, vd = 4096, 2.0, -0.37
        sp = [W.species(-1.0, 1.0, 0.5, n, 0.0, drift=(vd, 0.0, 0.0), load=W.LOAD_STRATIFIED)]
        cfg = W.base_config(n_cells=64, bc=bc, field_solve=0, length=L, species=sp)
        o = O.Oracle(cfg)
        flux, mom = o.moments(0)
        # partition of unity: the volume integrals are w N vd and w N vd^2
        dx = L / 64
        vol = np.full(len(flux), dx)
        if bc == 1:
            vol[0] = vol[-1] = 0.5 * dx
        assert np.sum(vol * flux) == pytest.approx(0.5 * n * vd, rel=1e-12)
        assert np.sum(vol * mom) == pytest.approx(0.5 * n * vd * vd, rel=1e-12)
        dens = o.density(0)
        np.testing.assert_allclose(flux, dens * vd, rtol=1e-12)
        np.testing.assert_allclose(mom, dens * vd * vd, rtol=1e-12)


def test_wall_energy_bookkeeping():
    """Free flight to the walls (no field, no gas): a particle reaches the
    wall its velocity points to, after N steps iff x0 + N vx dt leaves
    [0, L), carrying its own kinetic energy; each wall's energy is the sum of
    m w v^2 / 2 over those particles."""
    import oracle as O
    n, L, dt, N = 3000, 1.0, 0.05, 400
    sp = [W.species(-1.0, 2.0, 0.25, n, 1.0, load=W.LOAD_RANDOM)]
    cfg = W.base_config(n_cells=32, bc=1, field_solve=0, length=L, dt=dt, species=sp)
    o = O.Oracle(cfg)
    p = o.get_particles(0)
    e = 0.5 * 2.0 * 0.25 * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2)
    xN = p["x"] + N * p["vx"] * dt
    o.step(N)
    c = o.counters()
    assert c["absorbed"][0][0] == np.sum(xN < 0.0) and c["absorbed"][0][1] == np.sum(xN >= L)
    assert c["wall_energy"][0][0] == pytest.approx(e[xN < 0.0].sum(), rel=1e-12)
    assert c["wall_energy"][0][1] == pytest.approx(e[xN >= L].sum(), rel=1e-12)
    assert len(o.get_particles(0)["x"]) == np.sum((xN >= 0.0) & (xN < L))
