"""Seeded synthetic workloads shared by the oracle, the tests and the bench.

This module holds inputs only: physical constants, configuration records for the
runs the paper describes (a discharge is set up by gas, pressure, gap, voltage
waveform, magnetic field, walls and secondary emission, Section 1), the analytic
cross-section tables that stand in for the LXCat data the paper reads, and
seeded parameter draws.  None of the method's arithmetic (push, collisions,
deposition, field solve, collision-frequency bounds) lives here: both the
oracle and the GPU library compute everything derived from these records on
their own.

A configuration is a plain dict.  Keys:

  n_cells, bc (0 periodic, 1 Dirichlet), field_solve (1 Poisson, 0 imposed
  field only), length [m], dt [s], eps0, rho_bg (fixed background charge
  density), e_unit (charge unit used for energies in eV),
  v_amp, v_freq, v_phase (phi(0,t) = v_amp sin(2 pi v_freq t + v_phase),
  phi(L) = 0), e_ext[3], b_ext[3], gas_density [m^-3], gas_temp [K],
  gas_mass [kg], see_gamma, see_temp [eV], perturb_eps, perturb_mode, seed,
  species: list of {charge, mass, weight, capacity, n_init, vth, drift[3], load}

Species 0 is the electron species (it receives ionization and secondary
electrons); species 1, when present, is the ion species.
"""
from __future__ import annotations

import math

import numpy as np

# CODATA 2018 exact / recommended values (SI).
E_CHARGE = 1.602176634e-19
M_ELECTRON = 9.1093837015e-31
AMU = 1.66053906660e-27
EPS0 = 8.8541878128e-12
K_BOLTZMANN = 1.380649e-23
TORR = 133.322368421

LOAD_STRATIFIED = 0
LOAD_RANDOM = 1
LOAD_NONE = 2
DRIVE_VOLTAGE = 0
DRIVE_CAPACITOR = 1
DRIVE_CURRENT = 2
WAVE_SINE = 0
WAVE_TWO_HARMONIC = 1

XS_ELASTIC = 0
XS_EXCITATION = 1
XS_IONIZATION = 2
XS_ION_CX = 3
XS_ION_ISO = 4


def species(charge, mass, weight, n_init, vth, capacity=None, drift=(0.0, 0.0, 0.0),
            load=LOAD_STRATIFIED):
    if capacity is None:
        capacity = max(2 * int(n_init), 1024)
    return dict(charge=float(charge), mass=float(mass), weight=float(weight),
                capacity=int(capacity), n_init=int(n_init), vth=float(vth),
                drift=[float(d) for d in drift], load=int(load))


def base_config(**kw):
    cfg = dict(n_cells=128, bc=0, field_solve=1, length=1.0, dt=0.1, eps0=1.0,
               rho_bg=0.0, e_unit=1.0, v_amp=0.0, v_freq=0.0, v_phase=0.0,
               e_ext=[0.0, 0.0, 0.0], b_ext=[0.0, 0.0, 0.0], gas_density=0.0,
               gas_temp=300.0, gas_mass=0.0, see_gamma=0.0, see_temp=1.0,
               perturb_eps=0.0, perturb_mode=0, seed=1, species=[], renew_lz=0.0,
               drive=0, waveform=0, cap=0.0, j_amp=0.0)
    cfg.update(kw)
    return cfg


# --------------------------------------------------------------------------
# Langmuir wave in normalised units (Section 3.1): eps0 = e = m_e = n0 = 1, so
# omega_pe = 1 and, with v_th = sqrt(T/m) = 1, lambda_D = 1.
# --------------------------------------------------------------------------
def langmuir(k_lambda=0.3, n_cells=128, n_particles=65536, eps=0.01, mode=1,
             dt=0.1, seed=1, capacity=None):
    length = 2.0 * math.pi * mode / k_lambda
    w = length / n_particles            # n0 = 1
    el = species(-1.0, 1.0, w, n_particles, 1.0,
                 capacity=capacity if capacity else n_particles,
                 load=LOAD_STRATIFIED)
    return base_config(n_cells=n_cells, bc=0, length=length, dt=dt, eps0=1.0,
                       rho_bg=1.0, perturb_eps=eps, perturb_mode=mode, seed=seed,
                       species=[el])


# --------------------------------------------------------------------------
# Argon-like capacitive RF discharge (Section 3.2/3.3 type of run).
# --------------------------------------------------------------------------
AR_MASS = 39.948 * AMU
XE_MASS = 131.0 * AMU


def argon_table_energies(n=1000, e_lo=0.01, e_hi=1000.0):
    k = np.arange(n, dtype=np.float64)
    return e_lo * (e_hi / e_lo) ** (k / (n - 1))


def argon_tables(n=1000):
    """Synthetic cross sections standing in for the missing argon data.

    Elastic momentum transfer ~1e-19 m^2 with a Ramsauer-style dip near
    0.3 eV; one excitation (11.5 eV threshold); ionization (15.8 eV);
    isotropic-in-effect ion charge exchange 5e-19 m^2 (constant).
    """
    e = argon_table_energies(n)
    el = 1e-19 * (1.0 - 0.9 * np.exp(-np.log(e / 0.3) ** 2 / 0.5)) / (1.0 + e / 30.0)

    def thr(eth, amp):
        x = e / eth
        s = amp * (x - 1.0) / (x * x)
        s[x <= 1.0] = 0.0
        return s

    exc = thr(11.5, 4.0 * 1e-20)
    ion = thr(15.8, 4.0 * 3e-20)
    cx = np.full_like(e, 5e-19)
    return [
        dict(species=0, kind=XS_ELASTIC, threshold=0.0, energy=e, sigma=el),
        dict(species=0, kind=XS_EXCITATION, threshold=11.5, energy=e, sigma=exc),
        dict(species=0, kind=XS_IONIZATION, threshold=15.8, energy=e, sigma=ion),
        dict(species=1, kind=XS_ION_CX, threshold=0.0, energy=e, sigma=cx),
    ]


def gas_density(pressure_pa, temp_k=300.0):
    return pressure_pa / (K_BOLTZMANN * temp_k)


# Real particles per m^2 per macroparticle of the argon RF runs, fixed by a
# pilot run: a cold start of the 2.5 cm / 30 mTorr / 200 V discharge with
# 3e8 settled at about 4.5e4 macros per species after 250 periods, so 6.75e7
# gives about 2e5.  Sweeps use the same weight, so counts follow the physics.
PILOT_WEIGHT = 6.75e7
RF_DT = 1.0 / (13.56e6 * 1600)           # the time step of every RF run


def argon_rf(gap=0.025, n_cells=400, pressure_mtorr=30.0, v_amp=200.0,
             freq=13.56e6, steps_per_period=1600, n_init=100000, weight=None,
             see_gamma=0.1, te_ev=2.0, seed=2, capacity=None, dt=None):
    """Cold start: uniform quasi-neutral plasma, T_e = 2 eV, ions at T_g."""
    p_pa = pressure_mtorr * 1e-3 * TORR
    ng = gas_density(p_pa, 300.0)
    if dt is None:
        dt = 1.0 / (freq * steps_per_period)
    if weight is None:
        weight = PILOT_WEIGHT
    if capacity is None:
        capacity = max(8 * n_init, 1 << 20)
    vte = math.sqrt(te_ev * E_CHARGE / M_ELECTRON)
    vti = math.sqrt(K_BOLTZMANN * 300.0 / AR_MASS)
    el = species(-E_CHARGE, M_ELECTRON, weight, n_init, vte, capacity=capacity,
                 load=LOAD_RANDOM)
    io = species(E_CHARGE, AR_MASS, weight, n_init, vti, capacity=capacity,
                 load=LOAD_RANDOM)
    return base_config(n_cells=n_cells, bc=1, length=gap, dt=dt, eps0=EPS0,
                       e_unit=E_CHARGE, v_amp=v_amp, v_freq=freq, v_phase=0.0,
                       gas_density=ng, gas_temp=300.0, gas_mass=AR_MASS,
                       see_gamma=see_gamma, see_temp=1.0, seed=seed,
                       species=[el, io])


# --------------------------------------------------------------------------
# E x B drift-instability box (Section 3.6 type of run).  Axes: x azimuthal
# (simulated), B along y, imposed E along z, so v_E = -E/B along x.
# --------------------------------------------------------------------------
def exb(length=0.005, n_cells=1024, n_per_species=4_000_000, density=5e16,
        te_ev=10.0, ti_ev=0.2, e_field=2e4, b_field=0.02, dt=5e-12, seed=3,
        capacity=None):
    weight = density * length / n_per_species
    vte = math.sqrt(te_ev * E_CHARGE / M_ELECTRON)
    vti = math.sqrt(ti_ev * E_CHARGE / XE_MASS)
    v_e = e_field / b_field
    cap = capacity if capacity else n_per_species
    el = species(-E_CHARGE, M_ELECTRON, weight, n_per_species, vte, capacity=cap,
                 drift=(-v_e, 0.0, 0.0), load=LOAD_STRATIFIED)
    io = species(E_CHARGE, XE_MASS, weight, n_per_species, vti, capacity=cap,
                 load=LOAD_STRATIFIED)
    return base_config(n_cells=n_cells, bc=0, length=length, dt=dt, eps0=EPS0,
                       e_unit=E_CHARGE, e_ext=[0.0, 0.0, e_field],
                       b_ext=[0.0, b_field, 0.0], seed=seed, species=[el, io])


# --------------------------------------------------------------------------
# Electron cyclotron drift instability box (Section 3.6): the E x B box with
# the paper's reference fields and density, a whole number of resonant
# wavelengths lambda_1 = 2 pi v_E / omega_ce along the drift, and axial
# renewal after a virtual transit L_z.
# --------------------------------------------------------------------------
def lambda1(e_field=2e4, b_field=0.02):
    v_e = e_field / b_field
    return 2.0 * math.pi * v_e * M_ELECTRON / (E_CHARGE * b_field)


def ecdi(n_lambda=15, n_cells=1024, n_per_species=4_000_000, density=1e17, te_ev=10.0, ti_ev=0.2,
         e_field=2e4, b_field=0.02, lz=0.01, dt=5e-12, seed=11):
    cfg = exb(length=n_lambda * lambda1(e_field, b_field), n_cells=n_cells, n_per_species=n_per_species,
              density=density, te_ev=te_ev, ti_ev=ti_ev, e_field=e_field, b_field=b_field, dt=dt, seed=seed)
    cfg["renew_lz"] = lz
    return cfg


# --------------------------------------------------------------------------
# Maxwell-model swarm: electrons only, imposed uniform field, no Poisson,
# sigma(eps) = nu0 / (n_g v(eps)) so the collision frequency is constant.
# --------------------------------------------------------------------------
def maxwell_swarm(e_field=-1e3, nu0=1e9, n_particles=20000, gas_mass=AR_MASS * 1e6,
                  n_cells=64, length=0.01, dt=2e-11, seed=7, te_ev=0.5,
                  kind=XS_ELASTIC):
    ng = 1e22
    vte = math.sqrt(te_ev * E_CHARGE / M_ELECTRON)
    el = species(-E_CHARGE, M_ELECTRON, 1.0, n_particles, vte,
                 capacity=n_particles, load=LOAD_RANDOM)
    cfg = base_config(n_cells=n_cells, bc=0, field_solve=0, length=length, dt=dt,
                      eps0=EPS0, e_unit=E_CHARGE, e_ext=[e_field, 0.0, 0.0],
                      gas_density=ng, gas_temp=0.0, gas_mass=gas_mass, seed=seed,
                      species=[el])
    e = np.logspace(-4, 4, 2000)
    v = np.sqrt(2.0 * e * E_CHARGE / M_ELECTRON)
    tables = [dict(species=0, kind=kind, threshold=0.0, energy=e,
                   sigma=nu0 / (ng * v))]
    return cfg, tables


# --------------------------------------------------------------------------
# Parameter draws for sweeps of many discharges and for the warm-start model.
# --------------------------------------------------------------------------
def sweep_draws(n=64, seed=4):
    rng = np.random.default_rng(seed)
    p = np.exp(rng.uniform(np.log(10.0), np.log(200.0), n))    # mTorr
    v = rng.uniform(100.0, 400.0, n)                             # V
    gap = rng.uniform(0.015, 0.04, n)                            # m
    cells = np.rint(200 + 400 * (gap - 0.015) / 0.025).astype(int)
    return [dict(pressure_mtorr=float(p[i]), v_amp=float(v[i]), gap=float(gap[i]),
                 n_cells=int(cells[i]), freq=13.56e6, see_gamma=0.1)
            for i in range(n)]


# Steady-state particle counts of the argon configurations: about 2e5
# macro-particles per species for the single discharge, and counts between
# 5e4 and 2e6 per species (log-uniform, seeded) for the discharges of the
# sweep.  The throughput lines start from these counts instead of a cold start.
STEADY_COUNT_C2 = 200_000
STEADY_COUNT_RANGE = (5e4, 2e6)


def steady_counts(n, seed=40):
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(STEADY_COUNT_RANGE[0]), np.log(STEADY_COUNT_RANGE[1]), n))).astype(int)


def discharge_profile(m=64, te_ev=3.0, ti_ev=0.026):
    """Relative density and temperature (eV) of both species at m points over
    the gap, for a start at steady-state counts: a half-sine density, flat
    temperatures (electrons te_ev, ions at the gas temperature)."""
    x = (np.arange(m) + 0.5) / m
    dens = np.sin(np.pi * x)
    return np.stack([dens, dens]), np.stack([np.full(m, te_ev), np.full(m, ti_ev)])


def warm_draws(n, seed, f_range=(2e6, 60e6)):
    rng = np.random.default_rng(seed)
    p = np.exp(rng.uniform(np.log(10.0), np.log(200.0), n))
    v = rng.uniform(100.0, 400.0, n)
    f = np.exp(rng.uniform(np.log(f_range[0]), np.log(f_range[1]), n))
    gap = rng.uniform(0.015, 0.04, n)
    gamma = rng.uniform(0.0, 0.2, n)
    cells = np.rint(200 + 400 * (gap - 0.015) / 0.025).astype(int)
    return [dict(pressure_mtorr=float(p[i]), v_amp=float(v[i]), freq=float(f[i]),
                 gap=float(gap[i]), n_cells=int(cells[i]), see_gamma=float(gamma[i]))
            for i in range(n)]


def random_particles(cfg, s, n, seed, vscale=None):
    """Seeded random particle state (positions uniform in [0, L), Gaussian
    velocities of scale vth) for tests that start both sides from one state."""
    rng = np.random.default_rng(seed)
    sp = cfg["species"][s]
    vs = sp["vth"] if vscale is None else vscale
    x = rng.uniform(0.0, cfg["length"], n)
    v = rng.normal(0.0, vs, (3, n))
    ids = np.arange(n, dtype=np.uint32)
    return x, v[0].copy(), v[1].copy(), v[2].copy(), ids


# --------------------------------------------------------------------------
# Warm-start network: layer widths and seeded initial weights.
# --------------------------------------------------------------------------
WARM_WIDTHS = (5, 256, 256, 256, 768)


def mlp_init(widths=WARM_WIDTHS, seed=7):
    """Seeded initial parameters, flat, one [n_out][n_in + 1] block per layer
    (bias last): weights normal with variance 2 / n_in, biases zero."""
    rng = np.random.default_rng(seed)
    blocks = []
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        w = np.zeros((n_out, n_in + 1))
        w[:, :n_in] = rng.normal(0.0, math.sqrt(2.0 / n_in), (n_out, n_in))
        blocks.append(w.ravel())
    return np.concatenate(blocks)


def mlp_batch(n, n_in, n_out, seed):
    """Seeded inputs of unit scale and targets of unit scale for network tests."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 1.0, (n, n_in)), rng.normal(0.0, 1.0, (n, n_out))
