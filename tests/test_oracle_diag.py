"""Pins of the oracle's time-accumulated diagnostics (Section 1 lists
densities, potentials, mean energies and energy distributions among the
outputs): time-mean density, potential and electron mean energy at the
nodes, the bulk and wall electron energy histograms, and the per-species
impact-energy histograms at each wall.

Each pin is a case whose answer follows without the oracle: a frozen lattice
(no motion along x) keeps exactly uniform weights by the partition of unity
of linear weighting, a vacuum gap has a linear potential, and free flight to
the walls absorbs exactly the particles whose straight path leaves the gap.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

BINS = oracle.EEPF_BINS


def _frozen_lattice(bc, m_per_cell=8, n_cells=20, length=2.0, mass=2.0, weight=0.5, speeds=(1.0, 3.0)):
    """Electrons on a lattice of m_per_cell per cell, no velocity along x
    (speeds alternate between the given values, directions in the y-z plane),
    no field and no gas: nothing moves along x, so every step sees the same
    weights."""
    n = m_per_cell * n_cells
    sp = W.species(-1.0, mass, weight, 0, 1.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=n_cells, bc=bc, field_solve=0, length=length, dt=0.1, species=[sp])
    o = oracle.Oracle(cfg, load=False)
    x = (np.arange(n) + 0.3) * length / n
    rng = np.random.default_rng(3)
    ang = rng.uniform(0.0, 2.0 * math.pi, n)
    spd = np.where(np.arange(n) % 2 == 0, speeds[0], speeds[1])
    o.set_particles(0, x, np.zeros(n), spd * np.cos(ang), spd * np.sin(ang), np.arange(n))
    o.refresh_field()
    return o, cfg, x, spd


@pytest.mark.parametrize("bc", [0, 1])
def test_mean_energy_and_density_of_a_frozen_lattice(bc):
    # Two interleaved lattices of spacing 2 dx / m each carry density m/2 per
    # node (partition of unity), so the energy-weighted mean at every
    # interior node is the plain mean of the two energies, in every sample.
    mass, weight, m, nc, L = 2.0, 0.5, 8, 20, 2.0
    o, cfg, x, spd = _frozen_lattice(bc, m_per_cell=m, n_cells=nc, length=L, mass=mass, weight=weight)
    o.set_diag(True)
    o.step(5)
    a = o.avg()
    assert a["samples"] == 5.0
    dx = L / nc
    e1, e2 = 0.5 * mass * 1.0, 0.5 * mass * 9.0
    inner = slice(1, -1)
    np.testing.assert_allclose(a["mean_energy"][inner], 0.5 * (e1 + e2), rtol=1e-12)
    np.testing.assert_allclose(a["density"][0][inner], weight * m / dx, rtol=1e-12)
    # no field solve: the potential stays zero
    assert np.all(a["phi"] == 0.0)


def test_mean_energy_is_density_weighted_not_sample_averaged():
    # A lone electron at rest in the y-z plane inside one cell: its mean
    # energy at both neighbouring nodes is its own energy, whatever the
    # number of samples (a mean divided by the sample count would shrink).
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=4, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=10, bc=0, field_solve=0, length=1.0, dt=0.1, species=[sp])
    o = oracle.Oracle(cfg, load=False)
    o.set_particles(0, [0.33], [0.0], [2.0], [0.0], [0])
    o.set_diag(True)
    o.step(7)
    a = o.avg()
    me = a["mean_energy"]
    assert me[3] == pytest.approx(2.0, rel=1e-14) and me[4] == pytest.approx(2.0, rel=1e-14)
    assert np.count_nonzero(me) == 2
    # the mean density sums to one particle over the mesh
    assert np.sum(a["density"][0]) * 0.1 == pytest.approx(1.0, rel=1e-12)


def test_vacuum_potential_average():
    # No particles and a driven wall: phi_i(t) = V(t) (1 - i / N) exactly, so
    # the mean over steps 1..K is the mean of V(t_n) times the linear profile.
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    nc, dt, K, V, f, ph = 16, 0.013, 37, 3.0, 1.7, 0.4
    cfg = W.base_config(n_cells=nc, bc=1, field_solve=1, length=1.0, dt=dt, eps0=1.0, v_amp=V, v_freq=f,
                        v_phase=ph, species=[sp])
    o = oracle.Oracle(cfg, load=False)
    o.refresh_field()
    o.set_diag(True)
    o.step(K)
    a = o.avg()
    vmean = np.mean([V * math.sin(2 * math.pi * f * n * dt + ph) for n in range(1, K + 1)])
    np.testing.assert_allclose(a["phi"], vmean * (1.0 - np.arange(nc + 1) / nc), atol=1e-13 * V)
    assert np.all(a["density"] == 0.0) and np.all(a["mean_energy"] == 0.0)


def test_bulk_eepf_of_a_frozen_lattice():
    # Energies placed at bin centres with known counts; only the electrons in
    # the middle tenth of a bounded gap count, once per sample.
    nc, L, n, mass, emax = 40, 4.0, 400, 1.0, 32.0
    width = emax / BINS
    sp = W.species(-1.0, mass, 1.0, 0, 1.0, capacity=n, load=W.LOAD_NONE)
    cfg = W.base_config(n_cells=nc, bc=1, field_solve=0, length=L, dt=0.1, species=[sp])
    o = oracle.Oracle(cfg, load=False)
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, L, n)
    bins = rng.integers(0, BINS + 20, n)           # a few beyond the range
    eps = (bins + 0.5) * width
    vy = np.sqrt(2.0 * eps / mass)
    o.set_particles(0, x, np.zeros(n), vy, np.zeros(n), np.arange(n))
    o.set_diag(True, eepf_emax=emax)
    o.step(3)
    h = o.eepf()
    cells = np.floor(x / (L / nc)).astype(int)
    lo, hi = math.floor(0.45 * nc), math.ceil(0.55 * nc)
    sel = (cells >= lo) & (cells < hi) & (bins < BINS)
    want = 3 * np.bincount(bins[sel], minlength=BINS)[:BINS]
    np.testing.assert_array_equal(h["bulk"], want)
    assert np.all(h["wall"] == 0.0)
    assert h["bin_width"] == width and h["samples"] == 3.0


def test_wall_energy_distributions_free_flight():
    # Free flight to the walls: after N steps the absorbed particles of each
    # wall are those whose straight path x0 + N vx dt has left [0, L); each
    # contributes its own (unchanged) energy to that wall's histogram.
    n, L, dt, N = 4000, 1.0, 0.05, 300
    m_e, m_i = 1.0, 50.0
    sp = [W.species(-1.0, m_e, 0.25, n, 3.0, load=W.LOAD_RANDOM),
          W.species(1.0, m_i, 0.25, n, 0.6, load=W.LOAD_RANDOM)]
    cfg = W.base_config(n_cells=32, bc=1, field_solve=0, length=L, dt=dt, species=sp)
    o = oracle.Oracle(cfg)
    e_max = (20.0, 40.0)
    o.set_diag(True, eepf_emax=12.0)
    o.set_wall_edf(0, e_max[0])
    o.set_wall_edf(1, e_max[1])
    h = o.wall_edf()
    assert np.all(h["counts"] == 0.0)
    want = []
    for s, mass in enumerate((m_e, m_i)):
        p = o.get_particles(s)
        e = 0.5 * mass * (p["vx"] ** 2 + p["vy"] ** 2 + p["vz"] ** 2)
        xN = p["x"] + N * p["vx"] * dt
        want.append((e, xN))
    o.step(N)
    h = o.wall_edf()
    c = o.counters()
    for s in range(2):
        e, xN = want[s]
        w = e_max[s] / BINS
        assert h["bin_width"][s] == w
        for wall, hit in ((0, xN < 0.0), (1, xN >= L)):
            b = np.floor(e[hit] / w).astype(int)
            ref = np.bincount(b[b < BINS], minlength=BINS)[:BINS]
            np.testing.assert_array_equal(h["counts"][s][wall], ref)
            assert c["absorbed"][s][wall] == hit.sum()
    # the wall electron energy distribution is the electrons of both walls
    # over the electron range
    e, xN = want[0]
    hit = (xN < 0.0) | (xN >= L)
    b = np.floor(e[hit] / (12.0 / BINS)).astype(int)
    np.testing.assert_array_equal(o.eepf()["wall"], np.bincount(b[b < BINS], minlength=BINS)[:BINS])


def test_reset_clears_every_accumulator():
    o, cfg, x, spd = _frozen_lattice(1)
    o.set_diag(True)
    o.step(2)
    o.reset_avg()
    a, h, w = o.avg(), o.eepf(), o.wall_edf()
    assert a["samples"] == 0.0 and np.all(a["density"] == 0.0) and np.all(a["mean_energy"] == 0.0)
    assert np.all(h["bulk"] == 0.0) and np.all(w["counts"] == 0.0)
    o.step(1)
    assert o.avg()["samples"] == 1.0


def test_diagnostics_off_by_default():
    o, cfg, x, spd = _frozen_lattice(0)
    o.step(2)
    assert o.avg()["samples"] == 0.0 and np.all(o.eepf()["bulk"] == 0.0)


def test_births_enter_the_energy_profile():
    # Ions flying into the walls with secondary yield 1 and no electrons to
    # start: after one step the only electrons are that step's secondaries.
    # The energy profile integrates (partition of unity) to w times their
    # total energy, so births are sampled like every other electron.
    n, L, nc = 3000, 1.0, 32
    m_e, m_i, w = 1.0, 40.0, 0.5
    sp = [W.species(-1.0, m_e, w, 0, 1.0, capacity=4 * n, load=W.LOAD_NONE),
          W.species(1.0, m_i, w, n, 2.0, load=W.LOAD_RANDOM)]
    cfg = W.base_config(n_cells=nc, bc=1, field_solve=0, length=L, dt=0.2, see_gamma=1.0, see_temp=0.5,
                        species=sp)
    o = oracle.Oracle(cfg)
    o.set_diag(True)
    ions = o.get_particles(1)
    o.step(1)
    c = o.counters()
    e = o.get_particles(0)
    assert len(e["x"]) == c["see_emitted"].sum() > 0
    eps = 0.5 * m_e * (e["vx"] ** 2 + e["vy"] ** 2 + e["vz"] ** 2)
    a = o.avg()
    vol = np.full(nc + 1, L / nc)
    vol[0] = vol[-1] = 0.5 * L / nc
    assert np.sum(vol * a["density"][0] * a["mean_energy"]) == pytest.approx(w * eps.sum(), rel=1e-12)
    # and each ion is in its wall's histogram at its own (unchanged) energy
    ei = 0.5 * m_i * (ions["vx"] ** 2 + ions["vy"] ** 2 + ions["vz"] ** 2)
    x1 = ions["x"] + ions["vx"] * 0.2
    h = o.wall_edf()
    for wall, hit in ((0, x1 < 0.0), (1, x1 >= L)):
        b = np.floor(ei[hit] / h["bin_width"][1]).astype(int)
        np.testing.assert_array_equal(h["counts"][1][wall], np.bincount(b[b < BINS], minlength=BINS)[:BINS])
