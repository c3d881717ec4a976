"""Pins of the oracle's start from profiles (orc_load_profiles) against the
definition of the inverse-CDF draw: the Philox draws and the stratified
formula for a uniform profile, the closed-form CDF of a linear profile, and
the local Maxwellian scale sqrt(e T(x) / m)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

SEED = 9


def cfg_free(n_cells=64, length=2.0, capacity=4096):
    # no field and no imposed fields: the leapfrog start leaves v unchanged
    sp = [W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=capacity, load=W.LOAD_NONE),
          W.species(1.0, 4.0, 1.0, 0, 1.0, capacity=capacity, load=W.LOAD_NONE)]
    return W.base_config(n_cells=n_cells, bc=1, field_solve=0, length=length, dt=0.1, eps0=1.0,
                         e_unit=1.0, seed=SEED, species=sp)


def draws(j, species, call):
    return oracle.philox([j, 0xFFFFFFFF, (species << 24) | call, 0], [SEED & 0xFFFFFFFF, SEED >> 32])


def normal_pair(u1, u2):
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2 * math.pi * u2), r * math.sin(2 * math.pi * u2)


def load(cfg, dens, temp, n):
    o = oracle.Oracle(cfg, load=False)
    o.load_profiles(dens, temp, n)
    return o


def test_uniform_profile_is_the_stratified_draw():
    cfg = cfg_free()
    m, n = 17, 500
    o = load(cfg, np.full((2, m), 3.0), np.full((2, m), 2.0), [n, n])
    P = o.get_particles(0)
    x, ids = P["x"], P["id"]
    L = cfg["length"]
    expect = np.array([(j + oracle.u01(draws(j, 0, 0)[0])) * L / n for j in range(n)])
    np.testing.assert_allclose(x, expect, rtol=0, atol=1e-13 * L)
    assert list(ids) == list(range(n))


def test_linear_profile_closed_form_cdf():
    cfg = cfg_free()
    m, n, a = 33, 800, 3.0
    L = cfg["length"]
    xs = np.linspace(0.0, L, m)
    dens = np.stack([1.0 + a * xs / L] * 2)
    o = load(cfg, dens, np.ones((2, m)), [n, 10])
    x = o.get_particles(0)["x"]
    F = (x + a * x * x / (2 * L)) / (L * (1 + a / 2))
    y = np.array([(j + oracle.u01(draws(j, 0, 0)[0])) / n for j in range(n)])
    np.testing.assert_allclose(F, y, rtol=0, atol=1e-12)


def test_local_maxwellian_scale():
    cfg = cfg_free()
    m, n = 9, 400
    L = cfg["length"]
    xs = np.linspace(0.0, L, m)
    temp = np.stack([0.5 + 4.0 * (xs / L) ** 2, np.full(m, 0.25)])
    o = load(cfg, np.ones((2, m)), temp, [n, n])
    for s, mass in ((0, 1.0), (1, 4.0)):
        P = o.get_particles(s)
        x, vx, vy, vz = P["x"], P["vx"], P["vy"], P["vz"]
        Tx = np.interp(x, xs, temp[s])          # linear between the points
        for j in range(0, n, 37):
            r1 = draws(j, s, 1)
            g0, g1 = normal_pair(oracle.u01(r1[0]), oracle.u01(r1[1]))
            g2, _ = normal_pair(oracle.u01(r1[2]), oracle.u01(r1[3]))
            vth = math.sqrt(Tx[j] / mass)
            assert vx[j] == pytest.approx(vth * g0, rel=1e-12, abs=1e-14)
            assert vy[j] == pytest.approx(vth * g1, rel=1e-12, abs=1e-14)
            assert vz[j] == pytest.approx(vth * g2, rel=1e-12, abs=1e-14)


def test_histogram_follows_profile():
    cfg = cfg_free(capacity=200_000)
    m, n = 65, 100_000
    L = cfg["length"]
    xs = np.linspace(0.0, L, m)
    dens = np.stack([np.sin(np.pi * xs / L) ** 2 + 0.05] * 2)
    o = load(cfg, dens, np.ones((2, m)), [n, 1])
    x = o.get_particles(0)["x"]
    edges = np.linspace(0.0, L, 21)
    h, _ = np.histogram(x, edges)
    # expected mass per bin from the linear interpolant, integrated finely
    fine = np.linspace(0.0, L, 200_001)
    dfine = np.interp(fine, xs, dens[0])
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dfine[1:] + dfine[:-1]) * np.diff(fine))])
    cdf /= cdf[-1]
    expect = np.diff(np.interp(edges, fine, cdf)) * n
    # stratified draws: counts within 1 of the expectation per bin
    assert np.abs(h - expect).max() <= 1.5


def test_rejects_bad_profiles():
    cfg = cfg_free()
    with pytest.raises(oracle.OracleError):
        load(cfg, -np.ones((2, 5)), np.ones((2, 5)), [10, 10])
    with pytest.raises(oracle.OracleError):
        load(cfg, np.zeros((2, 5)), np.ones((2, 5)), [10, 10])
