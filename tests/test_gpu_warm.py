"""GPU start from profiles (pic_load_profiles) against the oracle's
(orc_load_profiles): positions, velocities after the leapfrog start, ids,
densities and field; then a few steps of the warm-started discharge."""
import numpy as np
import pytest

import oracle
from gpu_helpers import compare_species, small_argon

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def profiles(cfg, m=256):
    xs = np.linspace(0.0, 1.0, m)
    ne = 1e15 * (np.sin(np.pi * xs) ** 1.5 + 0.02)
    ni = 1e15 * (np.sin(np.pi * xs) ** 1.2 + 0.05)
    te = 1.5 + 3.0 * (1.0 - np.sin(np.pi * xs))          # eV, hotter near the walls
    ti = np.full(m, 300.0 * 1.380649e-23 / 1.602176634e-19)
    return np.stack([ne, ni]), np.stack([te, ti])


def test_profile_load_matches_oracle(pic):
    cfg, tabs = small_argon(n_init=5000)          # capacity 40000
    dens, temp = profiles(cfg)
    n = [30001, 27777]                                    # ragged: not whole tiles
    sim = pic.Sim(cfg, tabs)
    sim.load_profiles(dens, temp, n)
    o = oracle.Oracle(cfg, tabs, load=False)
    o.load_profiles(dens, temp, n)
    for s in range(2):
        pg, po = sim.get_particles(s), o.get_particles(s)
        assert len(pg["id"]) == n[s] and pg["next_id"] == n[s]
        vs = np.sqrt(temp[s].max() * 1.602176634e-19 / cfg["species"][s]["mass"])
        r = compare_species(pg, po, cfg, vs)
        assert r["id_equal"] and r["cell_mismatch"] == 0
        assert r["max_dx_over_dx"] < 1e-5
        assert r["max_rel_v"] < 1e-6
        dg, do = sim.density()[s], o.density(s)
        assert np.max(np.abs(dg - do)) <= 1e-5 * np.max(do)
    eg, eo = sim.efield(), o.field()[2]
    assert np.max(np.abs(eg - eo)) <= 1e-5 * np.max(np.abs(eo))


def test_warm_started_steps_match_oracle(pic):
    cfg, tabs = small_argon(n_init=5000)
    dens, temp = profiles(cfg)
    n = [20000, 20000]
    sim = pic.Sim(cfg, tabs)
    sim.load_profiles(dens, temp, n)
    o = oracle.Oracle(cfg, tabs, load=False)
    o.load_profiles(dens, temp, n)
    sim.step(3)
    o.step(3)
    for s in range(2):
        pg, po = sim.get_particles(s), o.get_particles(s)
        assert len(pg["id"]) == len(po["id"])
        assert np.array_equal(pg["id"], po["id"])


def test_profile_load_rejects_bad_input(pic):
    cfg, tabs = small_argon(n_init=1000)
    sim = pic.Sim(cfg, tabs)
    dens, temp = profiles(cfg, m=16)
    with pytest.raises(pic.PicError):
        sim.load_profiles(-dens, temp, [10, 10])
    with pytest.raises(pic.PicError):
        sim.load_profiles(dens, temp, [10, cfg["species"][1]["capacity"] + 1])
    with pytest.raises(pic.PicError):
        sim.load_profiles(np.zeros_like(dens), temp, [10, 10])
    # nothing changed
    assert sim.counts()["count"] == [1000, 1000]
