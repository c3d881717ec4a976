"""Power-decomposition moments on the GPU (PIC_DIAG_POWER) against the
oracle's moments of the same state: one diagnostic step from identical
states, so the time mean is the single step's value."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import small_argon, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def check(sim, o, cfg):
    pw = sim.power()
    assert pw["samples"] == 1.0
    ef = o.field()[2]
    for s in range(len(cfg["species"])):
        fo, mo = o.moments(s)
        dens = o.density(s)
        vth = max(cfg["species"][s]["vth"], 1e-30)
        scale_f = max(dens.max(), 1e-300) * vth * 10
        scale_m = max(dens.max(), 1e-300) * vth * vth * 100
        assert np.max(np.abs(pw["flux"][s] - fo)) <= 1e-5 * scale_f
        assert np.max(np.abs(pw["momentum"][s] - mo)) <= 1e-5 * scale_m
        po = cfg["species"][s]["charge"] * fo * ef
        assert np.max(np.abs(pw["power"][s] - po)) <= 1e-4 * max(np.max(np.abs(po)), 1e-300) + \
            1e-5 * scale_f * abs(cfg["species"][s]["charge"]) * np.max(np.abs(ef))


def test_power_moments_bounded_with_collisions(pic):
    cfg, tabs = small_argon(n_init=20000)
    sim = pic.Sim(cfg, tabs)
    sim.step(400)                                   # a developed, non-uniform state
    o = to_oracle(sim, cfg, tabs)
    sim.set_diag(True)
    sim.reset_avg()
    sim.step(1)
    o.step(1)
    check(sim, o, cfg)


def test_power_moments_periodic_streaming(pic):
    cfg = W.langmuir(n_particles=65536)
    sim = pic.Sim(cfg)
    sim.step(20)
    o = to_oracle(sim, cfg)
    sim.set_diag(True)
    sim.reset_avg()
    sim.step(1)
    o.step(1)
    check(sim, o, cfg)


def test_wall_energy_free_flight(pic):
    """Free flight (no field, no gas) from identical states: counts and
    energies per wall against the oracle."""
    n, L = 200_000, 0.02
    sp = [W.species(-1.602176634e-19, 9.1093837e-31, 1e8, n, 1e6, load=W.LOAD_RANDOM),
          W.species(1.602176634e-19, 6.6e-26, 1e8, n, 2e3, load=W.LOAD_RANDOM)]
    cfg = W.base_config(n_cells=200, bc=1, field_solve=0, length=L, dt=1e-10, eps0=8.8541878128e-12,
                        e_unit=1.602176634e-19, species=sp, seed=5)
    sim = pic.Sim(cfg)
    o = to_oracle(sim, cfg)
    sim.step(100)
    o.step(100)
    we = sim.wall_energy()
    c = o.counters()
    absorbed = sim.wall()["absorbed"]
    for s in range(2):
        for w in range(2):
            ref, k = c["wall_energy"][s][w], int(c["absorbed"][s][w])
            # a particle within an FP32 rounding of the wall may land on either side
            assert abs(int(absorbed[s][w]) - k) <= 2
            assert abs(we[s][w] - ref) <= 1e-5 * ref + 3.0 * ref / max(k, 1)


def _close_hist(hg, ho, what, per_bin=2, frac=1e-3):
    """Histograms filled on the GPU (FP32 energies) and in the oracle (FP64):
    an energy within rounding of a bin edge may fall on either side, so bins
    differ by at most a few counts and the totals by a small fraction."""
    hg, ho = np.asarray(hg), np.asarray(ho)
    assert np.max(np.abs(hg - ho)) <= per_bin, what
    assert abs(hg.sum() - ho.sum()) <= frac * ho.sum() + per_bin, what


def test_time_averages_and_distributions_match_oracle(pic):
    """One diagnostic step from identical states (argon with collisions, walls
    and secondaries): time-mean densities, potential and electron mean energy,
    bulk and wall electron energy distributions and the per-wall impact
    energy histograms of both species, against the oracle."""
    cfg, tabs = small_argon(n_init=20000)
    sim = pic.Sim(cfg, tabs)
    sim.step(400)
    o = to_oracle(sim, cfg, tabs)
    for x in (sim, o):
        x.set_diag(True, eepf_emax=32.0)
        x.set_wall_edf(0, 48.0)
        x.set_wall_edf(1, 400.0)
    sim.reset_avg()
    sim.step(1)
    o.step(1)
    ag, ao = sim.avg(), o.avg()
    assert ag["samples"] == ao["samples"] == 1.0
    for s in range(2):
        ref = ao["density"][s]
        assert np.max(np.abs(ag["density"][s] - ref)) <= 1e-5 * ref.max()
    assert np.max(np.abs(ag["phi"] - ao["phi"])) <= 1e-5 * np.max(np.abs(ao["phi"]))
    ne = ao["density"][0]
    sig = ne >= 0.01 * ne.max()
    np.testing.assert_allclose(ag["mean_energy"][sig], ao["mean_energy"][sig], rtol=1e-4)
    hg, ho = sim.eepf(), o.eepf()
    assert hg["bin_width"] == ho["bin_width"] and hg["samples"] == ho["samples"] == 1.0
    assert ho["bulk"].sum() > 100
    _close_hist(hg["bulk"], ho["bulk"], "bulk EEPF")
    _close_hist(hg["wall"], ho["wall"], "wall EEPF")
    wg, wo = sim.wall_edf(), o.wall_edf()
    np.testing.assert_array_equal(wg["bin_width"], wo["bin_width"])
    for s in range(2):
        for w in range(2):
            _close_hist(wg["counts"][s][w], wo["counts"][s][w], f"wall edf {s} {w}")


def test_wall_edf_free_flight(pic):
    """Free flight into the walls over 100 steps: the impact-energy
    histograms of both species at both walls against the oracle, and their
    totals against the absorption counters."""
    n, L = 200_000, 0.02
    sp = [W.species(-1.602176634e-19, 9.1093837e-31, 1e8, n, 1e6, load=W.LOAD_RANDOM),
          W.species(1.602176634e-19, 6.6e-26, 1e8, n, 2e3, load=W.LOAD_RANDOM)]
    cfg = W.base_config(n_cells=200, bc=1, field_solve=0, length=L, dt=1e-10, eps0=8.8541878128e-12,
                        e_unit=1.602176634e-19, species=sp, seed=5)
    sim = pic.Sim(cfg)
    o = to_oracle(sim, cfg)
    for x in (sim, o):
        x.set_diag(True, eepf_emax=16.0)
        x.set_wall_edf(0, 40.0)
        x.set_wall_edf(1, 2.0)
    sim.step(100)
    o.step(100)
    wg, wo = sim.wall_edf(), o.wall_edf()
    absorbed = sim.wall()["absorbed"]
    for s in range(2):
        for w in range(2):
            assert wo["counts"][s][w].sum() > (1000 if s == 0 else 20)
            _close_hist(wg["counts"][s][w], wo["counts"][s][w], f"wall edf {s} {w}")
            assert wg["counts"][s][w].sum() <= absorbed[s][w]
    _close_hist(sim.eepf()["wall"], o.eepf()["wall"], "wall EEPF")
    sim.reset_avg()
    assert np.all(sim.wall_edf()["counts"] == 0.0)


def test_batched_diagnostics_equal_single_runs(pic):
    """Discharges of different meshes in one context: each one's time
    averages, energy distributions (bulk window of its own mesh) and wall
    histograms equal those of a run of that discharge alone, bit for bit."""
    cfgs = []
    for i, (n, nc, gap, v) in enumerate(((8000, 200, 0.015, 150.0), (15000, 317, 0.021, 320.0))):
        cfgs.append(W.argon_rf(n_init=n, n_cells=nc, gap=gap, v_amp=v, seed=100 + i, capacity=4 * n,
                               weight=3e13 / n))
    tabs = W.argon_tables()
    batch = pic.Sim(cfgs, tabs)
    batch.set_diag(True, eepf_emax=40.0)
    batch.step(96)
    for b, cfg in enumerate(cfgs):
        one = pic.Sim(cfg, tabs)
        one.set_diag(True, eepf_emax=40.0)
        one.step(96)
        ab, ao = batch.avg(b), one.avg()
        for k in ("density", "phi", "mean_energy"):
            assert np.array_equal(ab[k], ao[k]), (b, k)
        eb, eo = batch.eepf(b), one.eepf()
        assert eo["bulk"].sum() > 0
        assert np.array_equal(eb["bulk"], eo["bulk"]) and np.array_equal(eb["wall"], eo["wall"]), b
        assert np.array_equal(batch.wall_edf(b)["counts"], one.wall_edf()["counts"]), b
        one.close()


def test_wall_edf_rejects_bad_ranges(pic):
    cfg, tabs = small_argon(n_init=2000)
    sim = pic.Sim(cfg, tabs)
    for s, e in ((2, 10.0), (-1, 10.0), (0, 0.0), (1, float("nan")), (0, float("inf"))):
        with pytest.raises(RuntimeError):
            sim.set_wall_edf(s, e)


def test_power_decomposition_matches_oracle(pic):
    """The decomposition of q Gamma E into inertia, pressure and the ohmic
    rest (momentum balance times Gamma / n), GPU against oracle: from
    identical states one sampled step stores the flux, then one more gives a
    sample with the time derivative.  Compared where the species' density is
    at least 5 % of its maximum (the terms divide by n)."""
    cfg, tabs = small_argon(n_init=20000)
    sim = pic.Sim(cfg, tabs)
    sim.step(400)
    o = to_oracle(sim, cfg, tabs)
    sim.set_diag(True)
    o.set_diag(True)
    sim.step(1)
    o.step(1)
    sim.reset_avg()
    o.reset_avg()
    sim.step(1)
    o.step(1)
    pw = sim.power()
    assert pw["samples"] == 1.0
    for s in range(2):
        po = o.power(s)
        dens = o.density(s)
        keep = dens >= 0.05 * dens.max()
        for what in ("power", "inertia", "pressure", "ohmic"):
            g, r = pw[what][s], po[what]
            scale = np.max(np.abs(po["power"][keep]))
            err = np.max(np.abs(g - r)[keep]) / scale
            print("species %d %-8s max |GPU - oracle| / max|q Gamma E| = %.3g" % (s, what, err), flush=True)
            assert err <= 1e-4, (s, what, err)
        # the closure holds on each side
        np.testing.assert_allclose(pw["inertia"][s] + pw["pressure"][s] + pw["ohmic"][s], pw["power"][s],
                                   rtol=1e-12, atol=1e-12 * np.max(np.abs(pw["power"][s])))
