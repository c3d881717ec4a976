"""The oracle's parallel step (OpenMP over fixed chunks of 4096 particles,
merged in chunk order) against itself at 1, 2 and 8 threads and against the
sequential step.

Thread-count invariance is exact: particles, ids, counters, births, fields,
energies and every sampled diagnostic are identical bit for bit.  Against
the sequential step, one step from the same state moves every particle by the
same arithmetic, so particles, ids and integer counters agree exactly and the
chunked floating-point sums (deposit, kinetic and wall energies) agree to
rounding."""
import numpy as np
import pytest

import oracle
import workloads as W


def _argon():
    # hot electrons in a dense gas and fast ions: ionization births, wall
    # losses and secondary electrons within a few tens of steps
    cfg = W.argon_rf(n_init=30000, seed=9, capacity=120000, weight=2e9, te_ev=20.0, pressure_mtorr=300.0)
    cfg["species"][1]["vth"] = 4e4
    return cfg, W.argon_tables()


def _state(o, S):
    out = {}
    for s in range(S):
        p = o.get_particles(s)
        for k in ("x", "vx", "vy", "vz", "id"):
            out["%d_%s" % (s, k)] = p[k]
    c = o.counters()
    for k, v in c.items():
        out["cnt_" + k] = np.asarray(v)
    rho, phi, ef = o.field()
    out.update(rho=rho, phi=phi, ef=ef)
    ke, fe = o.energy()
    out.update(ke=np.asarray(ke), fe=np.asarray(fe))
    return out


def _run(cfg, tabs, threads, steps, diag=True):
    o = oracle.Oracle(cfg, tabs)
    if diag:
        o.set_diag(True)
    o.set_threads(threads)
    o.step(steps)
    st = _state(o, len(cfg["species"]))
    if diag:
        a = o.avg()
        st["avg_density"] = a["density"]
        st["avg_phi"] = a["phi"]
        st["avg_energy"] = a["mean_energy"]
        e = o.eepf()
        st["eepf_bulk"] = e["bulk"]
        st["eepf_wall"] = e["wall"]
        st["wall_edf"] = o.wall_edf()["counts"]
    return st


@pytest.mark.parametrize("which", ["argon", "exb_renewal"])
def test_parallel_step_is_thread_count_invariant(which):
    if which == "argon":
        cfg, tabs = _argon()
        steps = 40
    else:
        cfg, tabs = W.exb(n_per_species=20000, n_cells=128), ()
        cfg["renew_lz"] = 2e-5
        steps = 30
    ref = _run(cfg, tabs, 1, steps)
    assert sum(len(v) for k, v in ref.items() if k.endswith("_id")) > 3 * 4096
    if which == "argon":
        assert ref["cnt_candidates"].sum() > 0 and ref["cnt_absorbed"].sum() > 0
        assert ref["cnt_see_emitted"].sum() > 0 and ref["cnt_coll"][0, 2] > 0   # secondaries, ionizations
    else:
        assert ref["cnt_renewed"].sum() > 0
    for n in (2, 8):
        other = _run(cfg, tabs, n, steps)
        assert other.keys() == ref.keys()
        for k in ref:
            assert np.array_equal(ref[k], other[k]), (n, k)


def test_parallel_step_matches_sequential_step():
    cfg, tabs = _argon()
    seq = oracle.Oracle(cfg, tabs)
    seq.step(20)
    par = oracle.Oracle(cfg, tabs, load=False)
    for s in range(2):
        p = seq.get_particles(s)
        par.set_particles(s, p["x"], p["vx"], p["vy"], p["vz"], p["id"], p["next_id"])
    par.set_step(seq.step_index)
    par.refresh_field()
    c0 = seq.counters()
    par.set_threads(4)
    seq.step(1)
    par.step(1)
    for s in range(2):
        a, b = seq.get_particles(s), par.get_particles(s)
        for k in ("x", "vx", "vy", "vz", "id"):
            assert np.array_equal(a[k], b[k]), (s, k)
    ca, cb = seq.counters(), par.counters()
    for k in ("absorbed", "see_emitted", "candidates", "nulls", "coll", "violations", "renewed"):
        assert np.array_equal(np.asarray(ca[k]) - np.asarray(c0[k]), np.asarray(cb[k])), k
    ra, pa, _ = seq.field()
    rb, pb, _ = par.field()
    np.testing.assert_allclose(rb, ra, rtol=1e-12, atol=1e-12 * np.abs(ra).max())
    np.testing.assert_allclose(pb, pa, rtol=1e-11, atol=1e-11 * np.abs(pa).max())
    np.testing.assert_allclose(par.energy()[0], np.asarray(seq.energy()[0]), rtol=1e-12)
