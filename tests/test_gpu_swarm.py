"""Swarm mode on the GPU (Section 4): one step of an electrons-only ionizing
swarm against the oracle from identical states, the Maxwell model's drift
and mean energy against the discrete closed forms (the same relations the
oracle is pinned by), and the trends of the argon coefficients with E/N."""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from gpu_helpers import compare_species, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def test_electrons_only_ionization_step_matches_oracle(pic):
    from paper_2609_17151_amd import swarm
    tabs = swarm.electron_tables(W.argon_tables())
    cfg = swarm.config(800.0, 3.22e22, 50_000, 2e-12, seed=5, te_ev=30.0)
    sim = pic.Sim(cfg, tabs)
    sim.step(20)
    o = to_oracle(sim, cfg, tabs)
    sim.step(1)
    o.step(1)
    pg, po = sim.get_particles(0), o.get_particles(0)
    cg, co = sim.coll()["coll"][0], o.counters()["coll"][0]
    assert co[2] > 0                                 # ionizations happened
    assert abs(len(pg["id"]) - len(po["id"])) <= 1
    common = min(len(pg["id"]), len(po["id"]))
    r = compare_species({k: v[:common] for k, v in pg.items() if k != "next_id"},
                        {k: v[:common] for k, v in po.items() if k != "next_id"}, cfg,
                        cfg["species"][0]["vth"])
    ok = (r["rel_v"] < 1e-5) & (r["dx"] < 1e-6 * cfg["length"])
    assert ok.mean() >= 0.9999
    assert sim.counts()["count"] == [len(pg["id"])]


def test_maxwell_model_on_gpu(pic):
    from paper_2609_17151_amd import swarm
    E, nu0, dt, mr, ng = 1e3, 1e9, 2e-11, 20.0, 1e22
    e = np.logspace(-4, 4, 2000)
    v = np.sqrt(2.0 * e * W.E_CHARGE / W.M_ELECTRON)
    tabs = [dict(species=0, kind=W.XS_ELASTIC, threshold=0.0, energy=e, sigma=nu0 / (ng * v))]
    en_td = E / ng / swarm.TD
    sw = swarm.Swarm([en_td], replicas=4, n=100_000, tables=tabs, n_gas=ng, dt=dt, gas_mass=mr * W.M_ELECTRON,
                     gas_temp=0.0)
    out = sw.run(3072, 4096, every=256)
    numax, _ = sw.sim.numax(0)
    p = (1.0 - math.exp(-numax * dt)) * nu0 / numax
    beta = 2.0 / mr
    f = 0.5 * integrate.quad(lambda c: c * math.sqrt(1.0 - beta * (1.0 - c)), -1.0, 1.0)[0]
    a = W.E_CHARGE * E / W.M_ELECTRON
    q = 1.0 - p * (1.0 - f)
    ws = q * a * dt / (1.0 - q)
    eps_pre = W.M_ELECTRON * a * dt * (ws + 0.5 * a * dt) / (p * beta)
    # the swarm samples the state after the collision stage: energy
    # eps_pre (1 - p beta), velocity W_s
    assert out["W"][0] == pytest.approx(ws, rel=0.01)
    assert out["energy"][0] == pytest.approx(eps_pre * (1.0 - p * beta) / W.E_CHARGE, rel=0.01)
    assert out["rates"][0][0] == pytest.approx(p / (ng * dt), rel=0.01)


def test_argon_coefficients_trend_with_e_over_n(pic):
    from paper_2609_17151_amd import swarm
    sw = swarm.Swarm([100.0, 300.0, 1000.0], replicas=4, n=50_000)
    out = sw.run(32768, 8192, every=128)
    w, eps, k = out["W"], out["energy"], out["rates"]
    assert np.all(np.diff(w) > 0) and np.all(np.diff(eps) > 0)
    assert np.all(w > 0)
    assert np.all(np.diff(k[:, 2]) >= 0) and k[-1, 2] > 0    # ionization grows with E/N
    assert np.all(out["W_err"] < 0.05 * w) and np.all(out["energy_err"] < 0.05 * eps)
    for i in range(3):
        h = out["eepf"][i]
        assert abs(h.sum() * 40.0 / 256 - 1.0) < 1e-9 or h.sum() == 0.0


def test_device_thinning_keeps_an_unbiased_ordered_subset(pic):
    # two discharges: the larger one above the threshold is thinned, each
    # particle kept with probability keep / live; the smaller one is left as it is
    big, small = W.langmuir(n_particles=20000, seed=3), W.langmuir(n_particles=5000, seed=4)
    sim = pic.Sim([big, small])
    sim.step(3)
    before = [sim.get_particles(0, b) for b in range(2)]
    sim.thin(0, 10000, 8000)
    after = [sim.get_particles(0, b) for b in range(2)]
    # untouched below the threshold
    for k in ("cell", "off", "vx", "vy", "vz", "id"):
        assert np.array_equal(after[1][k], before[1][k]), k
    # the survivors: the same particles, in their order, ids and next id kept
    n = len(after[0]["id"])
    sigma = math.sqrt(20000 * 0.4 * 0.6)
    assert abs(n - 8000) < 5 * sigma, n
    idx = np.searchsorted(before[0]["id"], after[0]["id"])
    assert np.all(np.diff(after[0]["id"].astype(np.int64)) > 0)
    assert np.array_equal(before[0]["id"][idx], after[0]["id"])
    for k in ("cell", "off", "vx", "vy", "vz"):
        assert np.array_equal(before[0][k][idx], after[0][k]), k
    assert after[0]["next_id"] == before[0]["next_id"]
    # an unbiased subset: the mean velocity moves by sampling noise only
    sd = np.std(before[0]["vx"]) * math.sqrt((1.0 - n / 20000) / n)
    assert abs(np.mean(after[0]["vx"]) - np.mean(before[0]["vx"])) < 5 * sd
    # the store stays consistent: more steps, no flags, the same thinning twice
    sim.step(5)
    assert sim.flags(0) == 0 and sim.flags(1) == 0
    twin = pic.Sim([big, small])
    twin.step(3)
    twin.thin(0, 10000, 8000)
    assert np.array_equal(twin.get_particles(0, 0)["id"], after[0]["id"])
    with pytest.raises(RuntimeError):
        sim.thin(0, 100, 200)          # keep above the threshold
    sim.close()
    twin.close()
