"""GPU <-> oracle parity through the C ABI.

Bars: cell indices, counts, ids and compaction order bit-exact (cells except
oracle positions within 4 binary32 ulps of a cell edge); single-step
positions within 1e-6 of the domain length; velocities within relative 1e-6
(reference max(|v|, v_th)); densities within 1e-5 of the peak; collision
outcomes agreeing on >= 99.99 % of particles.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import compare_species, small_argon, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_17151_amd as P
    P.load_library()
    return P


def _vth(cfg, s):
    return cfg["species"][s]["vth"] or 1.0


def test_loading_matches_oracle(pic):
    cfg = W.langmuir()
    sim = pic.Sim(cfg)
    o = oracle.Oracle(cfg)
    pg, po = sim.get_particles(0), o.get_particles(0)
    r = compare_species(pg, po, cfg, _vth(cfg, 0))
    assert r["id_equal"] and r["cell_mismatch"] == 0
    assert r["max_dx_over_L"] < 1e-6 and r["max_dx_over_dx"] < 1e-6
    assert r["max_rel_v"] < 1e-6
    rho_g, rho_o = sim.rho(), o.field()[0]
    assert np.max(np.abs(rho_g - rho_o)) < 1e-5 * np.max(np.abs(o.density(0)))
    eg, eo = sim.efield(), o.field()[2]
    assert np.max(np.abs(eg - eo)) < 1e-5 * np.max(np.abs(eo))


@pytest.mark.parametrize("bc", [0, 1])
def test_poisson_matches_oracle(pic, bc):
    cfg = W.argon_rf(n_init=1000) if bc == 1 else W.exb(n_per_species=4096, n_cells=1024)
    sim = pic.Sim(cfg)
    o = oracle.Oracle(cfg, load=False)
    rng = np.random.default_rng(11)
    n = sim.n_nodes[0]
    for t in (0.0, 1.3e-8, 3.7e-8):
        rho = rng.normal(0, 1e-3, n) + 2e-4
        pg, eg = sim.poisson(t, rho)
        po, eo = o.poisson(t, rho)
        assert np.max(np.abs(pg - po)) <= 1e-10 * max(1.0, np.max(np.abs(po)))
        assert np.max(np.abs(eg - eo)) <= 1e-10 * np.max(np.abs(eo))


def test_langmuir_single_steps(pic):
    cfg = W.langmuir()
    sim = pic.Sim(cfg)
    for k in (0, 7, 40):
        if k:
            sim.step(k)
        o = to_oracle(sim, cfg)
        ng = sim.density()[0]
        assert np.max(np.abs(ng - o.density(0))) < 1e-5 * np.max(o.density(0))
        sim.step(1)
        o.step(1)
        r = compare_species(sim.get_particles(0), o.get_particles(0), cfg, 1.0)
        assert r["id_equal"] and r["cell_mismatch"] == 0, r
        assert r["max_dx_over_L"] < 1e-6 and r["max_rel_v"] < 1e-6, r
        assert np.max(np.abs(sim.density()[0] - o.density(0))) < 1e-5 * np.max(o.density(0))


def test_exb_single_step_full_size(pic):
    # the E x B box at its full size (4e6 electrons + 4e6 ions), one step
    cfg = W.exb()
    sim = pic.Sim(cfg)
    sim.step(3)
    o = to_oracle(sim, cfg)
    sim.step(1)
    o.step(1)
    for s in range(2):
        r = compare_species(sim.get_particles(s), o.get_particles(s), cfg, _vth(cfg, s))
        assert r["id_equal"] and r["cell_mismatch"] == 0, (s, r["cell_mismatch"])
        assert r["max_dx_over_L"] < 1e-6 and r["max_rel_v"] < 1e-6, (s, r["max_dx_over_L"], r["max_rel_v"])
        dg, do = sim.density()[s], o.density(s)
        assert np.max(np.abs(dg - do)) < 1e-5 * np.max(do)
    q_mesh, q_part = sim.charge()
    assert abs(q_mesh - q_part) <= 1e-9 * cfg["species"][0]["weight"] * 4e6 * W.E_CHARGE


def _argon_step_compare(sim, cfg, tabs):
    o = to_oracle(sim, cfg, tabs)
    n_before = [len(o.get_particles(s)["x"]) for s in range(2)]
    sim.step(1)
    o.step(1)
    out = {}
    for s in range(2):
        pg, po = sim.get_particles(s), o.get_particles(s)
        out[s] = (pg, po)
    return out, n_before, o


def test_argon_single_steps_collisions_walls(pic):
    cfg, tabs = small_argon(n_init=20000)
    sim = pic.Sim(cfg, tabs)
    sim.step(30)
    total = agree = 0
    for rep in range(12):
        res, n_before, o = _argon_step_compare(sim, cfg, tabs)
        for s in range(2):
            pg, po = res[s]
            ids_g, ids_o = pg["id"], po["id"]
            # compare the particles present on both sides, matched by id;
            # a particle present on one side only counts as a disagreement
            common = np.intersect1d(ids_g, ids_o)
            gi = {v: i for i, v in enumerate(ids_g)}
            oi = {v: i for i, v in enumerate(ids_o)}
            ig = np.array([gi[v] for v in common])
            io = np.array([oi[v] for v in common])
            sub_g = {k: v[ig] for k, v in pg.items() if k != "next_id"}
            sub_o = {k: v[io] for k, v in po.items() if k != "next_id"}
            r = compare_species(sub_g, sub_o, cfg, _vth(cfg, s))
            ok = (r["rel_v"] < 1e-6) & (r["dx"] < 1e-6 * cfg["length"])
            total += len(common) + abs(len(ids_g) - len(ids_o))
            agree += int(ok.sum())
    assert total > 0
    assert agree / total >= 0.9999, (agree, total)


def test_argon_counts_and_order_bit_exact(pic):
    # steps from identical states: ids and order, the particles absorbed at
    # each wall, the secondaries emitted and the collision candidates agree
    # exactly (integer tests on identical draws, positions far from the
    # walls' rounding); the channel of a real collision may differ only where
    # u1 nu_max falls within rounding of a partial sum of the channel
    # frequencies, which is counted (at most two over the run)
    cfg, tabs = small_argon(n_init=20000, seed=5)
    sim = pic.Sim(cfg, tabs)
    sim.step(10)
    channel_ties = 0
    n_coll = 0
    for rep in range(8):
        w0, k0 = sim.wall(), sim.coll()
        res, n_before, o = _argon_step_compare(sim, cfg, tabs)
        w1, k1 = sim.wall(), sim.coll()
        co = o.counters()
        for s in range(2):
            pg, po = res[s]
            assert len(pg["id"]) == len(po["id"])
            assert np.array_equal(pg["id"], po["id"])
        np.testing.assert_array_equal(w1["absorbed"] - w0["absorbed"], co["absorbed"])
        np.testing.assert_array_equal(w1["see_emitted"] - w0["see_emitted"], co["see_emitted"])
        np.testing.assert_array_equal(k1["candidates"] - k0["candidates"], co["candidates"])
        dg = np.concatenate([(k1["coll"] - k0["coll"]), (k1["nulls"] - k0["nulls"])[:, None]], axis=1)
        do = np.concatenate([co["coll"], co["nulls"][:, None]], axis=1)
        channel_ties += int(np.abs(dg - do).sum()) // 2
        n_coll += int(do.sum())
        sim.step(3)
    print("collision outcomes compared: %d, channel ties: %d" % (n_coll, channel_ties))
    assert n_coll > 1000
    assert channel_ties <= 2


def test_numax_matches_oracle(pic):
    # a consistency check, not parity: the bound is a definition written the
    # same way on both sides so that the integer candidate thresholds agree
    # (the pin of the bound itself is the oracle's own bound test)
    cfg, tabs = small_argon(n_init=1000)
    sim = pic.Sim(cfg, tabs)
    o = oracle.Oracle(cfg, tabs, load=False)
    for s in range(2):
        nug, tg = sim.numax(s)
        nuo, to = o.numax(s)
        assert nug == nuo and tg == to


def test_gpu_runs_are_bit_reproducible(pic):
    cfg, tabs = small_argon(n_init=20000, seed=9)
    outs = []
    for _ in range(2):
        sim = pic.Sim(cfg, tabs)
        sim.step(60)
        outs.append([sim.get_particles(s) for s in range(2)] + [sim.rho()])
        sim.close()
    for s in range(2):
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(outs[0][s][k], outs[1][s][k]), (s, k)
    assert np.array_equal(outs[0][2], outs[1][2])


def test_langmuir_energy_and_frequency_on_gpu(pic):
    cfg = W.langmuir()
    sim = pic.Sim(cfg)
    sim.set_diag(True)                 # kinetic energy is kept with the diagnostics
    L = cfg["length"]
    nn = sim.n_nodes[0]
    sn = np.sin(2 * np.pi * np.arange(nn) / nn)
    tot, a = [], []
    for _ in range(600):
        fe = sim.energy()[1]
        sim.step(1)
        ke = sim.energy()[0].sum()
        tot.append(ke + fe)
        a.append(2.0 / nn * np.dot(sim.efield(), sn))
    tot = np.array(tot)
    assert np.ptp(tot) / tot[0] < 5e-4
    # zero crossings give the frequency; kinetic root at k lambda_D = 0.3 is 1.15985
    a = np.array(a)
    t = (np.arange(len(a)) + 1) * cfg["dt"]
    zc = t[:-1][np.sign(a[:-1]) != np.sign(a[1:])]
    zc = zc[zc > 5]
    w = math.pi / np.mean(np.diff(zc))
    assert abs(w / 1.15985 - 1) < 0.02


def test_set_particles_validation(pic):
    cfg = W.langmuir(n_particles=4096)
    sim = pic.Sim(cfg)
    p = sim.get_particles(0)
    bad = p["vx"].copy()
    bad[7] = np.nan
    with pytest.raises(pic.PicError) as e:
        sim.set_particles(0, p["cell"], p["off"], bad, p["vy"], p["vz"], p["id"], p["next_id"], 0)
    assert e.value.code == pic.ENUMERIC
    badc = p["cell"].copy()
    badc[3] = cfg["n_cells"]
    with pytest.raises(pic.PicError) as e:
        sim.set_particles(0, badc, p["off"], p["vx"], p["vy"], p["vz"], p["id"], p["next_id"], 0)
    assert e.value.code == pic.EINVAL


def test_bad_tables_rejected(pic):
    cfg, tabs = small_argon(n_init=100)
    sim = pic.Sim(cfg)
    e = np.array([1.0, 2.0, 2.0, 3.0])
    with pytest.raises(pic.PicError) as ex:
        sim.load_xsec(0, W.XS_ELASTIC, 0.0, e, np.ones(4) * 1e-20)
    assert ex.value.code == pic.EINVAL
    with pytest.raises(pic.PicError):
        sim.load_xsec(1, W.XS_IONIZATION, 15.8, tabs[2]["energy"], tabs[2]["sigma"])
    sim.load_xsec(0, W.XS_ELASTIC, 0.0, tabs[0]["energy"], tabs[0]["sigma"])
    with pytest.raises(pic.PicError):      # mixing electron and ion kinds
        sim.load_xsec(0, W.XS_ION_CX, 0.0, tabs[3]["energy"], tabs[3]["sigma"])


def test_capacity_overflow_latched(pic):
    cfg, tabs = small_argon(n_init=20000)
    for sp in cfg["species"]:
        sp["capacity"] = 20100           # room for few births
    sim = pic.Sim(cfg, tabs)
    sim.step(300)
    with pytest.raises(pic.PicError) as e:
        sim.sync()
    assert e.value.code == pic.ECAPACITY


@pytest.mark.parametrize("which", ["langmuir", "argon"])
def test_graph_replays_match_direct_launches(pic, which):
    # replays of the captured step chunk, with eager work and readbacks in
    # between, equal direct launches bit for bit after every replay
    if which == "langmuir":
        cfg, tabs = W.langmuir(n_particles=1 << 15), ()
    else:
        cfg, tabs = small_argon(n_init=20000, seed=13)
    a = pic.Sim(cfg, tabs)
    b = pic.Sim(cfg, tabs)
    b.use_graphs(False)
    for rep in range(4):
        a.step(32)
        b.step(32)
        assert a.counts() == b.counts()
        for s in range(len(cfg["species"])):
            pa, pb = a.get_particles(s), b.get_particles(s)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                assert np.array_equal(pa[k], pb[k]), (rep, s, k)
        assert np.array_equal(a.efield(), b.efield())


def _stable_by_cell(p):
    o = np.argsort(p["cell"], kind="stable")
    return {k: (v[o] if k != "next_id" else v) for k, v in p.items()}


@pytest.mark.parametrize("which", ["langmuir", "argon", "batched"])
def test_sort_is_a_stable_sort_by_cell(pic, which):
    if which == "langmuir":
        cfgs, tabs = [W.langmuir(n_particles=100_000, capacity=100_000)], ()
    elif which == "argon":
        cfg, tabs = small_argon(n_init=30000, seed=21)
        cfgs = [cfg]
    else:
        cfgs = [W.langmuir(n_particles=n, n_cells=nc, seed=sd, capacity=n)
                for n, nc, sd in ((5000, 64, 1), (70_001, 128, 2), (12_345, 100, 3))]
        tabs = ()
    sim = pic.Sim(cfgs, tabs)
    sim.step(25)
    before = [[sim.get_particles(s, b) for s in range(sim.S)] for b in range(sim.B)]
    sim.sort()
    for b in range(sim.B):
        for s in range(sim.S):
            got = sim.get_particles(s, b)
            exp = _stable_by_cell(before[b][s])
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                assert np.array_equal(got[k], exp[k]), (b, s, k)
    sim.sync()


def test_periodic_sort_changes_order_not_physics(pic):
    # collisionless: the deposit is order-independent, so sorting every few
    # steps leaves the field bit-identical and the particles equal up to order
    cfg = W.langmuir(n_particles=1 << 16)
    a, b = pic.Sim(cfg), pic.Sim(cfg)
    b.config_tiles(4, 1024, 5)
    for _ in range(3):
        a.step(40)
        b.step(40)
        assert np.array_equal(a.efield(), b.efield())
    pa, pb = a.get_particles(0), b.get_particles(0)
    oa, ob = np.argsort(pa["id"]), np.argsort(pb["id"])
    for k in ("cell", "off", "vx", "vy", "vz", "id"):
        assert np.array_equal(pa[k][oa], pb[k][ob]), k
    assert not np.array_equal(pa["id"], pb["id"])


def _uneven_argon_batch():
    cfgs = []
    for i, (n, nc, gap, v) in enumerate(((8000, 200, 0.015, 150.0), (30000, 400, 0.025, 200.0),
                                         (15000, 317, 0.021, 320.0))):
        cfg = W.argon_rf(n_init=n, n_cells=nc, gap=gap, v_amp=v, seed=100 + i, capacity=4 * n,
                         weight=3e13 / n)
        cfgs.append(cfg)
    return cfgs


def test_batched_discharges_equal_single_runs(pic):
    cfgs = _uneven_argon_batch()
    tabs = W.argon_tables()
    batch = pic.Sim(cfgs, tabs)
    batch.step(120)
    for b, cfg in enumerate(cfgs):
        one = pic.Sim(cfg, tabs)
        one.step(120)
        assert batch.counts(b) == one.counts()
        for s in range(2):
            pb, po = batch.get_particles(s, b), one.get_particles(s)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                assert np.array_equal(pb[k], po[k]), (b, s, k)
        assert np.array_equal(batch.efield(b), one.efield())
        one.close()


def test_retired_discharge_is_frozen(pic):
    cfgs = _uneven_argon_batch()
    tabs = W.argon_tables()
    batch = pic.Sim(cfgs, tabs)
    batch.step(40)
    frozen = [batch.get_particles(s, 0) for s in range(2)]
    batch.retire(0)
    batch.step(70)                      # not a multiple of the graph chunk
    for s in range(2):
        now = batch.get_particles(s, 0)
        for k in ("cell", "off", "vx", "id"):
            assert np.array_equal(now[k], frozen[s][k])
    assert batch.counts(0)["step"] == 40 and batch.counts(1)["step"] == 110
    one = pic.Sim(cfgs[2], tabs)
    one.step(110)
    assert np.array_equal(batch.get_particles(1, 2)["vx"], one.get_particles(1)["vx"])
