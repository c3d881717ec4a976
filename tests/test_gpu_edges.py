"""Edge cases on the GPU against the oracle: empty species and an empty
context, particle counts that leave ragged tiles for every tile shape, the
largest meshes (4096 periodic cells, 4095 bounded cells) with the field
solve at full size, and the meshes and batches the library must refuse."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_helpers import compare_species, small_argon, to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def test_empty_species_and_empty_context(pic):
    # electrons only, ions loaded empty: the ions stay empty, the electrons
    # step as the oracle's
    cfg = W.exb(n_per_species=4096, n_cells=256)
    cfg["species"][1]["load"] = W.LOAD_NONE
    sim = pic.Sim(cfg)
    o = to_oracle(sim, cfg)
    sim.step(1)
    o.step(1)
    assert sim.counts()["count"] == [4096, 0]
    r = compare_species(sim.get_particles(0), o.get_particles(0), cfg, cfg["species"][0]["vth"])
    assert r["id_equal"] and r["cell_mismatch"] == 0 and r["max_rel_v"] < 1e-6
    assert np.all(sim.density()[1] == 0.0)
    # nothing at all: a driven vacuum gap steps, its potential is the
    # oracle's and linear between the electrodes
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    vac = W.base_config(n_cells=64, bc=1, field_solve=1, length=1.0, dt=0.01, eps0=1.0, v_amp=2.0, v_freq=3.0,
                        species=[sp, dict(sp)])
    s2 = pic.Sim(vac)
    ov = oracle.Oracle(vac, load=False)
    s2.step(37)
    ov.step(37)
    phi = s2.phi()
    np.testing.assert_allclose(phi, ov.field()[1], rtol=0, atol=1e-12)
    assert np.max(np.abs(np.diff(phi, 2))) < 1e-12 and phi[-1] == 0.0 and abs(phi[0]) > 0.1
    assert s2.counts()["count"] == [0, 0]


@pytest.mark.parametrize("n", [1, 255, 1025, 4097, 12289])
def test_ragged_counts_every_tile_shape(pic, n):
    # counts that leave a partial last tile (and fewer particles than one
    # tile) for every streaming tile shape; one step against the oracle
    cfg = W.langmuir(n_particles=n, n_cells=64)
    cfg["species"][0]["capacity"] = max(n, 1)
    for ppt, thr in ((1, 256), (2, 256), (4, 256), (8, 256), (4, 512), (4, 1024)):
        sim = pic.Sim(cfg)
        sim.config_tiles(ppt, thr, 0)
        sim.step(2)
        o = to_oracle(sim, cfg)
        sim.step(1)
        o.step(1)
        r = compare_species(sim.get_particles(0), o.get_particles(0), cfg, 1.0)
        assert r["id_equal"] and r["cell_mismatch"] == 0, (n, ppt, thr)
        assert r["max_dx_over_L"] < 1e-6 and r["max_rel_v"] < 1e-6, (n, ppt, thr)
        sim.close()


@pytest.mark.parametrize("n", [1, 301, 2049])
def test_ragged_counts_general_kernel(pic, n):
    # the general kernel (walls, collisions, secondaries) with tiny and
    # ragged counts, every tile shape; births, losses and their order agree
    # exactly, kinematics to binary32 rounding (at most one particle per
    # species may differ by a collision decided on the other side of a
    # rounding edge)
    for ppt, thr in ((1, 256), (2, 256), (4, 256), (8, 256), (4, 512), (8, 512), (4, 1024)):
        cfg, tabs = small_argon(n_init=n)
        cfg["species"][0]["capacity"] = cfg["species"][1]["capacity"] = 8 * n + 64
        sim = pic.Sim(cfg, tabs)
        sim.config_tiles(ppt, thr, 0)
        sim.step(5)
        o = to_oracle(sim, cfg, tabs)
        sim.step(1)
        o.step(1)
        for s in range(2):
            pg, po = sim.get_particles(s), o.get_particles(s)
            assert np.array_equal(pg["id"], po["id"]), (n, ppt, thr, s)
            r = compare_species(pg, po, cfg, cfg["species"][s]["vth"] or 1.0)
            bad = (r["rel_v"] >= 1e-6) | (r["dx"] >= 1e-6 * cfg["length"])
            assert r["cell_mismatch"] <= 1 and bad.sum() <= 1, (n, ppt, thr, s, int(bad.sum()))
        sim.close()


@pytest.mark.parametrize("bc,cells", [(0, 4096), (1, 4095)])
def test_largest_meshes(pic, bc, cells):
    # the largest mesh each boundary allows: loading, one step and the field
    # solve of a random charge against the oracle
    if bc == 0:
        cfg = W.exb(n_per_species=65536, n_cells=cells, length=0.02)
    else:
        cfg = W.argon_rf(n_init=20000, n_cells=cells, gap=cells * 6.25e-5, capacity=160000)
    sim = pic.Sim(cfg)
    o = oracle.Oracle(cfg, load=False)
    rng = np.random.default_rng(3)
    n = sim.n_nodes[0]
    assert n == (cells if bc == 0 else cells + 1)
    rho = rng.normal(0, 1e-3, n) + 2e-4
    pg, eg = sim.poisson(2.1e-9, rho)
    po, eo = o.poisson(2.1e-9, rho)
    assert np.max(np.abs(pg - po)) <= 1e-10 * max(1.0, np.max(np.abs(po)))
    assert np.max(np.abs(eg - eo)) <= 1e-10 * np.max(np.abs(eo))
    o2 = to_oracle(sim, cfg)
    sim.step(1)
    o2.step(1)
    for s in range(2):
        r = compare_species(sim.get_particles(s), o2.get_particles(s), cfg, cfg["species"][s]["vth"] or 1.0)
        assert r["id_equal"] and r["cell_mismatch"] == 0, (s, r["cell_mismatch"])
        assert r["max_dx_over_L"] < 1e-6 and r["max_rel_v"] < 1e-6, (s, r["max_dx_over_L"], r["max_rel_v"])


def test_largest_batch(pic):
    # 256 discharges, the most one context holds, each a small Langmuir
    # plasma of its own count and seed; sampled discharges against the oracle
    cfgs = [W.langmuir(n_particles=500 + 37 * b, n_cells=32 + (b % 5), seed=100 + b) for b in range(256)]
    sim = pic.Sim(cfgs)
    sim.step(3)
    picks = (0, 1, 127, 200, 255)
    oracles = {b: to_oracle(sim, cfgs[b], batch=b) for b in picks}
    sim.step(2)
    for b in picks:
        oracles[b].step(2)
        r = compare_species(sim.get_particles(0, b), oracles[b].get_particles(0), cfgs[b], 1.0)
        assert r["id_equal"] and r["cell_mismatch"] == 0, b
        assert r["max_dx_over_L"] < 1e-6 and r["max_rel_v"] < 1e-6, b


def test_meshes_and_batches_refused(pic):
    sp = W.species(-1.0, 1.0, 1.0, 0, 1.0, capacity=16, load=W.LOAD_NONE)
    for bad in (dict(bc=0, n_cells=4097), dict(bc=1, n_cells=4096), dict(bc=0, n_cells=1)):
        with pytest.raises(RuntimeError):
            pic.Sim(W.base_config(species=[sp], **bad))
    with pytest.raises(RuntimeError):
        pic.Sim([W.base_config(species=[sp])] * 257)
    mixed = [W.base_config(species=[sp]), W.base_config(species=[sp, dict(sp)])]
    with pytest.raises(RuntimeError):
        pic.Sim(mixed)                  # every discharge of a context has the same species count


def test_dense_gas_many_collisions(pic):
    # at 3 Torr three quarters of the electrons are collision candidates in
    # every step and about a fifth collide: one step from identical states
    # against the oracle.  Births, losses and order agree exactly; the
    # collision kinematics run in FP64 and round once, so every particle,
    # collided or not, agrees to 1e-6
    cfg, tabs = small_argon(n_init=20000)
    dense = W.argon_rf(n_init=20000, pressure_mtorr=3000.0, weight=cfg["species"][0]["weight"],
                       capacity=cfg["species"][0]["capacity"])
    sim = pic.Sim(dense, tabs)
    sim.step(4)
    o = to_oracle(sim, dense, tabs)
    n0 = sim.counts()["count"][0]
    c0 = sim.coll()["candidates"][0]
    sim.step(1)
    o.step(1)
    assert (sim.coll()["candidates"][0] - c0) > 0.5 * n0
    for s in range(2):
        pg, po = sim.get_particles(s), o.get_particles(s)
        assert np.array_equal(pg["id"], po["id"]), s
        r = compare_species(pg, po, dense, dense["species"][s]["vth"] or 1.0)
        assert r["cell_mismatch"] == 0 and r["max_dx_over_L"] < 1e-6, s
        print("dense gas, species %d: max relative velocity error %.3g" % (s, r["max_rel_v"]))
        assert r["max_rel_v"] < 1e-6, (s, r["max_rel_v"])
