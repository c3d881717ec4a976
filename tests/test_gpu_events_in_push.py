"""Events in the push workgroups (pic_config_events) against the events
kernel: the step's collisions, renewals and secondary emissions are the
same arithmetic on the same records either way, so runs reach the same
state bit for bit -- particles, counts, ids, event counters, the field and
every time-averaged diagnostic.

Cases: a batch of three argon discharges of uneven size with collisions,
walls, secondary emission and ionization births, diagnostics on, under
each 256-thread tile shape (one, two and four particles per thread); and
an E x B box with axial renewal."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_17151_amd as P
    P.load_library()
    return P


def _argon_batch():
    return [W.argon_rf(n_init=n, n_cells=nc, gap=g, v_amp=v, seed=500 + i, capacity=4 * n, weight=3e13 / n)
            for i, (n, nc, g, v) in enumerate(((6000, 160, 0.015, 150.0), (21000, 317, 0.021, 320.0),
                                               (1300, 64, 0.012, 220.0)))]


def _state(sim):
    out = {}
    for b in range(sim.B):
        out[("counts", b)] = sim.counts(b)
        for s in range(sim.S):
            p = sim.get_particles(s, b)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                out[(k, b, s)] = p[k]
        out[("rho", b)] = sim.rho(b)
        out[("wall", b)] = sim.wall(b)
        out[("coll", b)] = sim.coll(b)
        out[("avg", b)] = sim.avg(b)
        out[("power", b)] = sim.power(b)
        out[("eepf", b)] = sim.eepf(b)
        out[("wall_edf", b)] = sim.wall_edf(b)
    return out


def _equal(a, b, where=()):
    if isinstance(a, dict):
        assert a.keys() == b.keys(), where
        for k in a:
            _equal(a[k], b[k], where + (k,))
    elif isinstance(a, (list, tuple)):
        assert len(a) == len(b), where
        for i, (x, y) in enumerate(zip(a, b)):
            _equal(x, y, where + (i,))
    else:
        assert np.array_equal(np.asarray(a), np.asarray(b)), where


@pytest.mark.parametrize("ppt", [1, 2, 4])
def test_argon_batch_events_in_push_equal_events_kernel(pic, ppt):
    cfgs, tabs = _argon_batch(), W.argon_tables()
    runs = []
    for fuse in (False, True):
        sim = pic.Sim(cfgs, tabs)
        sim.config_tiles(ppt, 256, 0, 16)
        sim.config_events(fuse)
        sim.set_diag(True)
        sim.step(300)
        runs.append(_state(sim))
        sim.close()
    born = sum(int(runs[0][("counts", b)]["next_id"][1]) for b in range(len(cfgs)))
    assert born > sum(c["species"][1]["n_init"] for c in cfgs)      # ionization happened
    assert sum(int(runs[0][("wall", b)]["see_emitted"].sum()) for b in range(len(cfgs))) > 0
    _equal(runs[0], runs[1])


def test_renewal_events_in_push_equal_events_kernel(pic):
    # a short axial transit (0.2 mm) so that electrons renew within the run
    cfg = W.ecdi(n_per_species=60000, n_cells=256, lz=2e-4)
    runs = []
    for fuse in (False, True):
        sim = pic.Sim(cfg)
        sim.config_tiles(2, 256, 0, 16)
        sim.config_events(fuse)
        sim.step(300)
        st = dict(renewed=sim.renewed(), counts=sim.counts(), rho=sim.rho())
        for s in range(2):
            p = sim.get_particles(s)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                st[(k, s)] = p[k]
            st[("z", s)] = sim.axial(s)
        runs.append(st)
        sim.close()
    assert runs[0]["renewed"].sum() > 0
    _equal(runs[0], runs[1])


def test_config_events_rejects_other_values(pic):
    sim = pic.Sim(W.langmuir(n_particles=4096))
    with pytest.raises(RuntimeError):
        sim._check(pic._lib.pic_config_events(sim.h, 2), "pic_config_events")
    sim.close()


@pytest.mark.parametrize("ppt,threads", [(8, 256), (8, 512), (4, 1024)])
def test_tile_shapes_reach_the_same_state(pic, ppt, threads):
    # the general kernel's other tile shapes (events kernel) against four
    # particles per thread on 256 threads: the same steps, the same state
    cfgs, tabs = _argon_batch(), W.argon_tables()
    runs = []
    for shape in ((4, 256), (ppt, threads)):
        sim = pic.Sim(cfgs, tabs)
        sim.config_tiles(shape[0], shape[1], 0, 16)
        sim.set_diag(True)
        sim.step(200)
        runs.append(_state(sim))     # every quantity here is an integer sum or follows from one
        sim.close()
    _equal(runs[0], runs[1])


def test_births_of_more_tiles_than_finalize_threads(pic):
    # one discharge whose species span more than 1024 tiles of 256 particles:
    # the finalize's births workgroup covers several tiles per thread; the
    # state must equal that of a run with 1024-particle tiles (fewer tiles)
    n = 300_000
    cfg = W.argon_rf(n_init=n, capacity=2 * n, weight=3e13 / n, seed=7, te_ev=6.0, pressure_mtorr=120.0)
    tabs = W.argon_tables()
    runs = []
    for shape in ((1, 256), (4, 1024)):
        sim = pic.Sim(cfg, tabs)
        sim.config_tiles(shape[0], shape[1], 0, 16)
        sim.step(40)
        runs.append(_state(sim))
        sim.close()
    assert runs[0][("counts", 0)]["next_id"][1] > n        # ions were born
    _equal(runs[0], runs[1])
