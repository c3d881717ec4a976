"""The step-schedule autotuner: candidate sets, the choice of the fastest,
the cache (host logic, on a stand-in context), and on the GPU that a tuned
run reaches exactly the state of an untuned one."""
import json

import numpy as np
import pytest

import workloads as W
from paper_2609_17151_amd import autotune


class FakeSim:
    def __init__(self, cfg):
        self.cfgs, self.B, self.S = [cfg], 1, len(cfg["species"])
        self.applied, self.stepped, self.fused = [], 0, []

    def counts(self, b):
        return dict(count=[1000] * self.S, step=0, flags=0, next_id=[1000 + 10 * self.stepped] * self.S)

    def config_tiles(self, ppt, threads, sort_every, compact_every):
        self.applied.append((ppt, threads, sort_every, compact_every))

    def config_events(self, in_push):
        self.fused.append(bool(in_push))

    def step(self, n):
        self.stepped += n


def fake_timer(sim, n):
    ppt, thr, srt, cmp_ = sim.applied[-1]
    sim.stepped += n
    return 1.0 + 0.1 * ppt + (0.0 if thr == 512 else 0.05) + 0.01 * srt + 0.001 * cmp_


def test_candidates_by_kernel_mode():
    g = autotune.candidates(True)
    s = autotune.candidates(False)
    assert {(c["ppt"], c["threads"]) for c in g} == set(autotune.GENERAL)
    assert {c["compact_every"] for c in g} == set(autotune.COMPACT_EVERY)
    # a captured graph replays 32 steps: every compaction interval divides it
    assert all(32 % c["compact_every"] == 0 for c in g)
    assert {(c["ppt"], c["threads"]) for c in s} == set(autotune.STREAMING)
    # births take ids in their parents' order, so a sort would change the
    # random numbers of a run with births: no sort in the general kernel
    assert {c["sort_every"] for c in g} == {0}
    assert {c["sort_every"] for c in s} == set(autotune.SORT_EVERY)
    # events in the push workgroups: general 256-thread tiles only
    assert {(c["ppt"], c["threads"], c["fuse"]) for c in g if c["fuse"]} == {(1, 256, 1), (2, 256, 1), (4, 256, 1)}
    assert {(c["threads"], c["fuse"]) for c in g} == {(256, 0), (256, 1), (512, 0), (1024, 0)}
    assert {c["fuse"] for c in s} == {0}


def test_picks_fastest_and_caches(tmp_path):
    cfg = W.langmuir(n_particles=4096)
    sim = FakeSim(cfg)
    cache = str(tmp_path / "tune.json")
    choice, table = autotune.tune(sim, steps=8, warm=0, cache=cache, timer=fake_timer)
    assert choice == dict(ppt=1, threads=256, sort_every=0, compact_every=16, fuse=0)
    best = min(table, key=lambda r: r["ms_per_step"])
    assert all(choice[k] == best[k] for k in choice)
    assert sim.applied[-1] == (choice["ppt"], choice["threads"], choice["sort_every"], choice["compact_every"])
    assert sim.fused[-1] is False
    stored = json.load(open(cache))
    assert autotune.signature(sim) in stored
    # a known workload is applied from the cache without timing
    sim2 = FakeSim(cfg)
    c2, _ = autotune.tune(sim2, steps=8, warm=0, cache=cache, timer=fake_timer)
    assert c2 == choice and sim2.stepped == 0 and len(sim2.applied) == 1


@pytest.mark.gpu
def test_tuned_run_reaches_the_untuned_state():
    import paper_2609_17151_amd as P
    from gpu_helpers import small_argon
    cfg, tabs = small_argon(n_init=20000)
    a = P.Sim(cfg, tabs)
    choice, table = autotune.tune(a, steps=16, warm=8)
    # the chosen schedule replays captured step graphs
    g0 = a.graphs()["steps"]
    a.step(64)
    assert a.graphs()["steps"] - g0 >= 32, (choice, a.graphs())
    n = a.counts()["step"]
    b = P.Sim(cfg, tabs)
    b.step(n)
    assert a.counts()["count"] == b.counts()["count"]
    for s in range(2):
        pa, pb = a.get_particles(s), b.get_particles(s)
        ia, ib = np.argsort(pa["id"]), np.argsort(pb["id"])
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(pa[k][ia], pb[k][ib]), k
    np.testing.assert_array_equal(a.rho(), b.rho())


def test_compaction_interval_needs_capacity_headroom():
    # 1000 slots in use and 10 births per step: with capacity 1500 (90 %:
    # 1350) a compaction every 8 or 16 steps fits (1160, 1320 slots at twice
    # the birth rate), every 32 steps does not (1640)
    cfg, _ = W.argon_rf(n_init=1000), None
    for sp in cfg["species"]:
        sp["capacity"] = 1500
    sim = FakeSim(cfg)
    rate = autotune.birth_rate(sim, steps=4)
    assert rate[(0, 0)] == 10.0
    assert autotune.fits(sim, 8, rate) and autotune.fits(sim, 16, rate)
    assert not autotune.fits(sim, 32, rate)
    choice, table = autotune.tune(sim, steps=4, warm=0, timer=fake_timer)
    assert {r["compact_every"] for r in table} == {8, 16}
    assert choice["compact_every"] in (8, 16)


def test_most_frequent_compaction_when_no_interval_fits():
    # 1000 slots in use, 10 births per step, capacity 1100 (90 %: 990): no
    # interval fits, so the candidates compact every 8 steps
    cfg = W.argon_rf(n_init=1000)
    for sp in cfg["species"]:
        sp["capacity"] = 1100
    sim = FakeSim(cfg)
    choice, table = autotune.tune(sim, steps=4, warm=0, timer=fake_timer)
    assert table and {r["compact_every"] for r in table} == {min(autotune.COMPACT_EVERY)}
    assert choice["compact_every"] == min(autotune.COMPACT_EVERY)
