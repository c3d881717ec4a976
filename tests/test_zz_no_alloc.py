"""The allocation-free sort (pic_sort_noalloc) against the allocating one
(pic_sort), through the C ABI: two contexts in bit-identical states, one
sorted each way; cells, offsets, velocities, ids and order must be
identical (integer work: bit-exact).  Calls in a row -- the full E x B box
(the most scratch any configuration here needs), then a smaller argon
discharge, then a small Langmuir plasma -- share the fixed scratch, which
keeps the previous call's contents.  A context whose sort needs more than
the fixed scratch is refused with PIC_ESCRATCH and nothing queued."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import small_argon

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def _sorted_both_ways(pic, cfg, tabs=(), steps=3):
    a = pic.Sim(cfg, tabs)
    b = pic.Sim(cfg, tabs)
    a.step(steps)
    b.step(steps)
    a.sort()
    b.sort_noalloc()
    for s in range(len(cfg["species"])):
        pa, pb = a.get_particles(s), b.get_particles(s)
        assert len(pa["id"]) > 0
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(pa[k], pb[k]), (s, k)
        assert pa["next_id"] == pb["next_id"]
        assert np.all(np.diff(pb["cell"]) >= 0)           # sorted by cell
    # the sorted contexts keep stepping alike
    a.step(2)
    b.step(2)
    for s in range(len(cfg["species"])):
        pa, pb = a.get_particles(s), b.get_particles(s)
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(pa[k], pb[k]), (s, k)
    a.close()
    b.close()


def test_noalloc_sort_equals_sort_in_calls_of_decreasing_size(pic):
    print("no-alloc sort: E x B box, 4e6 + 4e6 particles, 1024 cells", flush=True)
    _sorted_both_ways(pic, W.exb())
    print("no-alloc sort: argon discharge, 30000 per species, 400 cells", flush=True)
    cfg, tabs = small_argon(n_init=30000, seed=21)
    _sorted_both_ways(pic, cfg, tabs)
    print("no-alloc sort: Langmuir plasma, 5000 particles, 64 cells", flush=True)
    _sorted_both_ways(pic, W.langmuir(n_particles=5000, n_cells=64, capacity=5000))


def test_noalloc_sort_refuses_more_than_its_scratch(pic):
    # 1.2e7 slots on 1024 cells need 11719 tiles x 1024 cells x 4 B = 48 MB
    cfg = W.langmuir(n_particles=4096, n_cells=1024, capacity=12_000_000)
    sim = pic.Sim(cfg)
    before = sim.get_particles(0)
    with pytest.raises(pic.PicError) as err:
        sim.sort_noalloc()
    assert err.value.code == pic.ESCRATCH
    after = sim.get_particles(0)
    for k in ("cell", "off", "id"):
        assert np.array_equal(before[k], after[k])
    sim.close()
