"""Resume from a checkpoint file on the GPU: a run stopped, saved, loaded
into a new context and continued equals the uninterrupted run bit for bit
(particles in canonical order, ids, next ids, step, field), with
collisions, walls and secondaries, and for a batch with a retired
discharge."""
import numpy as np
import pytest

import workloads as W
from gpu_helpers import small_argon

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import paper_2609_17151_amd as P
    return P


def _same(a, b, B, S):
    for bi in range(B):
        ca, cb = a.counts(bi), b.counts(bi)
        assert ca["step"] == cb["step"] and ca["count"] == cb["count"] and ca["next_id"] == cb["next_id"], bi
        for s in range(S):
            pa, pb = a.get_particles(s, bi), b.get_particles(s, bi)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                assert np.array_equal(pa[k], pb[k]), (bi, s, k)
        assert np.array_equal(a.efield(bi), b.efield(bi)), bi


def test_resume_equals_uninterrupted_run(pic, tmp_path):
    from paper_2609_17151_amd import checkpoint as K
    cfg, tabs = small_argon(n_init=20000)
    a = pic.Sim(cfg, tabs)
    a.step(70)                          # holes from absorption are still present
    path = str(tmp_path / "argon.npz")
    K.save(a, path)
    a.step(45)
    b = K.load(path)
    assert b.counts()["step"] == 70
    b.step(45)
    _same(a, b, 1, 2)
    b.close()


def test_resume_batch_with_retired_discharge(pic, tmp_path):
    from paper_2609_17151_amd import checkpoint as K
    cfgs = [W.argon_rf(n_init=n, n_cells=nc, gap=g, v_amp=v, seed=200 + i, capacity=4 * n, weight=3e13 / n)
            for i, (n, nc, g, v) in enumerate(((8000, 200, 0.015, 150.0), (15000, 317, 0.021, 320.0)))]
    tabs = W.argon_tables()
    a = pic.Sim(cfgs, tabs)
    a.step(33)
    a.retire(0)
    path = str(tmp_path / "batch.npz")
    frozen = [a.get_particles(s, 0) for s in range(2)]
    K.save(a, path)
    a.step(40)
    b = K.load(path)
    assert b.retired == {0}
    b.step(40)
    for bi in (1,):
        for s in range(2):
            pa, pb = a.get_particles(s, bi), b.get_particles(s, bi)
            for k in ("cell", "off", "vx", "vy", "vz", "id"):
                assert np.array_equal(pa[k], pb[k]), (bi, s, k)
        assert np.array_equal(a.efield(bi), b.efield(bi))
    for s in range(2):
        pb = b.get_particles(s, 0)
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            assert np.array_equal(frozen[s][k], pb[k]), (s, k)
    b.close()
