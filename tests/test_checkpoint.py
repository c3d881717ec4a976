"""Checkpoint files on the host: the file round trip with a stand-in
context (no GPU), the format check, and the rule that live discharges
share one step.  The resume itself is tested on the GPU
(test_gpu_checkpoint.py)."""
import numpy as np
import pytest

import workloads as W
from paper_2609_17151_amd import checkpoint as K


class FakeSim:
    """What the checkpoint uses of a context, held in host arrays."""

    def __init__(self, cfgs, tables=(), step=7, seed=0):
        self.cfgs = cfgs
        self.B, self.S = len(cfgs), len(cfgs[0]["species"])
        self.tables = [dict(t) for t in tables]
        self.retired = set()
        self.step_index = [step] * self.B
        rng = np.random.default_rng(seed)
        self.parts = {}
        for b in range(self.B):
            for s in range(self.S):
                n = int(rng.integers(0, 50))
                self.parts[(b, s)] = dict(cell=rng.integers(0, cfgs[b]["n_cells"], n).astype(np.int32),
                                          off=rng.random(n).astype(np.float32),
                                          vx=rng.normal(size=n).astype(np.float32),
                                          vy=rng.normal(size=n).astype(np.float32),
                                          vz=rng.normal(size=n).astype(np.float32),
                                          id=rng.permutation(1000)[:n].astype(np.uint32), next_id=1000 + s)
        self.calls = []

    def counts(self, b):
        return dict(step=self.step_index[b])

    def get_particles(self, s, b=0):
        return dict(self.parts[(b, s)])

    def set_particles(self, s, cell, off, vx, vy, vz, ids, next_id, step, batch=0):
        self.calls.append((batch, s, int(step)))
        self.parts[(batch, s)] = dict(cell=cell, off=off, vx=vx, vy=vy, vz=vz, id=ids, next_id=next_id)
        self.step_index = [int(step)] * self.B

    def retire(self, b, retired=True):
        self.retired.add(b)


def _cfgs():
    return [W.argon_rf(n_init=100, n_cells=50 + 10 * i, seed=i) for i in range(3)]


def test_round_trip(tmp_path):
    tabs = W.argon_tables(n=20)
    a = FakeSim(_cfgs(), tabs, step=123)
    a.retired.add(2)
    a.step_index[2] = 40                 # a retired discharge stopped earlier
    path = str(tmp_path / "c.npz")
    K.save(a, path)
    made = {}

    def make(cfgs, tables):
        made["cfgs"], made["tables"] = cfgs, tables
        return FakeSim(cfgs, tables, step=0, seed=99)

    b = K.load(path, make_sim=make)
    assert all(sp["load"] == 2 for c in made["cfgs"] for sp in c["species"])
    assert len(made["tables"]) == len(tabs)
    for t0, t1 in zip(tabs, made["tables"]):
        assert t0["species"] == t1["species"] and t0["kind"] == t1["kind"]
        assert np.array_equal(t0["energy"], t1["energy"]) and np.array_equal(t0["sigma"], t1["sigma"])
    assert b.cfgs == a.cfgs                           # the saved record, load modes included
    assert b.retired == {2}
    assert {c[2] for c in b.calls} == {123}
    for key, p in a.parts.items():
        q = b.parts[key]
        for k in K.FIELDS:
            assert q[k].dtype == p[k].dtype and np.array_equal(q[k], p[k]), (key, k)
        assert q["next_id"] == p["next_id"]


def test_foreign_file_rejected(tmp_path):
    path = str(tmp_path / "x.npz")
    np.savez(path, format=np.array("something else"))
    with pytest.raises(ValueError):
        K.read(path)


def test_live_discharges_must_share_a_step(tmp_path):
    a = FakeSim(_cfgs())
    a.step_index[1] = 8
    with pytest.raises(ValueError):
        K.save(a, str(tmp_path / "c.npz"))


def test_file_loads_without_pickle(tmp_path):
    a = FakeSim(_cfgs(), W.argon_tables(n=10))
    path = str(tmp_path / "c.npz")
    K.save(a, path)
    with np.load(path, allow_pickle=False) as z:
        assert all(z[k].dtype != object for k in z.files)
