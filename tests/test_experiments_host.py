"""Host logic of the experiment drivers: which cold runs give a valid
reference, and the bench line's summary of the measured wall times."""
import json
import os

import numpy as np

import bench
from paper_2609_17151_amd import experiments as E
from paper_2609_17151_amd import steady


def _cold(dists, counts, flags=None):
    nw = max(len(d) for d in dists)
    pad = lambda r: np.pad(np.asarray(r, dtype=np.float64), (0, nw - len(r)), constant_values=np.nan)
    out = dict(ids=np.arange(len(dists)), dist=np.array([pad(d) for d in dists]),
               times=np.array([pad(np.arange(1, len(d) + 1) * 10.0) for d in dists]),
               steps=np.array([pad(np.arange(1, len(d) + 1) * 100) for d in dists]),
               counts=np.array(counts))
    if flags is not None:
        out["flags"] = np.array(flags)

    class F(dict):
        files = list(out)
    return F(out)


def test_cold_summary_excludes_dead_flagged_and_short_runs():
    steady_run = [0.5, 0.3] + [0.01] * 20               # converges at the third window
    c = _cold([steady_run, steady_run, steady_run[:10] + [0.01] * 2, steady_run],
              [[100, 100], [0, 50], [100, 100], [100, 100]], flags=[0, 0, 0, 1])
    s = E.cold_summary(c)
    assert s[0]["alive"] and s[0]["periods"] == 3 * 5
    assert not s[1]["alive"]                             # an empty species: died out
    assert not s[2]["alive"]                             # stopped before the others
    assert not s[3]["alive"]                             # a device flag latched
    assert s[0]["tol"] == steady.noise_tolerance(np.array(steady_run))


def test_bench_line_carries_the_wall_time_summary():
    out = bench.c5_summary()
    assert out is not None and out["measured_in_this_run"] is False
    path = os.path.join(bench.ROOT, out["source"])
    assert os.path.exists(path)
    with open(os.path.join(bench.ROOT, "profiles", "c5_wall_time_summary.json")) as f:
        s = json.load(f)
    # the batched warm start beats the plain method per converged discharge
    assert out["batched_warm_s_per_converged_discharge"] < out["plain_s_per_converged_discharge"]
    assert s["draws"] == out["draws"]


def test_kernel_hash_follows_code_not_comments():
    src = 'int f(int a) {  // the first "word"\n  /* two\n lines */ return a + 1;\n}\n\nconst char* s = "// kept";\n'
    edited = src.replace("the first", "the last").replace("two\n lines", "one line") + "\n// more\n"
    assert bench.code_only(src) == bench.code_only(edited)
    assert "// kept" in bench.code_only(src)
    assert bench.code_only(src) != bench.code_only(src.replace("a + 1", "a + 2"))
    # every committed push summary was taken of the kernel built from this tree
    assert bench.measured_traffic() is not None
    assert bench.rocprof_push_us() is not None


def test_scaled_sweep_keeps_each_discharges_density():
    import workloads as W
    c0, w0 = bench.sweep_counts(W)
    assert np.all(w0 == W.PILOT_WEIGHT)
    c, w = bench.sweep_counts(W, 1.77e7)
    assert abs(2 * c.sum() - 1.77e7) < 0.01 * 1.77e7 and c.min() >= 1000
    # the real particles each discharge represents are unchanged
    np.testing.assert_allclose(c * w, c0 * w0, rtol=1e-12)


def test_bench_schedule_string_is_applied_as_given():
    class Sim:
        def __init__(self):
            self.tiles, self.events = None, None

        def config_tiles(self, ppt, threads, sort_every, compact_every):
            self.tiles = (ppt, threads, sort_every, compact_every)

        def config_events(self, in_push):
            self.events = in_push

    sim = Sim()
    out = bench.tuned(sim, "4,1024,32,0")
    assert sim.tiles == (4, 1024, 0, 32) and sim.events is False
    assert out["choice"] == dict(ppt=4, threads=1024, sort_every=0, compact_every=32, fuse=0)
    sim = Sim()
    assert bench.tuned(sim, False) == dict(choice="default") and sim.tiles is None
