"""Host logic of the steady-state rule, the network features and the sweep
scheduler (per-discharge RF windows, retirement), driven by a stand-in
context that records what it is asked to do."""
import numpy as np
import pytest

from paper_2609_17151_amd import steady, warm
from paper_2609_17151_amd.sweep import Sweep


def test_resample_endpoints_and_linearity():
    y = np.linspace(3.0, 7.0, 401)
    r = steady.resample(y)
    assert r.shape == (steady.NPTS,)
    assert r[0] == 3.0 and r[-1] == 7.0
    np.testing.assert_allclose(r, np.linspace(3.0, 7.0, steady.NPTS), atol=1e-12)


def test_converged_at_needs_a_run_of_windows():
    ref = np.ones((3, 8))
    near, far = ref * 1.01, ref * 1.05
    ws = [far] * 5 + [near] * 9 + [far] + [near] * 10
    assert steady.converged_at(ws, ref) == 15
    assert steady.converged_at(ws[:24], ref) is None
    # every profile must be within the tolerance
    mixed = np.ones((3, 8))
    mixed[2] *= 1.03
    assert steady.converged_at([mixed] * 12, ref) is None


def test_features_round_trip():
    rng = np.random.default_rng(1)
    prof = np.stack([rng.uniform(0, 2e15, 256), rng.uniform(0, 2e15, 256), rng.uniform(0.5, 6, 256)])
    back = steady.from_features(steady.to_features(prof))
    np.testing.assert_allclose(back, prof, rtol=1e-9, atol=1e3)


def test_inputs_scaled_to_unit_range():
    import workloads as W
    for d in W.warm_draws(200, seed=3):
        x = warm.inputs(d)
        assert np.all(x >= -1e-12) and np.all(x <= 1 + 1e-12)
    assert warm.steps_per_period(dict(freq=13.56e6)) == 1600


class FakeSim:
    """Counts steps; each discharge's time average is its own id plus the step
    it was read at, so windows can be checked."""

    def __init__(self, B):
        self.B, self.S = B, 2
        self.step_no = 0
        self.retired = set()
        self.calls = []

    def set_diag(self, on):
        pass

    def reset_avg(self, b, check=True):
        pass

    def counts(self, b):
        return dict(step=self.step_no, count=[0, 0], flags=0)

    def step(self, n):
        assert n > 0
        self.calls.append(n)
        self.step_no += n

    def avg(self, b, check=True):
        v = np.full(5, b * 1000.0 + self.step_no)
        return dict(density=np.stack([v, v]), phi=v, mean_energy=v, samples=1.0)

    def retire(self, b):
        self.retired.add(b)

    def sync(self, check=True):
        pass


def test_sweep_windows_follow_each_period():
    sim = FakeSim(3)
    spp = [10, 7, 25]
    sw = Sweep(sim, spp, window_periods=2, max_periods=6, chunk=0).run()
    for b in range(3):
        assert sw.window_step[b] == [2 * spp[b] * k for k in (1, 2, 3)]
        assert [w[0][0] for w in sw.windows[b]] == [b * 1000.0 + s for s in sw.window_step[b]]
    assert sim.retired == {0, 1, 2}
    assert sim.step_no == 2 * 25 * 3


def test_sweep_early_stop_retires():
    sim = FakeSim(2)
    sw = Sweep(sim, [4, 4], window_periods=1, max_periods=100, chunk=0)
    sw.run(stop=lambda b, s: b == 0 and len(s.windows[0]) == 3)
    assert len(sw.windows[0]) == 3 and len(sw.windows[1]) == 100
    with pytest.raises(ValueError):
        Sweep(FakeSim(2), [4], window_periods=1, chunk=0)


def test_noise_tolerance():
    assert steady.noise_tolerance([0.5] * 5 + [0.001] * 10) == steady.TOL
    d = [0.3, 0.2] + [0.01, 0.03] * 5
    rms = float(np.sqrt(np.mean(np.array([0.01, 0.03] * 5) ** 2)))
    assert steady.noise_tolerance(d) == pytest.approx(3 * rms)
    assert steady.noise_tolerance([float("nan")] * 3) == steady.TOL


class FakeWindowSim(FakeSim):
    """Closes windows on its own as the device does: a window of discharge b
    ends every `len` steps after set_windows, its mean is b * 1000 + the step
    it ended at; retired discharges close no more windows."""

    def __init__(self, B):
        super().__init__(B)
        self.win = {}

    def set_windows(self, b, steps):
        self.win[b] = (steps, self.step_no, [])

    def step(self, n):
        assert n > 0
        self.calls.append(n)
        for _ in range(n):
            self.step_no += 1
            for b, (ln, st, done) in self.win.items():
                if ln and b not in self.retired and (self.step_no - st) % ln == 0:
                    done.append(self.step_no)

    def windows(self, b, first=0, count=None):
        done = self.win[b][2]
        out = []
        for s in done[first:]:
            v = np.full(5, b * 1000.0 + s)
            out.append(dict(density=np.stack([v, v]), phi=v, mean_energy=v, samples=1.0))
        return out


def test_device_windows_follow_each_period_and_retire():
    sim = FakeWindowSim(3)
    spp = [10, 7, 25]
    sw = Sweep(sim, spp, window_periods=2, max_periods=6, chunk=32).run()
    for b in range(3):
        assert sw.window_step[b] == [2 * spp[b] * k for k in (1, 2, 3)]
        assert [w[0][0] for w in sw.windows[b]] == [b * 1000.0 + s for s in sw.window_step[b]]
        times = sw.window_time[b]
        assert all(t1 >= t0 for t0, t1 in zip(times, times[1:]))
    assert sim.retired == {0, 1, 2}
    assert all(c == 32 for c in sim.calls)
    # the last discharge needed 150 steps: five chunks of 32
    assert sim.step_no == 160


def test_device_windows_early_stop():
    sim = FakeWindowSim(2)
    sw = Sweep(sim, [4, 4], window_periods=1, max_periods=100, chunk=16)
    sw.run(stop=lambda b, s: b == 0 and len(s.windows[0]) == 3)
    # windows after the stopping one are not kept, even inside the same chunk
    assert len(sw.windows[0]) == 3 and len(sw.windows[1]) == 100
    with pytest.raises(ValueError):
        Sweep(FakeWindowSim(1), [1], window_periods=1, chunk=64).run()


def test_retune_when_the_running_discharges_halve(monkeypatch):
    # four discharges of 1, 1, 2 and 4 windows: the schedule is tuned at the
    # start (4 running), again when 2 run, and again when 1 runs
    tuned = []

    def fake_tune(self, cache=None):
        running = self.done.count(False)
        tuned.append(running)
        self._tuned_running = running
        return 0

    monkeypatch.setattr(Sweep, "_tune", fake_tune)
    sim = FakeWindowSim(4)
    lengths = [1, 1, 2, 4]
    sw = Sweep(sim, [8, 8, 8, 8], window_periods=1, max_periods=4, chunk=8, tune=True)
    sw.run(stop=lambda b, s: len(s.windows[b]) >= lengths[b])
    assert tuned == [4, 2, 1]
    sim2 = FakeWindowSim(4)
    tuned.clear()
    Sweep(sim2, [8, 8, 8, 8], window_periods=1, max_periods=4, chunk=8, tune=True, retune=False).run(
        stop=lambda b, s: len(s.windows[b]) >= lengths[b])
    assert tuned == [4]
