"""Batched sweeps of RF discharges on one context, each with its own RF period.

All discharges of a context advance together, one step at a time, but every
discharge has its own number of steps per RF period; a window is a whole
number of that discharge's periods.  A discharge is retired once it has run
its periods or once a caller-supplied rule says it is done; retired
discharges cost nothing in later steps.  A discharge whose device flags latch
(capacity overflow, non-finite values, ...) is retired and its flags kept.

Two ways to take the windows:
  * chunk > 0 (default): every discharge's windows are closed on the device
    by the step itself (pic_set_windows); the host steps the batch in chunks
    of `chunk` steps and then reads the windows each running discharge has
    completed, so nothing waits on the host between window ends.  A discharge
    may run up to one chunk past its last window before it is retired.
  * chunk = 0: the batch is advanced to the next window boundary of any
    discharge and that discharge's averages are read and cleared there (one
    host synchronisation per window).
"""
from __future__ import annotations

import time

import numpy as np

from . import steady


class Sweep:
    def __init__(self, sim, steps_per_period, window_periods=5, max_periods=300, electron=0, ion=1,
                 progress=20.0, chunk=2048, tune=False, tune_cache=None, retune=True):
        self.sim = sim
        self.tune = bool(tune)
        self.tune_cache = tune_cache
        self.retune = bool(retune)
        self.schedule = None                            # the autotuner's choice, when tuned
        self.schedules = []                             # (step, running discharges, choice) of every tuning
        self._tuned_running = 0
        self.chunk = int(chunk)
        self.B = sim.B
        self.spp = [int(s) for s in steps_per_period]
        if len(self.spp) != self.B or min(self.spp) < 1:
            raise ValueError("one positive steps-per-period value per discharge")
        self.window_periods = int(window_periods)
        self.max_periods = int(max_periods)
        self.electron, self.ion = electron, ion
        self.windows = [[] for _ in range(self.B)]      # [3, NPTS] profiles per window
        self.window_time = [[] for _ in range(self.B)]  # wall seconds at the end of each window
        self.window_step = [[] for _ in range(self.B)]
        self.done = [False] * self.B
        self.flags = [0] * self.B                       # latched device conditions, per discharge
        self.steps = 0
        self.t0 = None
        self.progress = progress                        # seconds between progress lines (0: none)

    def window_steps(self, b):
        return self.window_periods * self.spp[b]

    def _tune(self, cache=None):
        """Time the step schedules on the batch itself (real steps) and apply
        the fastest; returns the steps the tuning took."""
        from . import autotune
        running = [b for b in range(self.B) if not self.done[b]]
        s0 = self.sim.counts(running[0])["step"]
        self.schedule, _ = autotune.tune(self.sim, steps=16, warm=8, cache=cache)
        took = self.sim.counts(running[0])["step"] - s0
        self._tuned_running = len(running)
        self.schedules.append((int(s0), len(running), self.schedule))
        return took

    def run(self, stop=None):
        """Advance until every discharge is done.  `stop(b, sweep)` is called
        after each window of discharge b; a true result retires it early.
        With tune=True the autotuner first picks the step schedule on the
        batch (its steps come before the first window, inside the wall time),
        and with retune (device windows) again whenever the running
        discharges have halved since, as a smaller batch can favour another
        schedule (its steps count as steps of the run)."""
        t_start = time.perf_counter()
        if self.tune:
            self._tune(self.tune_cache)
        if self.chunk > 0:
            return self._run_device(stop, t_start)
        sim = self.sim
        sim.set_diag(True)
        for b in range(self.B):
            sim.reset_avg(b)
        start = sim.counts(0)["step"]
        nxt = [start + self.window_steps(b) for b in range(self.B)]
        self.t0 = t_start
        self.steps = start
        last = self.t0
        while not all(self.done):
            now = time.perf_counter()
            if self.progress and now - last >= self.progress:
                last = now
                print("sweep: step %d, %d of %d discharges running, %.0f s"
                      % (self.steps, self.done.count(False), self.B, now - self.t0), flush=True)
            target = min(nxt[b] for b in range(self.B) if not self.done[b])
            sim.step(target - self.steps)
            self.steps = target
            for b in range(self.B):
                if self.done[b] or nxt[b] != target:
                    continue
                self.windows[b].append(steady.window(sim, b, self.electron, self.ion))
                self.window_time[b].append(time.perf_counter() - self.t0)
                self.window_step[b].append(target)
                nxt[b] += self.window_steps(b)
                periods = len(self.windows[b]) * self.window_periods
                self.flags[b] = sim.counts(b)["flags"]
                if self.flags[b] or periods >= self.max_periods or (stop is not None and stop(b, self)):
                    sim.retire(b)
                    self.done[b] = True
        sim.sync(check=False)
        return self

    def _window_done(self, b, w, step, wall, stop):
        self.windows[b].append(np.stack([steady.resample(w["density"][self.electron]),
                                         steady.resample(w["density"][self.ion]),
                                         steady.resample(w["mean_energy"])]))
        self.window_time[b].append(wall)
        self.window_step[b].append(step)
        periods = len(self.windows[b]) * self.window_periods
        return periods >= self.max_periods or (stop is not None and stop(b, self))

    def _run_device(self, stop, t_start):
        sim = self.sim
        sim.set_diag(True)
        for b in range(self.B):
            if self.chunk > 32 * self.window_steps(b):
                raise ValueError("a chunk would span more windows than the device ring holds")
            sim.set_windows(b, self.window_steps(b))
        start = sim.counts(0)["step"]
        self.t0 = t_start
        self.steps = start
        last = time.perf_counter()
        while not all(self.done):
            t_a, s_a = time.perf_counter() - self.t0, self.steps
            sim.step(self.chunk)
            sim.sync(check=False)                       # the chunk's end in wall time
            self.steps += self.chunk
            t_b = time.perf_counter() - self.t0
            for b in range(self.B):
                if self.done[b]:
                    continue
                new = sim.windows(b, first=len(self.windows[b]))
                retire = False
                for w in new:
                    k = len(self.windows[b])
                    step = start + (k + 1) * self.window_steps(b)
                    # the window's end, placed in the chunk's wall time
                    wall = t_a + (t_b - t_a) * (step - s_a) / self.chunk
                    if self._window_done(b, w, step, wall, stop):
                        retire = True
                        break
                self.flags[b] = sim.counts(b)["flags"]
                if retire or self.flags[b]:
                    sim.retire(b)
                    sim.set_windows(b, 0)
                    self.done[b] = True
            running = self.done.count(False)
            if self.tune and self.retune and 0 < running <= self._tuned_running // 2:
                self.steps += self._tune()
            now = time.perf_counter()
            if self.progress and now - last >= self.progress:
                last = now
                print("sweep: step %d, %d of %d discharges running, %.0f s"
                      % (self.steps, self.done.count(False), self.B, now - self.t0), flush=True)
        sim.sync(check=False)
        return self

    def reference(self, b, span=50):
        """Mean of the windows of discharge b over its last `span` periods
        (periods 251-300 of a 300-period run)."""
        nw = max(1, span // self.window_periods)
        ws = self.windows[b][-nw:]
        if len(ws) < nw:
            raise ValueError("the run is shorter than the reference span")
        return np.mean(ws, axis=0)
