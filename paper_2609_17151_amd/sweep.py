"""Batched sweeps of RF discharges on one context, each with its own RF period.

All discharges of a context advance together, one step at a time, but every
discharge has its own number of steps per RF period.  The driver advances the
batch to the next window boundary of any discharge (a window is a whole
number of that discharge's periods), reads and clears that discharge's time
averages (steady.window), and retires a discharge once it has run its
periods or once a caller-supplied rule says it is done; retired discharges
cost nothing in later steps.  A discharge whose device flags latch (capacity
overflow, non-finite values, ...) is retired at once and its flags kept.
"""
from __future__ import annotations

import time

import numpy as np

from . import steady


class Sweep:
    def __init__(self, sim, steps_per_period, window_periods=5, max_periods=300, electron=0, ion=1,
                 progress=20.0):
        self.sim = sim
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

    def run(self, stop=None):
        """Advance until every discharge is done.  `stop(b, sweep)` is called
        after each window of discharge b; a true result retires it early."""
        sim = self.sim
        sim.set_diag(True)
        for b in range(self.B):
            sim.reset_avg(b)
        start = sim.counts(0)["step"]
        nxt = [start + self.window_steps(b) for b in range(self.B)]
        self.t0 = time.perf_counter()
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

    def reference(self, b, span=50):
        """Mean of the windows of discharge b over its last `span` periods
        (periods 251-300 of a 300-period run)."""
        nw = max(1, span // self.window_periods)
        ws = self.windows[b][-nw:]
        if len(ws) < nw:
            raise ValueError("the run is shorter than the reference span")
        return np.mean(ws, axis=0)
