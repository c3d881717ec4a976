"""Host logic of the warm start: draws to configurations, the particle
counts and temperatures handed to pic_load_profiles, and empty discharges for
warm starts (driven by a stand-in context)."""
import numpy as np
import pytest

import workloads as W
from paper_2609_17151_amd import steady, warm


class Capture:
    def __init__(self):
        self.calls = []

    def load_profiles(self, dens, temp, n, batch=0):
        self.calls.append((np.array(dens), np.array(temp), list(n), batch))


def test_config_cold_and_empty():
    d = W.warm_draws(3, seed=1, f_range=(10e6, 50e6))[0]
    cold = warm.config(d, weight=1e9)
    empty = warm.config(d, weight=1e9, cold=False)
    assert cold["dt"] == W.RF_DT and cold["v_freq"] == d["freq"] and cold["length"] == d["gap"]
    assert all(sp["n_init"] > 0 for sp in cold["species"])
    assert all(sp["n_init"] == 0 and sp["load"] == W.LOAD_NONE for sp in empty["species"])
    assert warm.steps_per_period(d) == round(1.0 / (d["freq"] * W.RF_DT))


def test_start_from_features_counts_and_temperatures():
    d = dict(pressure_mtorr=30.0, v_amp=200.0, freq=13.56e6, gap=0.025, n_cells=400, see_gamma=0.1)
    cfg = warm.config(d, weight=1e9, capacity=10_000_000)
    x = np.linspace(0.0, 1.0, steady.NPTS)
    ne = 2e15 * np.sin(np.pi * x) ** 2
    ni = 3e15 * np.sin(np.pi * x)
    eps = 1.5 + 3.0 * x
    feats = steady.to_features(np.stack([ne, ni, eps]))
    sim = Capture()
    n = warm.start_from_features(sim, 5, cfg, feats)
    dens, temp, counts, batch = sim.calls[0]
    assert batch == 5 and counts == n
    # integral of sin^2 over the gap is gap/2, of sin is 2 gap / pi
    assert n[0] == pytest.approx(2e15 * 0.025 / 2 / 1e9, rel=1e-3)
    assert n[1] == pytest.approx(3e15 * 0.025 * 2 / np.pi / 1e9, rel=1e-3)
    np.testing.assert_allclose(temp[0], 2.0 / 3.0 * eps, rtol=1e-9)
    assert np.allclose(temp[1], 1.380649e-23 * 300.0 / 1.602176634e-19)
    np.testing.assert_allclose(dens[0], ne, rtol=1e-9, atol=1e4)


def test_counts_clipped_to_capacity():
    d = dict(pressure_mtorr=30.0, v_amp=200.0, freq=13.56e6, gap=0.025, n_cells=400, see_gamma=0.1)
    cfg = warm.config(d, weight=1.0, capacity=1000)
    feats = steady.to_features(np.stack([np.full(256, 1e15)] * 2 + [np.full(256, 3.0)]))
    sim = Capture()
    assert warm.start_from_features(sim, 0, cfg, feats) == [1000, 1000]
