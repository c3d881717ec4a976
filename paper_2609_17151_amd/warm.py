"""Learned warm start of RF discharges.

A network maps the parameters of a discharge (pressure, voltage amplitude,
frequency, gap, secondary-emission yield) to its converged, time-averaged
electron density, ion density and electron mean-energy profiles (steady.NPTS
points each).  The prediction only replaces the uniform cold start: the
discharge is started from the predicted profiles (pic_load_profiles) and the
plain method then runs to its own periodic steady state.  The paper's nearest
counterpart is resuming a converged case after a parameter change (Section 2).

Inputs, scaled to about [0, 1]: ln p over [ln 10, ln 200] mTorr, V / 400,
ln f over [ln 2, ln 60] MHz, gap / 4 cm, gamma / 0.2.  Outputs: steady's
features (log10 densities, mean energy), standardised with the training set's
mean and standard deviation per output.
"""
from __future__ import annotations

import math

import numpy as np

import workloads as W

from . import steady

E_CHARGE = 1.602176634e-19
K_BOLTZMANN = 1.380649e-23


def inputs(draw):
    return np.array([
        (math.log(draw["pressure_mtorr"]) - math.log(10.0)) / (math.log(200.0) - math.log(10.0)),
        draw["v_amp"] / 400.0,
        (math.log(draw.get("freq", 13.56e6)) - math.log(2e6)) / (math.log(60e6) - math.log(2e6)),
        draw["gap"] / 0.04,
        draw.get("see_gamma", 0.1) / 0.2,
    ])


def steps_per_period(draw, dt=W.RF_DT):
    return max(1, int(round(1.0 / (draw.get("freq", 13.56e6) * dt))))


def config(draw, weight=W.PILOT_WEIGHT, seed=1, n_init=100_000, capacity=1 << 20, cold=True):
    """The discharge of a parameter draw; a cold start (uniform plasma) or an
    empty one to be filled by a warm start."""
    freq = draw.get("freq", 13.56e6)
    cfg = W.argon_rf(gap=draw["gap"], n_cells=draw["n_cells"], pressure_mtorr=draw["pressure_mtorr"],
                     v_amp=draw["v_amp"], freq=freq, see_gamma=draw.get("see_gamma", 0.1), weight=weight,
                     n_init=n_init, capacity=capacity, seed=seed, dt=W.RF_DT)
    if not cold:
        for sp in cfg["species"]:
            sp["load"] = W.LOAD_NONE
            sp["n_init"] = 0
    return cfg


class Model:
    """The warm-start network on the GPU (paper_2609_17151_amd.MLP) with its
    input and output scaling."""

    def __init__(self, widths=W.WARM_WIDTHS, seed=7, max_batch=4096):
        from . import MLP
        self.widths = tuple(widths)
        self.net = MLP(self.widths, max_batch)
        self.net.set_params(W.mlp_init(self.widths, seed=seed))
        self.mean = np.zeros(self.widths[-1])
        self.std = np.ones(self.widths[-1])
        self.history = []

    def fit(self, X, Y, steps=4000, lr=1e-3, lr_end=1e-5, batch=128, seed=0):
        """Adam on minibatches of the standardised targets, the learning rate
        decaying geometrically from lr to lr_end."""
        import torch
        X = np.asarray(X, dtype=np.float64)
        Y = np.asarray(Y, dtype=np.float64)
        self.mean = Y.mean(axis=0)
        self.std = np.maximum(Y.std(axis=0), 1e-6)
        Z = (Y - self.mean) / self.std
        xh = X.astype(np.float32)
        zh = Z.astype(np.float32)
        rng = np.random.default_rng(seed)
        n = len(X)
        batch = min(batch, n)
        # device memory for one minibatch and the losses; the minibatch rows
        # are picked on the host and copied in (torch only holds memory here)
        xb = torch.empty((batch, xh.shape[1]), dtype=torch.float32, device="cuda")
        zb = torch.empty((batch, zh.shape[1]), dtype=torch.float32, device="cuda")
        losses = torch.empty(steps, dtype=torch.float32, device="cuda")
        for k in range(steps):
            rate = lr * (lr_end / lr) ** (k / max(steps - 1, 1))
            idx = rng.choice(n, size=batch, replace=False)
            xb.copy_(torch.from_numpy(xh[idx]))
            zb.copy_(torch.from_numpy(zh[idx]))
            self.net.train_step(xb, zb, lr=rate, loss_out=losses[k:k + 1])
        self.history = [float(v) for v in losses.cpu().numpy()]
        return self

    def predict(self, X):
        """Network features (steady.to_features layout) for inputs X."""
        z = self.net.forward(np.asarray(X, dtype=np.float64)).cpu().numpy().astype(np.float64)
        return z * self.std + self.mean

    def loss(self, X, Y):
        """Mean squared error of the standardised outputs."""
        Z = (np.asarray(Y) - self.mean) / self.std
        P = (self.predict(X) - self.mean) / self.std
        return float(np.mean((P - Z) ** 2))

    def state(self):
        return dict(widths=np.array(self.widths), params=self.net.params(), mean=self.mean, std=self.std)

    def set_state(self, st):
        self.net.set_params(st["params"])
        self.mean, self.std = np.asarray(st["mean"]), np.asarray(st["std"])


def start_from_features(sim, batch, cfg, feats):
    """Fill discharge `batch` of `sim` from predicted features: n_s macros with
    n_s = integral of the density / weight, electrons at T = (2/3) <eps>, ions
    at the gas temperature."""
    prof = steady.from_features(feats)
    m = prof.shape[1]
    L = cfg["length"]
    xs = np.linspace(0.0, L, m)
    dens = np.stack([prof[0], prof[1]])
    counts = []
    for s in range(2):
        total = float(np.sum(0.5 * (dens[s][1:] + dens[s][:-1]) * np.diff(xs)))
        cap = cfg["species"][s]["capacity"]
        counts.append(int(min(cap, max(0, round(total / cfg["species"][s]["weight"])))))
    te = (2.0 / 3.0) * prof[2]
    ti = np.full(m, K_BOLTZMANN * cfg["gas_temp"] / E_CHARGE)
    sim.load_profiles(dens, np.stack([te, ti]), counts, batch=batch)
    return counts
