"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the GPU library.

The network is not a method of the paper.  The paper restarts a case from a
converged state after a parameter change (Section 2); the warm start replaces
the uniform cold start of a new discharge with density and mean-energy
profiles predicted from the discharge parameters, and the plain method then
runs to its own periodic steady state.

Definitions written out here, in FP64:
  * a fully connected network, layer l: z = W_l a + b_l, with the exact GELU
    g(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 after every hidden layer and
    no activation after the last (Hendrycks and Gimpel, 2016);
  * the loss: mean squared error over every output of every sample,
    L = sum (y - t)^2 / (batch * n_out);
  * its gradient by the chain rule, layer by layer from the output back;
  * Adam (Kingma and Ba, 2015): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
    w <- w - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps) at update k.

Parameter layout (the interface of the GPU library too): one block per layer,
in order, each the row-major matrix [n_out][n_in + 1] whose last column is the
bias, so that a layer is one product with its input extended by a 1.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def n_params(widths):
    """Number of parameters of the network with layer widths `widths`."""
    return sum(widths[i + 1] * (widths[i] + 1) for i in range(len(widths) - 1))


def split(params, widths):
    """Views of the flat parameter vector, one [n_out, n_in + 1] block per layer."""
    out, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        out.append(params[o:o + n_out * (n_in + 1)].reshape(n_out, n_in + 1))
        o += n_out * (n_in + 1)
    assert o == params.size
    return out


def gelu(z):
    """Exact GELU, z Phi(z)."""
    return 0.5 * z * (1.0 + erf(z / _SQRT2))


def gelu_grad(z):
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / _SQRT2)) + z * np.exp(-0.5 * z * z) * _INV_SQRT_2PI


def forward(params, widths, x):
    """Outputs and the per-layer (input, pre-activation) pairs of a batch x [batch, n_in]."""
    W = split(np.asarray(params, dtype=np.float64), widths)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for i, Wa in enumerate(W):
        z = a @ Wa[:, :-1].T + Wa[:, -1]
        cache.append((a, z))
        a = gelu(z) if i < len(W) - 1 else z
    return a, cache


def loss_and_grad(params, widths, x, t):
    """MSE loss and its gradient with respect to the flat parameters."""
    params = np.asarray(params, dtype=np.float64)
    W = split(params, widths)
    y, cache = forward(params, widths, x)
    t = np.asarray(t, dtype=np.float64)
    nb, n_out = y.shape
    d = y - t
    loss = float(np.sum(d * d) / (nb * n_out))
    dz = 2.0 * d / (nb * n_out)                  # dL/dz of the output layer
    grads = [None] * len(W)
    for i in range(len(W) - 1, -1, -1):
        a, _ = cache[i]
        g = np.empty_like(W[i])
        g[:, :-1] = dz.T @ a
        g[:, -1] = dz.sum(axis=0)
        grads[i] = g
        if i > 0:
            da = dz @ W[i][:, :-1]                 # dL/d(activation of layer i-1)
            dz = da * gelu_grad(cache[i - 1][1])
    return loss, np.concatenate([g.ravel() for g in grads])


class Adam:
    """Adam with bias correction, state in FP64."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.k = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, w, g):
        self.k += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.k)
        vh = self.v / (1.0 - self.b2 ** self.k)
        return w - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(params, widths, x, t, steps, lr=1e-3, batch=None, rng=None):
    """Plain Adam training on (x, t), full batch unless `batch` is given; returns
    the parameters and the loss history."""
    w = np.array(params, dtype=np.float64)
    opt = Adam(w.size, lr=lr)
    hist = []
    for _ in range(steps):
        if batch is None:
            xb, tb = x, t
        else:
            idx = rng.choice(len(x), size=batch, replace=False)
            xb, tb = x[idx], t[idx]
        loss, g = loss_and_grad(w, widths, xb, tb)
        hist.append(loss)
        w = opt.step(w, g)
    return w, hist
