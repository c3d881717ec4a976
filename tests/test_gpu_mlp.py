"""Parity of the BF16 matrix-core warm-start network with the FP64 reference
(oracle/mlp.py), through the pic_mlp C ABI.

Tolerances: the products round both operands to BF16 (8 significant bits,
relative rounding 2^-9) and accumulate in FP32, so a layer output carries a
relative error of order 2^-9 sqrt(depth); gradients are compared per layer by
cosine >= 0.999 and relative L2 <= 2e-2, outputs by relative L2 <= 2e-2.
Adam's arithmetic is FP32 elementwise and is compared to 1e-6 of the step.
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as ref

pytestmark = pytest.mark.gpu

SMALL = (5, 8, 8, 8, 6)


@pytest.fixture(scope="module")
def P():
    import paper_2609_17151_amd as P
    return P


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def per_layer(g, widths):
    return ref.split(g, widths)


@pytest.mark.parametrize("widths,batch", [(W.WARM_WIDTHS, 300), (SMALL, 37), (W.WARM_WIDTHS, 1)])
def test_forward_matches_reference(P, widths, batch):
    p = W.mlp_init(widths, seed=11)
    p[np.arange(p.size) % 7 == 0] += 0.05                     # non-zero biases
    x, _ = W.mlp_batch(batch, widths[0], widths[-1], seed=12)
    net = P.MLP(widths, max_batch=512)
    net.set_params(p)
    y = net.forward(x).cpu().numpy()
    y_ref, _ = ref.forward(p.astype(np.float32).astype(np.float64), widths, x.astype(np.float32))
    assert y.shape == (batch, widths[-1])
    assert rel_l2(y, y_ref) <= 2e-2
    net.close()


def test_first_layer_exact_up_to_bf16(P):
    # one layer, K = 6: products of BF16-rounded operands summed in FP32 are
    # the FP64 sum of the same rounded operands to FP32 accuracy
    widths = (5, 40)
    p = W.mlp_init(widths, seed=13) + 0.01
    x, _ = W.mlp_batch(70, 5, 40, seed=14)
    net = P.MLP(widths, max_batch=128)
    net.set_params(p)
    y = net.forward(x).cpu().numpy().astype(np.float64)
    Wa = bf16_round(p).reshape(40, 6)
    xa = np.hstack([bf16_round(x), np.ones((70, 1))])
    y_ref = xa @ Wa.T
    np.testing.assert_allclose(y, y_ref, rtol=1e-5, atol=1e-6)
    net.close()


@pytest.mark.parametrize("widths,batch", [(W.WARM_WIDTHS, 200), (SMALL, 37)])
def test_gradient_matches_reference(P, widths, batch):
    p = W.mlp_init(widths, seed=21) + 0.01
    x, t = W.mlp_batch(batch, widths[0], widths[-1], seed=22)
    net = P.MLP(widths, max_batch=256)
    net.set_params(p)
    loss, g = net.grad(x, t)
    loss_ref, g_ref = ref.loss_and_grad(p.astype(np.float32).astype(np.float64), widths, x.astype(np.float32),
                                        t.astype(np.float32))
    assert loss == pytest.approx(loss_ref, rel=2e-2)
    for gl, rl in zip(per_layer(g.astype(np.float64), widths), per_layer(g_ref, widths)):
        assert cosine(gl.ravel(), rl.ravel()) >= 0.999
        assert rel_l2(gl.ravel(), rl.ravel()) <= 2e-2
    # deterministic: the same batch gives the same bits
    loss2, g2 = net.grad(x, t)
    assert loss2 == loss and np.array_equal(g, g2)
    net.close()


def test_adam_first_update(P):
    widths = SMALL
    p = (W.mlp_init(widths, seed=31) + 0.01).astype(np.float32)
    x, t = W.mlp_batch(50, widths[0], widths[-1], seed=32)
    net = P.MLP(widths, max_batch=64)
    net.set_params(p)
    _, g = net.grad(x, t)
    lr, eps = 1e-2, 1e-8
    loss = net.train_step(x, t, lr=lr, eps=eps)
    p1 = net.params().astype(np.float64)
    # first update: m_hat = g, v_hat = g^2 (from the same FP32 gradient)
    g64 = g.astype(np.float64)
    expect = p.astype(np.float64) - lr * g64 / (np.abs(g64) + eps)
    assert np.abs(p1 - expect).max() <= 1e-6 * lr + 1e-7
    assert float(loss.cpu()[0]) == pytest.approx(ref.loss_and_grad(p.astype(np.float64), widths, x, t)[0], rel=2e-2)
    net.close()


def test_training_tracks_reference(P):
    widths = (5, 64, 64, 64, 24)
    p = W.mlp_init(widths, seed=41)
    x, _ = W.mlp_batch(256, 5, 24, seed=42)
    grid = np.linspace(0.0, 1.0, 24)
    t = np.tanh(x[:, :1]) * np.sin(np.pi * grid) + 0.3 * x[:, 1:2] * grid   # smooth profiles
    steps, lr = 300, 3e-3
    _, hist_ref = ref.train(p, widths, x, t, steps=steps, lr=lr)
    net = P.MLP(widths, max_batch=256)
    net.set_params(p)
    import torch
    xd = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    td = torch.as_tensor(t, dtype=torch.float32, device="cuda")
    losses = [net.train_step(xd, td, lr=lr) for _ in range(steps)]
    hist = np.array([float(v.cpu()[0]) for v in losses])
    assert hist[0] == pytest.approx(hist_ref[0], rel=2e-2)
    assert hist[-1] < 0.05 * hist[0]
    assert hist[-1] <= 2.0 * hist_ref[-1] + 1e-4
    net.close()


def test_argument_errors(P):
    net = P.MLP(SMALL, max_batch=8)
    x, t = W.mlp_batch(9, 5, 6, seed=1)
    with pytest.raises(P.PicError):
        net.forward(x)                                  # batch above the maximum
    with pytest.raises(P.PicError):
        net.set_params(np.zeros(3, dtype=np.float32))   # wrong parameter count
    with pytest.raises(P.PicError):
        net.train_step(x[:4], t[:4], lr=-1.0)
    net.close()
