"""Pins of the residual-network oracle (oracle/residual.py), CPU only.

- against a model assembled from torch's own layers (nn.Linear, nn.ReLU,
  nn.BatchNorm1d in eval mode with running statistics) in FP64, wired as Sec. IV-A and
  Fig. 1 describe: initial linear, blocks of linear -> ReLU -> BatchNorm with a skip
  connection and the network input concatenated to each block's input, final linear;
- closed forms: with gamma = beta = 0 every block is the identity, so the network is
  the composition of the first and last linear layers; a one-block network on a
  hand-sized example;
- pack/unpack round trip and the parameter count;
- the BF16 emulation stays within BF16 error of the FP64 forward.
"""
import numpy as np
import pytest
import torch

import svgen
from oracle import residual as ores

IN = 15


class TorchResNet(torch.nn.Module):
    def __init__(self, in_dim, width, n_blocks, bn_eps):
        super().__init__()
        self.first = torch.nn.Linear(in_dim, width)
        self.lin = torch.nn.ModuleList([torch.nn.Linear(width + in_dim, width) for _ in range(n_blocks)])
        self.bn = torch.nn.ModuleList([torch.nn.BatchNorm1d(width, eps=bn_eps) for _ in range(n_blocks)])
        self.last = torch.nn.Linear(width, 1)

    def forward(self, x):
        h = self.first(x)
        for lin, bn in zip(self.lin, self.bn):
            h = h + bn(torch.relu(lin(torch.cat([h, x], dim=1))))
        return self.last(h)[:, 0]


def torch_model(flat, in_dim, width, n_blocks, bn_eps):
    net = ores.unpack(flat, in_dim, width, n_blocks)
    m = TorchResNet(in_dim, width, n_blocks, bn_eps).double().eval()
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    with torch.no_grad():
        m.first.weight.copy_(t(net["W0"]))
        m.first.bias.copy_(t(net["b0"]))
        for lin, bn, blk in zip(m.lin, m.bn, net["blocks"]):
            lin.weight.copy_(t(np.concatenate([blk["Wh"], blk["Wx"]], axis=1)))
            lin.bias.copy_(t(blk["c"]))
            bn.weight.copy_(t(blk["gamma"]))
            bn.bias.copy_(t(blk["beta"]))
            bn.running_mean.copy_(t(blk["mu"]))
            bn.running_var.copy_(t(blk["var"]))
        m.last.weight.copy_(t(net["w_out"][None, :]))
        m.last.bias.copy_(t([net["b_out"]]))
    return m


def rows(n, seed):
    g = np.random.default_rng(seed)
    return np.concatenate([g.uniform(-0.6, 0.6, (n, 3)), g.uniform(-3.0, 3.0, (n, IN - 3))], axis=1)


@pytest.mark.parametrize("width,n_blocks", [(32, 1), (64, 3), (128, 5)])
def test_against_torch_layers(width, n_blocks):
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 10 + n_blocks)
    X = rows(200, n_blocks)
    eps = 1e-5
    ref = torch_model(flat, IN, width, n_blocks, eps)(torch.as_tensor(X)).detach().numpy()
    got = ores.forward(flat, IN, width, n_blocks, X, eps)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_identity_blocks_close_form():
    width, n_blocks = 48, 4
    net = ores.unpack(svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 3), IN, width, n_blocks)
    for blk in net["blocks"]:
        blk["gamma"][:] = 0.0
        blk["beta"][:] = 0.0
    flat = ores.pack(net)
    X = rows(50, 4)
    expect = (X @ net["W0"].T + net["b0"]) @ net["w_out"] + net["b_out"]
    np.testing.assert_allclose(ores.forward(flat, IN, width, n_blocks, X, 1e-5), expect, rtol=1e-13, atol=1e-13)


def test_one_block_by_hand():
    """in_dim 1, width 2: every term written out."""
    net = {"W0": np.array([[2.0], [-1.0]]), "b0": np.array([0.5, 0.25]),
           "blocks": [{"Wh": np.array([[1.0, 0.0], [0.5, 2.0]]), "Wx": np.array([[1.0], [-3.0]]),
                       "c": np.array([0.0, 1.0]), "gamma": np.array([2.0, 1.0]), "beta": np.array([0.5, -0.5]),
                       "mu": np.array([1.0, 0.0]), "var": np.array([4.0, 1.0])}],
           "w_out": np.array([1.0, 10.0]), "b_out": 3.0}
    flat = ores.pack(net)
    x = 1.0
    h0 = np.array([2.0 * x + 0.5, -x + 0.25])                       # [2.5, -0.75]
    z = np.array([h0[0] + x, 0.5 * h0[0] + 2.0 * h0[1] - 3.0 * x + 1.0])   # [3.5, -2.25]
    a = np.maximum(z, 0.0)                                           # [3.5, 0]
    eps = 0.0
    bn = np.array([2.0 * (a[0] - 1.0) / 2.0 + 0.5, 1.0 * (a[1] - 0.0) / 1.0 - 0.5])   # [3.0, -0.5]
    h1 = h0 + bn                                                     # [5.5, -1.25]
    expect = h1[0] * 1.0 + h1[1] * 10.0 + 3.0                        # -4.0
    assert expect == -4.0
    got = ores.forward(flat, 1, 2, 1, np.array([[x]]), eps)
    np.testing.assert_allclose(got, [expect], rtol=0, atol=1e-14)


def test_pack_roundtrip_and_count():
    spec = svgen.ResSpec(IN, 64, 3)
    flat = svgen.res_init(spec, 5).astype(np.float64)
    assert flat.size == ores.n_params(IN, 64, 3) == spec.n_params
    np.testing.assert_array_equal(ores.pack(ores.unpack(flat, IN, 64, 3)), flat)
    with pytest.raises(ValueError):
        ores.unpack(flat[:-1], IN, 64, 3)


def test_bf16_emulation_close_to_fp64():
    width, n_blocks = 128, 5
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 21)
    X = rows(300, 9).astype(np.float32)
    y = ores.forward(flat, IN, width, n_blocks, X, 1e-5)
    yb = ores.forward_bf16(flat, IN, width, n_blocks, X, 1e-5)
    err = np.abs(yb - y) / (1.0 + np.abs(y))
    assert err.max() < 2e-2
    assert err.mean() < 5e-3


# ---------------------------------------------------------------- training form
def _torch_grads(m):
    """Gradients of the torch model in the flat layout (running statistics: zero)."""
    parts = [m.first.weight.grad.reshape(-1), m.first.bias.grad]
    W = m.first.weight.shape[0]
    for lin, bn in zip(m.lin, m.bn):
        g = lin.weight.grad
        parts += [g[:, :W].reshape(-1), g[:, W:].reshape(-1), lin.bias.grad, bn.weight.grad, bn.bias.grad,
                  torch.zeros(W, dtype=torch.float64), torch.zeros(W, dtype=torch.float64)]
    parts += [m.last.weight.grad.reshape(-1), m.last.bias.grad]
    return torch.cat(parts).numpy()


@pytest.mark.parametrize("width,n_blocks,B", [(32, 3, 96), (64, 1, 40), (16, 5, 200)])
def test_training_pass_matches_torch_batchnorm(width, n_blocks, B):
    """Loss, gradient and running statistics of the batch-statistic forward pass against
    torch's layers in training mode (nn.BatchNorm1d normalising with the batch's
    statistics, momentum 0.1), with autograd in FP64."""
    eps = 1e-5
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 31).astype(np.float64)
    X = rows(B, 32)
    t = np.random.default_rng(33).uniform(-0.15, 0.3, B)
    sigma = 0.1
    loss, g = ores.loss_and_grad_train(flat, IN, width, n_blocks, X, t, sigma, eps)
    m = torch_model(flat, IN, width, n_blocks, eps).train()
    pred = m(torch.tensor(X))
    L = torch.mean(torch.abs(pred - torch.clamp(torch.tensor(t), -sigma, sigma)))
    L.backward()
    assert loss == pytest.approx(L.item(), rel=1e-13)
    np.testing.assert_allclose(g, _torch_grads(m), rtol=1e-9, atol=1e-13)
    upd = ores.running_update(flat, IN, width, n_blocks, X, eps)
    net = ores.unpack(upd, IN, width, n_blocks)
    for blk, bn in zip(net["blocks"], m.bn):
        np.testing.assert_allclose(blk["mu"], bn.running_mean.numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(blk["var"], bn.running_var.numpy(), rtol=1e-12, atol=1e-14)


def test_training_forward_normalises_each_block():
    """After a block's BatchNorm in training form, gamma = 1 and beta = 0 leave every
    feature with batch mean 0 and batch variance v / (v + eps) (v its raw variance);
    with gamma = 0 the block adds beta only."""
    width, n_blocks, B, eps = 24, 2, 64, 1e-5
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 41).astype(np.float64)
    net = ores.unpack(flat, IN, width, n_blocks)
    for blk in net["blocks"]:
        blk["gamma"][:] = 1.0
        blk["beta"][:] = 0.0
    X = rows(B, 42)
    _, c = ores.forward_train(ores.pack(net), IN, width, n_blocks, X, eps)
    for i in range(n_blocks):
        d = c["h"][i + 1] - c["h"][i]
        np.testing.assert_allclose(d.mean(axis=0), 0.0, atol=1e-12)
        np.testing.assert_allclose(d.var(axis=0), c["v"][i] / (c["v"][i] + eps), rtol=1e-10)
    for blk in net["blocks"]:
        blk["gamma"][:] = 0.0
        blk["beta"][:] = 0.25
    _, c = ores.forward_train(ores.pack(net), IN, width, n_blocks, X, eps)
    for i in range(n_blocks):
        np.testing.assert_allclose(c["h"][i + 1] - c["h"][i], 0.25, rtol=0, atol=1e-15)


def test_training_gradient_matches_central_differences():
    """FP64 central differences of the batch-statistic loss (targets far from the
    predictions, so the loss is smooth in theta)."""
    width, n_blocks, B, eps = 8, 2, 30, 1e-5
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 51).astype(np.float64)
    X = rows(B, 52)
    y, _ = ores.forward_train(flat, IN, width, n_blocks, X, eps)
    t = y + np.where(np.arange(B) % 2 == 0, 0.5, -0.5)
    _, g = ores.loss_and_grad_train(flat, IN, width, n_blocks, X, t, 10.0, eps)
    net = ores.unpack(flat, IN, width, n_blocks)
    skip = set()   # running statistics have zero gradient by definition
    off = IN * width + width
    for _ in range(n_blocks):
        base = off + width * width + width * IN + 3 * width
        skip |= set(range(base, base + 2 * width))
        off += width * width + width * IN + 5 * width
    rng = np.random.default_rng(53)
    idx = [i for i in rng.choice(flat.size, 120, replace=False) if i not in skip]
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp = np.mean(np.abs(ores.forward_train(flat + e, IN, width, n_blocks, X, eps)[0] - t))
        lm = np.mean(np.abs(ores.forward_train(flat - e, IN, width, n_blocks, X, eps)[0] - t))
        assert g[i] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9), i
    assert len(idx) > 60
    assert not any(g[i] for i in skip)


def test_training_bf16_emulation_reduces_to_fp64():
    """Without rounding the emulation is the FP64 training gradient; with it, the
    gradient moves by a measurable amount that stays within 10% (the BatchNorm backward
    amplifies the forward roundings of relative size 2^-9)."""
    width, n_blocks, B, eps = 64, 2, 200, 1e-5
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 61).astype(np.float64)
    X = rows(B, 62)
    y, _ = ores.forward_train(flat, IN, width, n_blocks, X, eps)
    t = y + np.where(np.arange(B) % 2 == 0, 0.5, -0.5)
    l0, g0 = ores.loss_and_grad_train(flat, IN, width, n_blocks, X, t, 10.0, eps)
    l1, g1 = ores.loss_and_grad_train_bf16(flat, IN, width, n_blocks, X, t, 10.0, eps, rounding=False)
    assert l1 == pytest.approx(l0, rel=1e-14)
    np.testing.assert_allclose(g1, g0, rtol=1e-10, atol=1e-15)
    l2, g2 = ores.loss_and_grad_train_bf16(flat, IN, width, n_blocks, X, t, 10.0, eps)
    assert abs(l2 - l0) < 1e-2 * l0
    rel = np.linalg.norm(g2 - g0) / np.linalg.norm(g0)
    assert 1e-4 < rel < 0.1, rel
