"""Pins for the FP64 network oracle: PyTorch FP64 modules, autograd and
torch.optim.Adam as independent library routines, central finite differences,
and closed-form special cases."""
import math

import numpy as np
import pytest
import torch

import svgen
from oracle import mlp as om


def torch_net(flat, in_dim, width, n_hidden):
    layers = []
    dims = [in_dim] + [width] * n_hidden
    for i in range(n_hidden):
        layers += [torch.nn.Linear(dims[i], dims[i + 1]), torch.nn.Softplus(beta=1.0, threshold=1e9)]
    layers.append(torch.nn.Linear(width, 1))
    net = torch.nn.Sequential(*layers).double()
    off = 0
    with torch.no_grad():
        for mod in net:
            if isinstance(mod, torch.nn.Linear):
                o, i = mod.weight.shape
                mod.weight.copy_(torch.tensor(flat[off:off + o * i].reshape(o, i), dtype=torch.float64))
                off += o * i
                mod.bias.copy_(torch.tensor(flat[off:off + o], dtype=torch.float64))
                off += o
    assert off == flat.size
    return net


@pytest.mark.parametrize("shape", [(15, 32, 2), (15, 256, 4), (15, 64, 8)])
def test_forward_matches_torch_sequential(shape):
    spec = svgen.MLPSpec(*shape)
    flat = svgen.mlp_init(spec, 3).astype(np.float64)
    X = np.random.default_rng(0).uniform(-2, 2, (300, shape[0]))
    y, _ = om.forward(flat, *shape, X)
    ref = torch_net(flat, *shape)(torch.tensor(X)).detach().numpy()[:, 0]
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-13)


def test_forward_special_cases():
    spec = svgen.MLPSpec(15, 16, 3)
    flat = np.zeros(spec.n_params)
    flat[-1] = 0.25                       # output bias only
    X = np.random.default_rng(1).normal(size=(7, 15))
    y, _ = om.forward(flat, 15, 16, 3, X)
    np.testing.assert_array_equal(y, 0.25)
    # all-zero hidden weights: every hidden unit is softplus(0) = ln 2; output = ln2 * sum(w_out) + b
    flat2 = np.zeros(spec.n_params)
    flat2[-17:-1] = 1.0
    y2, _ = om.forward(flat2, 15, 16, 3, X)
    np.testing.assert_allclose(y2, 16 * math.log(2.0), rtol=1e-15)
    assert om.softplus(np.array([0.0]))[0] == math.log(2.0)
    z = np.array([-800.0, -30.0, 30.0, 800.0])          # no overflow in the stable form
    np.testing.assert_allclose(om.softplus(z), [0.0, math.exp(-30.0), 30.0, 800.0], rtol=1e-12, atol=1e-300)


def _batch(seed, B=64, sigma=0.1):
    g = np.random.default_rng(seed)
    X = g.uniform(-1.5, 1.5, (B, 15))
    t = g.uniform(-0.15, 0.3, B)
    return X, t


def test_gradient_matches_autograd():
    shape = (15, 32, 3)
    spec = svgen.MLPSpec(*shape)
    flat = svgen.mlp_init(spec, 4).astype(np.float64)
    X, t = _batch(5)
    sigma = 0.1
    loss, g = om.loss_and_grad(flat, *shape, X, t, sigma)
    net = torch_net(flat, *shape)
    pred = net(torch.tensor(X))[:, 0]
    tt = torch.tensor(t)
    L = torch.mean(torch.abs(pred - torch.clamp(tt, -sigma, sigma)))
    L.backward()
    ref = torch.cat([torch.cat([m.weight.grad.reshape(-1), m.bias.grad]) for m in net
                     if isinstance(m, torch.nn.Linear)]).numpy()
    assert loss == pytest.approx(L.item(), rel=1e-14)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_gradient_matches_central_differences():
    """Width-32 network, central differences h = 1e-6 in FP64.  Targets and outputs
    are kept away from the kinks of |.| and clamp so the loss is smooth at theta."""
    shape = (15, 32, 2)
    spec = svgen.MLPSpec(*shape)
    flat = svgen.mlp_init(spec, 6).astype(np.float64)
    X, _ = _batch(7, B=48)
    y, _ = om.forward(flat, *shape, X)
    sigma = 10.0                                     # no clamping active
    t = y + np.where(np.arange(48) % 2 == 0, 0.05, -0.05)   # residuals far from 0
    _, g = om.loss_and_grad(flat, *shape, X, t, sigma)
    rng = np.random.default_rng(8)
    idx = rng.choice(flat.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp = om.clamped_l1(om.forward(flat + e, *shape, X)[0], t, sigma)
        lm = om.clamped_l1(om.forward(flat - e, *shape, X)[0], t, sigma)
        fd = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_decisions_default_to_own_prediction():
    shape = (15, 32, 2)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 16).astype(np.float64)
    X, t = _batch(17, B=32)
    y, _ = om.forward(flat, *shape, X)
    l1, g1 = om.loss_and_grad(flat, *shape, X, t, 0.1)
    l2, g2 = om.loss_and_grad(flat, *shape, X, t, 0.1, decide=y)
    assert l1 == l2
    np.testing.assert_array_equal(g1, g2)
    # flipping every decision flips the gradient
    _, g3 = om.loss_and_grad(flat, *shape, X, t, 10.0, decide=2 * t - y)
    _, g4 = om.loss_and_grad(flat, *shape, X, t, 10.0)
    np.testing.assert_allclose(g3, -g4, rtol=1e-12, atol=1e-15)


def test_clamp_acts_on_targets_only():
    """Targets beyond sigma count as sigma; predictions are never clamped, so a
    prediction beyond sigma is still pulled back (its gradient is the full sign)."""
    shape = (15, 16, 2)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 9).astype(np.float64)
    X, _ = _batch(10, B=16)
    y, _ = om.forward(flat, *shape, X)
    sigma = 0.05
    far = np.full(16, 3.0)
    l_far, g_far = om.loss_and_grad(flat, *shape, X, far, sigma)
    l_sig, g_sig = om.loss_and_grad(flat, *shape, X, np.full(16, sigma), sigma)
    assert l_far == l_sig == pytest.approx(np.mean(np.abs(y - sigma)), rel=1e-14)
    np.testing.assert_array_equal(g_far, g_sig)
    assert np.linalg.norm(g_far) > 0
    # d loss / d b_out = mean sign(y - clamp(t)) over every sample, also those with |y| > sigma
    _, g_lo = om.loss_and_grad(flat, *shape, X, np.full(16, -3.0), 0.01)
    assert np.any(np.abs(y) > 0.01)
    assert g_lo[-1] == pytest.approx(np.mean(np.sign(y + 0.01)), abs=1e-15)


def test_both_sides_clamp_matches_autograd():
    """DeepSDF's form, |clamp(y) - clamp(t)|, against torch autograd through torch.clamp
    on both sides (predictions spread beyond sigma so that some have no gradient)."""
    shape = (15, 32, 3)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 4).astype(np.float64)
    flat[-1] = 0.0
    flat[-33:-1] *= 8.0
    X, t = _batch(25, B=96)
    sigma = 0.1
    flat[-1] = -np.median(om.forward(flat, *shape, X)[0])   # centred: part of the batch beyond sigma
    y, _ = om.forward(flat, *shape, X)
    assert 10 < np.sum(np.abs(y) >= sigma) < 86
    loss, g = om.loss_and_grad(flat, *shape, X, t, sigma, clamp_pred=True)
    net = torch_net(flat, *shape)
    pred = net(torch.tensor(X))[:, 0]
    L = torch.mean(torch.abs(torch.clamp(pred, -sigma, sigma) - torch.clamp(torch.tensor(t), -sigma, sigma)))
    L.backward()
    ref = torch.cat([torch.cat([m.weight.grad.reshape(-1), m.bias.grad]) for m in net
                     if isinstance(m, torch.nn.Linear)]).numpy()
    assert loss == pytest.approx(L.item(), rel=1e-14)
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-14)


def test_both_sides_clamp_dead_zone():
    """Every prediction beyond sigma: the loss is the clamped gap and the gradient is
    zero; the target-only form still has one."""
    shape = (15, 16, 2)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 9).astype(np.float64)
    flat[-1] = 5.0                                   # b_out: every prediction far above sigma
    X, _ = _batch(10, B=16)
    y, _ = om.forward(flat, *shape, X)
    assert np.all(y > 1.0)
    t = np.linspace(-0.2, 0.2, 16)
    l2, g2 = om.loss_and_grad(flat, *shape, X, t, 0.1, clamp_pred=True)
    assert l2 == pytest.approx(np.mean(0.1 - np.clip(t, -0.1, 0.1)), rel=1e-14)
    assert not np.any(g2)
    _, g1 = om.loss_and_grad(flat, *shape, X, t, 0.1)
    assert g1[-1] == pytest.approx(1.0, abs=1e-15)


def test_adam_matches_torch():
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) * 10 ** rng.uniform(-3, 1) for _ in range(25)]
    opt = om.Adam(p0)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    topt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        opt.step(g)
        tp.grad = torch.tensor(g)
        topt.step()
        np.testing.assert_allclose(opt.p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_screened_verdict_special_cases():
    rng = np.random.default_rng(12)
    delta = rng.uniform(-0.05, 0.2, (40, 30))
    dhat = delta + rng.normal(0, 0.05, delta.shape)
    exact = (delta.min(axis=1) <= 0.01).astype(np.uint8)
    v_inf, nf = om.screened_verdicts(dhat, delta, 0.01, np.inf, certified=False)
    np.testing.assert_array_equal(v_inf, exact)          # every point falls back
    assert np.all(nf == 30)
    v_c, _ = om.screened_verdicts(dhat, delta, 0.01, 0.03, certified=True)
    np.testing.assert_array_equal(v_c, exact)            # certified mode is exact by construction
    v_t, _ = om.screened_verdicts(dhat, delta, 0.01, -1.0, certified=False)
    np.testing.assert_array_equal(v_t, 0)                # nothing sent: trust mode says free


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(13)
    x = np.concatenate([rng.normal(size=5000) * 10 ** rng.uniform(-6, 3, 5000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 3.4e38]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.round_bf16(x), ref)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert om.round_bf16(np.float32(1.0 + 2 ** -8)) == 1.0


@pytest.mark.parametrize("n_hidden", [1, 2, 4])
def test_bf16_emulation_matches_torch_rounding(n_hidden):
    """The BF16-rounding forward pass against the same rounding points written with
    torch's bfloat16 casts and FP64 torch modules."""
    shape = (15, 64, n_hidden)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 14).astype(np.float64)
    X = np.random.default_rng(15).uniform(-1, 1, (40, 15))
    net = torch_net(flat, *shape)
    lin = [m for m in net if isinstance(m, torch.nn.Linear)]
    bf = lambda t: t.float().to(torch.bfloat16).to(torch.float64)
    h = torch.tensor(X)
    for l, mod in enumerate(lin[:-1]):
        W = mod.weight if l == 0 else bf(mod.weight)
        h = torch.nn.functional.softplus(h @ W.T + mod.bias, beta=1.0, threshold=1e9)
        if l + 1 < n_hidden or n_hidden == 1:
            h = bf(h)
    ref = (h @ lin[-1].weight.T + lin[-1].bias)[:, 0].detach().numpy()
    np.testing.assert_allclose(om.forward_bf16(flat, *shape, X), ref, rtol=1e-12, atol=1e-14)
    y64, _ = om.forward(flat, *shape, X)
    assert np.max(np.abs(om.forward_bf16(flat, *shape, X) - y64)) < 0.05   # rounding changes values a little
