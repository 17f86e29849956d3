"""Pins of the BF16 error bars (oracle/bf16_error.py) and of the BF16 emulations, CPU only.

- The bar's first-order sum over rounding sites against a direct simulation: every
  rounding site of the network perturbed by an independent uniform factor in
  [-1, 1] times its magnitude, the forward pass re-run, and the variance of the
  output error over many draws compared with the predicted one (sum_s a_s^2 / 3 for
  uniform factors).  A site the adjoint sum left out, a wrong sensitivity or a
  wrong magnitude moves that ratio away from 1.
- The deterministic BF16 emulations (the kernels' rounding points with round to
  nearest even) stay within the bar against the FP64 networks.
- Plausible misplacements of a rounding point, planted in copies of the emulations
  here, move the median row by more than 0.5% of the bar: the GPU tests' median
  criterion (GPU vs emulation) would reject a kernel that made them.
- Hand-sized cases whose BF16 codes are worked out in the comments: one where the
  documented rounding placement of the softplus network gives a value that each
  alternative placement misses, and one where the residual network's low-part
  input columns change the output by 0.06.
- The residual emulation against a model built from torch layers with torch's
  bfloat16 casts at the documented points.
"""
import math

import numpy as np
import pytest
import torch

import svgen
from oracle import bf16_error as be
from oracle import mlp as om
from oracle import residual as ores

U, U32 = be.U_BF16, be.U_FP32
IN = 15
BN_EPS = 1e-5


def _rows(n, seed):
    g = np.random.default_rng(seed)
    return np.concatenate([g.uniform(-0.6, 0.6, (n, 3)), g.uniform(-3.0, 3.0, (n, IN - 3))], axis=1) \
        .astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------- direct simulations
def perturbed_mlp(flat, in_dim, width, L, X, rng):
    """The softplus network with every rounding site of its BF16 path replaced by an
    independent uniform perturbation of the site's magnitude."""
    uni = lambda shape: rng.uniform(-1.0, 1.0, shape)
    layers = om.unpack(flat, in_dim, width, L)
    h = X
    for l, (W, b) in enumerate(layers[:-1], start=1):
        Wp = W * (1 + U * uni(W.shape)) if l >= 2 else W
        z = h @ Wp.T + b
        z = z + be.gamma(W.shape[1] + 1) * (np.abs(h) @ np.abs(W).T + np.abs(b)) * uni(z.shape)
        hl = om.softplus(z) + 2.0 ** -20 * (1 + np.abs(z)) * uni(z.shape)
        if l < L or L == 1:
            hl = hl * (1 + U * uni(hl.shape))
        h = hl
    W, b = layers[-1]
    return (h @ W.T + b)[:, 0]


def perturbed_residual(flat, in_dim, width, nb, X, eps, rng):
    uni = lambda shape: rng.uniform(-1.0, 1.0, shape)
    net = ores.unpack(flat, in_dim, width, nb)
    h = X @ net["W0"].T + net["b0"]
    h = h + be.gamma(in_dim + 1) * (np.abs(X) @ np.abs(net["W0"]).T + np.abs(net["b0"])) * uni(h.shape)
    h = h * (1 + U * uni(h.shape))
    Xs = X * (1 + U * U * (1 + U) * uni(X.shape))          # one split error per input, every block
    K = width + 2 * in_dim
    for i, blk in enumerate(net["blocks"]):
        Wh = blk["Wh"] * (1 + U * uni(blk["Wh"].shape))
        Wx = blk["Wx"] * (1 + U * uni(blk["Wx"].shape))
        z = h @ Wh.T + Xs @ Wx.T + blk["c"]
        z = z + be.gamma(K + 1) * (np.abs(h) @ np.abs(blk["Wh"]).T + np.abs(X) @ np.abs(blk["Wx"]).T * (1 + 2 * U)
                                   + np.abs(blk["c"])) * uni(z.shape)
        scale = blk["gamma"] / np.sqrt(blk["var"] + eps)
        a = np.maximum(z, 0.0)
        hn = h + scale * (a - blk["mu"]) + blk["beta"]
        hn = hn + 8 * U32 * (np.abs(h) + np.abs(scale * a) + np.abs(blk["beta"]) + np.abs(scale * blk["mu"])) \
            * uni(hn.shape)
        if i + 1 < nb:
            hn = hn * (1 + U * uni(hn.shape))
        h = hn
    return h @ net["w_out"] + net["b_out"]


@pytest.mark.parametrize("shape", [(IN, 64, 3), (IN, 128, 1), (IN, 96, 5)])
def test_mlp_site_sum_matches_simulation(shape):
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 7).astype(np.float64)
    X = _rows(48, 1)
    y, S2, _ = be.mlp_sites(flat, *shape, X)
    np.testing.assert_allclose(y, om.forward(flat, *shape, X)[0], rtol=1e-13, atol=1e-13)
    rng = np.random.default_rng(2)
    d = np.stack([perturbed_mlp(flat, *shape, X, rng) - y for _ in range(400)])
    ratio = d.var(axis=0).mean() / (S2.mean() / 3.0)
    print(f"mlp {shape}: simulated / predicted variance {ratio:.3f}")
    assert 0.85 <= ratio <= 1.15


@pytest.mark.parametrize("shape", [(IN, 64, 3), (IN, 128, 4)])
def test_residual_site_sum_matches_simulation(shape):
    flat = svgen.res_init(svgen.ResSpec(*shape), 7).astype(np.float64)
    X = _rows(48, 3)
    y, S2, _ = be.residual_sites(flat, *shape, X, BN_EPS)
    np.testing.assert_allclose(y, ores.forward(flat, *shape, X, BN_EPS), rtol=1e-12, atol=1e-12)
    rng = np.random.default_rng(4)
    d = np.stack([perturbed_residual(flat, *shape, X, BN_EPS, rng) - y for _ in range(400)])
    ratio = d.var(axis=0).mean() / (S2.mean() / 3.0)
    print(f"residual {shape}: simulated / predicted variance {ratio:.3f}")
    # the ReLU margin counts a few near-kink features with derivative 1: slightly above 1 / ratio
    assert 0.85 <= ratio <= 1.15


def test_site_sum_of_a_single_product_by_hand():
    """in_dim 1, width 1, two layers: every site written out."""
    w1, b1, w2, b2, wo, bo = 0.75, -0.25, 1.5, 0.125, 2.0, 0.5
    flat = np.array([w1, b1, w2, b2, wo, bo])
    x = 0.5
    z1 = w1 * x + b1
    h1 = om.softplus(np.array([z1]))[0]
    z2 = w2 * h1 + b2
    h2 = om.softplus(np.array([z2]))[0]
    s1, s2 = om.sigmoid(np.array([z1]))[0], om.sigmoid(np.array([z2]))[0]
    gh2 = wo
    gz2 = gh2 * s2
    gh1 = gz2 * w2
    gz1 = gh1 * s1
    S2 = ((gh2 * 2 ** -20 * (1 + abs(z2))) ** 2                       # softplus of layer 2
          + (gz2 * be.gamma(2) * (abs(w2 * h1) + abs(b2))) ** 2        # FP32 sum of layer 2
          + (gz2 * U * abs(w2 * h1)) ** 2                              # BF16 weight of layer 2
          + (gh1 * 2 ** -20 * (1 + abs(z1))) ** 2                      # softplus of layer 1
          + (gh1 * U * h1) ** 2                                        # h1 rounded to BF16
          + (gz1 * be.gamma(2) * (abs(w1 * x) + abs(b1))) ** 2)        # FP32 sum of layer 1
    y, got, D = be.mlp_sites(flat, 1, 1, 2, np.array([[x]]))
    assert y[0] == pytest.approx(wo * h2 + bo, rel=1e-15)
    assert got[0] == pytest.approx(S2, rel=1e-12)
    assert D[0] == pytest.approx(be.gamma(2) * (abs(wo * h2) + abs(bo)), rel=1e-15)


# ---------------------------------------------------------------- emulations within the bar
@pytest.mark.parametrize("shape,n", [((IN, 512, 8), 160), ((IN, 128, 1), 300), ((IN, 256, 4), 300)])
def test_mlp_emulation_within_bar(shape, n):
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 11)
    X = _rows(n, 5)
    y64, bar = be.mlp_bar(flat, *shape, X)
    err = np.abs(om.forward_bf16(flat, *shape, X) - y64)
    print(f"mlp {shape}: emulation error / bar max {np.max(err / bar):.3f}, median bar {np.median(bar):.2e}")
    assert np.all(err <= bar)


@pytest.mark.parametrize("shape,n", [((IN, 512, 5), 120), ((IN, 1024, 11), 60), ((IN, 128, 2), 300)])
def test_residual_emulation_within_bar(shape, n):
    flat = svgen.res_init(svgen.ResSpec(*shape), 13)
    X = _rows(n, 6)
    y64, bar = be.residual_bar(flat, *shape, X, BN_EPS)
    err = np.abs(ores.forward_bf16(flat, *shape, X, BN_EPS) - y64)
    print(f"residual {shape}: emulation error / bar max {np.max(err / bar):.3f}, median bar {np.median(bar):.2e}")
    assert np.all(err <= bar)


# ---------------------------------------------------------------- planted misplacements
def mlp_misplaced(flat, in_dim, width, L, X, kind):
    """Copies of the softplus emulation with one rounding point moved."""
    layers = om.unpack(flat, in_dim, width, L)
    h = np.asarray(X, np.float64)
    for l, (W, b) in enumerate(layers[:-1]):
        if l == 0:
            round_w = kind == "first_weights_rounded"
        else:
            round_w = not (l == 1 and kind == "second_weights_kept")
        h = om.softplus(h @ (om.round_bf16(W) if round_w else W).T + b)
        if l + 1 < L or L == 1 or kind == "last_activation_rounded":
            h = om.round_bf16(h)
    W, b = layers[-1]
    return (h @ W.T + b)[:, 0]


def residual_misplaced(flat, in_dim, width, nb, X, eps, kind):
    net = ores.unpack(flat, in_dim, width, nb)
    X = np.asarray(X, np.float32).astype(np.float64)
    hi = om.round_bf16(X)
    lo = om.round_bf16(X.astype(np.float32) - hi.astype(np.float32))
    Xs = hi if kind == "low_part_dropped" else hi + lo
    h = X @ net["W0"].T + net["b0"]
    if kind != "h0_kept":
        h = om.round_bf16(h)
    for i, blk in enumerate(net["blocks"]):
        z = h @ om.round_bf16(blk["Wh"]).T + Xs @ om.round_bf16(blk["Wx"]).T + blk["c"]
        y = h + ores.batchnorm(np.maximum(z, 0.0), blk, eps)
        h = y if (i + 1 == nb and kind != "last_rounded") else om.round_bf16(y)
    return h @ net["w_out"] + net["b_out"]


def test_misplaced_rounding_points_fail_the_median_criterion():
    """Each misplacement moves the median row by more than 0.5% of the bar, the
    GPU-vs-emulation criterion; the emulation itself moves it by nothing."""
    X = _rows(200, 8)
    shape = (IN, 512, 8)
    flat = svgen.mlp_init(svgen.MLPSpec(*shape), 17)
    _, bar = be.mlp_bar(flat, *shape, X)
    em = om.forward_bf16(flat, *shape, X)
    assert np.median(np.abs(mlp_misplaced(flat, *shape, X, "none") - em) / bar) == 0.0
    for kind in ("first_weights_rounded", "second_weights_kept", "last_activation_rounded"):
        med = np.median(np.abs(mlp_misplaced(flat, *shape, X, kind) - em) / bar)
        print(f"mlp {kind}: median / bar {med:.4f}")
        assert med > 0.005, kind
    rshape = (IN, 512, 5)
    rflat = svgen.res_init(svgen.ResSpec(*rshape), 19)
    _, rbar = be.residual_bar(rflat, *rshape, X, BN_EPS)
    rem = ores.forward_bf16(rflat, *rshape, X, BN_EPS)
    assert np.median(np.abs(residual_misplaced(rflat, *rshape, X, BN_EPS, "none") - rem) / rbar) == 0.0
    for kind in ("low_part_dropped", "h0_kept", "last_rounded"):
        med = np.median(np.abs(residual_misplaced(rflat, *rshape, X, BN_EPS, kind) - rem) / rbar)
        print(f"residual {kind}: median / bar {med:.4f}")
        assert med > 0.005, kind


# ---------------------------------------------------------------- hand-sized cases
def _sp(z):
    return max(z, 0.0) + math.log1p(math.exp(-abs(z)))


def test_mlp_rounding_placement_by_hand():
    """in_dim 1, width 1, L = 2; x = 1; W1 = fp32(0.3), b1 = fp32(0.2005); W2 = fp32(0.3),
    b2 = 0; w_out = 1, b_out = 0.

    Documented placement: layer 1 in FP32 with unrounded weights, its activation rounded
    to BF16, layer 2's weight rounded, the last hidden activation unrounded.
      z1 = 0.50050000846...; h1 = softplus(z1) = 0.97438...; in [0.5, 1) BF16 values are
      k / 256, and 0.97438 * 256 = 249.44, so h1 -> 249 / 256.
      W2: in [0.25, 0.5) BF16 values are k / 512; 0.3 * 512 = 153.6 -> 154 / 512.
      y = softplus(249/256 * 154/512).
    Alternatives and why each differs:
      h1 unrounded:            y = softplus(softplus(z1) * 154/512);
      W1 rounded (154/512):    z1 = 0.50128..., h1 * 256 = 249.57 -> 250 / 256;
      W2 unrounded:            y = softplus(249/256 * fp32(0.3));
      last activation rounded: softplus(...) = 0.85009, and 0.85009 * 256 = 217.62 -> y = 218 / 256.
    """
    w, b1 = float(np.float32(0.3)), float(np.float32(0.2005))
    flat = np.array([w, b1, w, 0.0, 1.0, 0.0])
    documented = _sp(249 / 256 * 154 / 512)
    got = om.forward_bf16(flat, 1, 1, 2, np.array([[1.0]]))[0]
    assert got == pytest.approx(documented, abs=1e-15)
    alternatives = {"h1 unrounded": _sp(_sp(w + b1) * 154 / 512), "W1 rounded": _sp(250 / 256 * 154 / 512),
                    "W2 unrounded": _sp(249 / 256 * w), "last rounded": 218 / 256}
    for name, v in alternatives.items():
        assert abs(v - documented) > 2e-4, name
    X = np.array([[1.0]])
    for kind, name in (("first_weights_rounded", "W1 rounded"), ("second_weights_kept", "W2 unrounded"),
                       ("last_activation_rounded", "last rounded")):
        assert mlp_misplaced(flat, 1, 1, 2, X, kind)[0] == pytest.approx(alternatives[name], abs=1e-15)


def test_residual_low_part_by_hand():
    """in_dim 1, width 1, one block: W0 = 0, b0 = 0 (h0 = 0), Wh = 0, Wx = 64, c = 0,
    gamma = 1, beta = 0, mu = 0, var = 1 - 2^-10 with bn_eps = 2^-10 (scale exactly 1),
    w_out = 1, b_out = 0; so y = 64 (x_hi + x_lo) with x = fp32(0.6123456).
      x_hi: in [0.5, 1) BF16 values are k / 256; x * 256 = 156.76 -> 157 / 256.
      x - x_hi = -0.00093567... lies in [2^-11, 2^-10), where BF16 values are k / 2^18;
      -0.00093567 * 2^18 = -245.28 -> x_lo = -245 / 2^18.
      y = 64 (157/256 - 245/2^18) = 39.25 - 0.0598144531... = 39.1901855468...
    Without the low part the output would be 39.25, 0.06 away."""
    x = float(np.float32(0.6123456))
    net = {"W0": np.zeros((1, 1)), "b0": np.zeros(1),
           "blocks": [{"Wh": np.zeros((1, 1)), "Wx": np.array([[64.0]]), "c": np.zeros(1), "gamma": np.ones(1),
                       "beta": np.zeros(1), "mu": np.zeros(1), "var": np.array([1.0 - 2.0 ** -10])}],
           "w_out": np.ones(1), "b_out": 0.0}
    flat = ores.pack(net)
    expect = 64.0 * (157 / 256 - 245 / 2 ** 18)
    got = ores.forward_bf16(flat, 1, 1, 1, np.array([[x]]), 2.0 ** -10)[0]
    assert got == pytest.approx(expect, abs=1e-12)
    dropped = residual_misplaced(flat, 1, 1, 1, np.array([[x]]), 2.0 ** -10, "low_part_dropped")[0]
    assert dropped == pytest.approx(39.25, abs=1e-12)
    assert abs(dropped - got) > 0.05


class TorchResNetBF16(torch.nn.Module):
    """The residual network from torch layers, with bfloat16 casts where the BF16 path
    rounds: h0, block weights, the input as high part plus rounded remainder, block
    results except the last.  Arithmetic between the casts in FP64."""

    def __init__(self, flat, in_dim, width, n_blocks, bn_eps):
        super().__init__()
        net = ores.unpack(flat, in_dim, width, n_blocks)
        t = lambda a: torch.as_tensor(np.asarray(a, np.float64))
        self.first = torch.nn.Linear(in_dim, width).double()
        self.lin = torch.nn.ModuleList([torch.nn.Linear(width + in_dim, width).double() for _ in range(n_blocks)])
        self.bn = torch.nn.ModuleList([torch.nn.BatchNorm1d(width, eps=bn_eps).double() for _ in range(n_blocks)])
        self.last = torch.nn.Linear(width, 1).double()
        with torch.no_grad():
            self.first.weight.copy_(t(net["W0"]))
            self.first.bias.copy_(t(net["b0"]))
            for lin, bn, blk in zip(self.lin, self.bn, net["blocks"]):
                lin.weight.copy_(self.bf(t(np.concatenate([blk["Wh"], blk["Wx"]], axis=1))))
                lin.bias.copy_(t(blk["c"]))
                bn.weight.copy_(t(blk["gamma"]))
                bn.bias.copy_(t(blk["beta"]))
                bn.running_mean.copy_(t(blk["mu"]))
                bn.running_var.copy_(t(blk["var"]))
            self.last.weight.copy_(t(net["w_out"][None, :]))
            self.last.bias.copy_(t([net["b_out"]]))
        self.eval()

    @staticmethod
    def bf(v):
        return v.float().to(torch.bfloat16).to(torch.float64)

    def forward(self, x):
        x32 = x.float()
        hi = x32.to(torch.bfloat16)
        lo = (x32 - hi.float()).to(torch.bfloat16)
        xs = hi.double() + lo.double()
        h = self.bf(self.first(x))
        n = len(self.lin)
        for i, (lin, bn) in enumerate(zip(self.lin, self.bn)):
            h = h + bn(torch.relu(lin(torch.cat([h, xs], dim=1))))
            if i + 1 < n:
                h = self.bf(h)
        return self.last(h)[:, 0]


@pytest.mark.parametrize("width,n_blocks", [(32, 1), (64, 3), (128, 5)])
def test_residual_emulation_against_torch_bf16_layers(width, n_blocks):
    flat = svgen.res_init(svgen.ResSpec(IN, width, n_blocks), 30 + n_blocks)
    X = _rows(150, 31)
    ref = TorchResNetBF16(flat, IN, width, n_blocks, BN_EPS)(torch.as_tensor(X)).detach().numpy()
    got = ores.forward_bf16(flat, IN, width, n_blocks, X, BN_EPS)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    for kind in ("low_part_dropped", "h0_kept", "last_rounded"):
        assert np.max(np.abs(residual_misplaced(flat, IN, width, n_blocks, X, BN_EPS, kind) - ref)) > 1e-6, kind
