"""FP64 oracle for the paper's residual swept-volume network (Sec. IV-A, Fig. 1).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

The network, read from Sec. IV-A and Fig. 1:

    h_0 = W_0 x_in + b_0                              (initial linear layer, no activation)
    z_b = W_b [h_{b-1}; x_in] + c_b                    (block linear layer; the network
                                                        input is concatenated to the block
                                                        input: the jump connection)
    h_b = h_{b-1} + BN_b(relu(z_b)),   b = 1..L         (ReLU, then BatchNorm, then the skip)
    delta_hat = w_out . h_L + b_out                     (final linear layer)

with x_in = [x; q0; q1] and the BatchNorm in its inference form with running
statistics, BN(a) = gamma (a - mu) / sqrt(var + eps) + beta.

Reading: the paper says each block's linear layer keeps the block dimension and also
that the network input is concatenated to each block output.  Both hold if the
concatenated vector [h; x_in] feeds the next block's linear layer (n_dim + in_dim ->
n_dim) while the skip adds h alone; that is the reading taken here.

Parameters arrive as one flat FP32 vector: W_0 [W][in], b_0 [W], then per block
Wh [W][W], Wx [W][in] (the columns of W_b acting on h and on x_in), c, gamma, beta,
mu, var (each [W]), then w_out [W], b_out [1]; converted exactly to float64.

A matrix product (numpy ``@``) is used as a library primitive; nothing else is fused
or reordered.
"""
from __future__ import annotations

import numpy as np

from .mlp import round_bf16


def n_params(in_dim: int, width: int, n_blocks: int) -> int:
    W = width
    return W * in_dim + W + n_blocks * (W * W + W * in_dim + 5 * W) + W + 1


def unpack(flat, in_dim: int, width: int, n_blocks: int) -> dict:
    """Flat vector -> {'W0','b0','blocks': [dict(Wh, Wx, c, gamma, beta, mu, var)], 'w_out', 'b_out'}."""
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != n_params(in_dim, width, n_blocks):
        raise ValueError(f"parameter vector has {flat.size} entries, expected {n_params(in_dim, width, n_blocks)}")
    W = width
    off = 0

    def take(n, shape=None):
        nonlocal off
        a = flat[off:off + n]
        off += n
        return a.reshape(shape) if shape else a

    net = {"W0": take(W * in_dim, (W, in_dim)), "b0": take(W), "blocks": []}
    for _ in range(n_blocks):
        net["blocks"].append({"Wh": take(W * W, (W, W)), "Wx": take(W * in_dim, (W, in_dim)), "c": take(W),
                              "gamma": take(W), "beta": take(W), "mu": take(W), "var": take(W)})
    net["w_out"] = take(W)
    net["b_out"] = take(1)[0]
    return net


def pack(net: dict) -> np.ndarray:
    parts = [net["W0"].ravel(), net["b0"]]
    for b in net["blocks"]:
        parts += [b["Wh"].ravel(), b["Wx"].ravel(), b["c"], b["gamma"], b["beta"], b["mu"], b["var"]]
    parts += [net["w_out"], np.array([net["b_out"]])]
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


def batchnorm(a, blk, eps):
    """Inference BatchNorm with running statistics (the layer's eval form)."""
    return blk["gamma"] * (a - blk["mu"]) / np.sqrt(blk["var"] + eps) + blk["beta"]


def forward(flat, in_dim, width, n_blocks, X, bn_eps):
    """delta_hat [B] for input rows X [B][in_dim]."""
    net = unpack(flat, in_dim, width, n_blocks)
    X = np.asarray(X, np.float64)
    h = X @ net["W0"].T + net["b0"]
    for blk in net["blocks"]:
        z = np.concatenate([h, X], axis=1) @ np.concatenate([blk["Wh"], blk["Wx"]], axis=1).T + blk["c"]
        h = h + batchnorm(np.maximum(z, 0.0), blk, bn_eps)
    return h @ net["w_out"] + net["b_out"]


def forward_bf16(flat, in_dim, width, n_blocks, X, bn_eps):
    """Debugging aid: the network with the BF16 path's rounding points, otherwise FP64.

    - h_0 from FP32-exact weights and unrounded inputs, rounded to BF16;
    - each block: the weights Wh and Wx rounded to BF16; h (BF16) and the input as the
      sum of its BF16 rounding and the BF16 rounding of the remainder; the block's result
      rounded to BF16 except after the last block, whose result feeds the output layer
      unrounded.
    """
    net = unpack(flat, in_dim, width, n_blocks)
    X = np.asarray(X, np.float32).astype(np.float64)
    x_hi = round_bf16(X)
    x_lo = round_bf16((X.astype(np.float32) - x_hi.astype(np.float32)))
    Xs = x_hi + x_lo
    h = round_bf16(X @ net["W0"].T + net["b0"])
    for i, blk in enumerate(net["blocks"]):
        z = h @ round_bf16(blk["Wh"]).T + Xs @ round_bf16(blk["Wx"]).T + blk["c"]
        y = h + batchnorm(np.maximum(z, 0.0), blk, bn_eps)
        h = y if i + 1 == n_blocks else round_bf16(y)
    return h @ net["w_out"] + net["b_out"]


# ---------------------------------------------------------------- training
# BatchNorm in its training form (Sec. IV-A names BatchNorm layers; Sec. V trains with
# PyTorch): each block normalises with the statistics of the batch,
#     mu_B = mean over the batch of a,  v_B = mean over the batch of (a - mu_B)^2,
#     BN(a) = gamma (a - mu_B) / sqrt(v_B + eps) + beta,
# and afterwards moves its running statistics towards them with momentum m:
#     mu <- (1 - m) mu + m mu_B,  var <- (1 - m) var + m v_B B / (B - 1)
# (PyTorch's rule: the running variance takes the unbiased batch variance).


def forward_train(flat, in_dim, width, n_blocks, X, bn_eps):
    """delta_hat [B] with batch-statistic BatchNorm, and what the backward pass needs."""
    net = unpack(flat, in_dim, width, n_blocks)
    X = np.asarray(X, np.float64)
    h = X @ net["W0"].T + net["b0"]
    cache = {"X": X, "h": [h], "a": [], "n": [], "mu": [], "v": []}
    for blk in net["blocks"]:
        z = np.concatenate([h, X], axis=1) @ np.concatenate([blk["Wh"], blk["Wx"]], axis=1).T + blk["c"]
        a = np.maximum(z, 0.0)
        mu = a.mean(axis=0)
        v = ((a - mu) ** 2).mean(axis=0)
        n = (a - mu) / np.sqrt(v + bn_eps)
        h = h + blk["gamma"] * n + blk["beta"]
        for k, val in (("a", a), ("n", n), ("mu", mu), ("v", v), ("h", h)):
            cache[k].append(val)
    y = h @ net["w_out"] + net["b_out"]
    return y, cache


def loss_and_grad_train(flat, in_dim, width, n_blocks, X, target, sigma, bn_eps, decide=None):
    """Target-clamped L1 loss (oracle.mlp.clamped_l1) of the batch-statistic forward pass
    and its gradient w.r.t. the flat vector, by backpropagation.  The running-statistic
    entries (mu, var) get zero gradient: they are not trained but averaged
    (running_update).  `decide`: the predictions the loss's sign decisions are taken on.

    BatchNorm backward, with n = (a - mu_B) / s, s = sqrt(v_B + eps), g = dL/dh_b:
      dgamma = sum g n,  dbeta = sum g,
      da = gamma / s (g - mean(g) - n mean(g n))      (means over the batch);
    ReLU passes da where z > 0 (a > 0); the skip passes g to h_{b-1} unchanged.
    """
    net = unpack(flat, in_dim, width, n_blocks)
    y, c = forward_train(flat, in_dim, width, n_blocks, X, bn_eps)
    B = y.shape[0]
    tc = np.clip(np.asarray(target, np.float64), -sigma, sigma)
    loss = float(np.mean(np.abs(y - tc)))
    yd = y if decide is None else np.asarray(decide, np.float64)
    dy = np.sign(yd - tc) / B
    grads = {"w_out": c["h"][-1].T @ dy, "b_out": dy.sum(), "blocks": [None] * n_blocks}
    g = dy[:, None] * net["w_out"][None, :]
    for i in range(n_blocks - 1, -1, -1):
        blk = net["blocks"][i]
        n, a = c["n"][i], c["a"][i]
        s = np.sqrt(c["v"][i] + bn_eps)
        dgamma, dbeta = (g * n).sum(axis=0), g.sum(axis=0)
        da = blk["gamma"] / s * (g - g.mean(axis=0) - n * (g * n).mean(axis=0))
        dz = da * (a > 0)
        hp = c["h"][i]
        grads["blocks"][i] = {"Wh": dz.T @ hp, "Wx": dz.T @ c["X"], "c": dz.sum(axis=0), "gamma": dgamma,
                              "beta": dbeta, "mu": np.zeros(width), "var": np.zeros(width)}
        g = g + dz @ blk["Wh"]
    grads["W0"] = g.T @ c["X"]
    grads["b0"] = g.sum(axis=0)
    return loss, pack(grads)


def running_update(flat, in_dim, width, n_blocks, X, bn_eps, momentum=0.1):
    """The flat vector with every block's running statistics moved towards this batch's
    (after a training forward pass on X)."""
    net = unpack(flat, in_dim, width, n_blocks)
    _, c = forward_train(flat, in_dim, width, n_blocks, X, bn_eps)
    B = np.asarray(X).shape[0]
    for blk, mu, v in zip(net["blocks"], c["mu"], c["v"]):
        blk["mu"] = (1 - momentum) * blk["mu"] + momentum * mu
        blk["var"] = (1 - momentum) * blk["var"] + momentum * v * B / (B - 1)
    return pack(net)


def loss_and_grad_train_bf16(flat, in_dim, width, n_blocks, X, target, sigma, bn_eps, rounding=True):
    """Debugging aid and error gauge: loss_and_grad_train with the BF16 training path's
    rounding points, otherwise FP64 (rounding=False gives loss_and_grad_train exactly).

    Rounded to BF16 (round to nearest even): the block weights Wh_b, Wx_b; the network
    input as the sum of its BF16 rounding and the BF16 rounding of the remainder; h_0 and
    every block input h_b (b < L; h_L stays unrounded); a_b = relu(z_b) (the batch
    statistics are taken on the rounded values); dz_b; g_0 = dL/dh_0 (W_0 and b_0 sums).
    The BatchNorm backward amplifies the forward roundings (its gradient is a small
    remainder of large terms), so the distance of this emulation from the FP64 gradient
    measures what the BF16 path can reach.
    """
    R = round_bf16 if rounding else (lambda v: np.asarray(v, np.float64))
    net = unpack(flat, in_dim, width, n_blocks)
    X = np.asarray(X, np.float64)
    if rounding:
        x_hi = round_bf16(X)
        Xs = x_hi + round_bf16(X.astype(np.float32) - x_hi.astype(np.float32))
    else:
        Xs = X
    h = R(X @ net["W0"].T + net["b0"])
    hs, As, ns, invs = [h], [], [], []
    for i, blk in enumerate(net["blocks"]):
        z = h @ R(blk["Wh"]).T + Xs @ R(blk["Wx"]).T + blk["c"]
        a = R(np.maximum(z, 0.0))
        mu = a.mean(axis=0)
        inv = 1.0 / np.sqrt(((a - mu) ** 2).mean(axis=0) + bn_eps)
        n = (a - mu) * inv
        hn = h + blk["gamma"] * n + blk["beta"]
        h = hn if i + 1 == n_blocks else R(hn)
        hs.append(h)
        As.append(a)
        ns.append(n)
        invs.append(inv)
    y = h @ net["w_out"] + net["b_out"]
    B = y.shape[0]
    tc = np.clip(np.asarray(target, np.float64), -sigma, sigma)
    loss = float(np.mean(np.abs(y - tc)))
    dy = np.sign(y - tc) / B
    grads = {"w_out": h.T @ dy, "b_out": dy.sum(), "blocks": [None] * n_blocks}
    g = dy[:, None] * net["w_out"][None, :]
    for i in range(n_blocks - 1, -1, -1):
        blk = net["blocks"][i]
        n = ns[i]
        dgamma, dbeta = (g * n).sum(axis=0), g.sum(axis=0)
        dz = R(blk["gamma"] * invs[i] * (g - g.mean(axis=0) - n * (g * n).mean(axis=0)) * (As[i] > 0))
        grads["blocks"][i] = {"Wh": dz.T @ hs[i], "Wx": dz.T @ X, "c": dz.sum(axis=0), "gamma": dgamma,
                              "beta": dbeta, "mu": np.zeros(width), "var": np.zeros(width)}
        g = g + dz @ R(blk["Wh"])
    g0 = R(g)
    grads["W0"] = g0.T @ X
    grads["b0"] = g0.sum(axis=0)
    return loss, pack(grads)
