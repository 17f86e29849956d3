"""FP64 oracle for the swept-volume network f_theta(x, q0, q1) -> delta.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

The network is a plain fully connected MLP (Sec. IV-A describes a fully
connected network that maps the query point and the motion's start and goal
configurations to one signed distance; the hot path replaces the paper's
ReLU/BatchNorm residual blocks with softplus layers):

    h_0 = [x; q0; q1]                      (input order of Sec. I / Fig. 1)
    h_l = softplus(W_l h_{l-1} + b_l),  l = 1..L
    delta_hat = w_out . h_L + b_out        (no output activation)

softplus(z) = max(z, 0) + log1p(exp(-|z|)).  Parameters arrive as one flat FP32
vector, per layer W (row-major [out][in]) then b, and are converted exactly to
float64.  Training follows Sec. V (Adam with PyTorch's default constants,
lr = 1e-3, betas = (0.9, 0.999)); the loss is an L1 on distances clamped to
[-sigma, sigma], on the targets only or on both sides (the paper states no loss;
the clamp follows the DeepSDF work it cites for its jump connections).

A matrix product (numpy ``@``) is used as a library primitive; nothing else is
fused or reordered.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(in_dim: int, width: int, n_hidden: int):
    return [(width, in_dim)] + [(width, width)] * (n_hidden - 1) + [(1, width)]


def unpack(flat, in_dim: int, width: int, n_hidden: int):
    """Flat parameter vector -> list of (W [out][in], b [out]) in float64."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = [], 0
    for o, i in layer_shapes(in_dim, width, n_hidden):
        W = flat[off:off + o * i].reshape(o, i)
        off += o * i
        b = flat[off:off + o]
        off += o
        out.append((W, b))
    if off != flat.size:
        raise ValueError(f"parameter vector has {flat.size} entries, expected {off}")
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    """Derivative of softplus; written in the overflow-free split form."""
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def features(x, q0, q1):
    """Network input rows [x; q0; q1] from [B][3], [B][dof], [B][dof]."""
    return np.concatenate([np.asarray(x, np.float64), np.asarray(q0, np.float64),
                           np.asarray(q1, np.float64)], axis=1)


def forward(flat, in_dim, width, n_hidden, H0):
    """delta_hat [B] for input rows H0 [B][in_dim]; also returns the pre-activations."""
    layers = unpack(flat, in_dim, width, n_hidden)
    h = np.asarray(H0, np.float64)
    zs, hs = [], [h]
    for W, b in layers[:-1]:
        z = h @ W.T + b
        h = softplus(z)
        zs.append(z)
        hs.append(h)
    W, b = layers[-1]
    y = (h @ W.T + b)[:, 0]
    return y, (zs, hs)


def clamped_l1(pred, target, sigma, clamp_pred=False):
    """An L1 loss on distances clamped to s (the paper states no loss; the clamp follows
    the DeepSDF work it cites for its jump connections):

    clamp_pred False: L = mean |pred - clamp(target, -s, s)|, the target clamped only;
    clamp_pred True:  L = mean |clamp(pred, -s, s) - clamp(target, -s, s)|, DeepSDF's
                      form, under which a prediction outside [-s, s] has no gradient.
    """
    p = np.clip(pred, -sigma, sigma) if clamp_pred else np.asarray(pred)
    return float(np.mean(np.abs(p - np.clip(target, -sigma, sigma))))


def loss_and_grad(flat, in_dim, width, n_hidden, H0, target, sigma, decide=None, clamp_pred=False):
    """Clamped-L1 loss (see clamped_l1) and its gradient w.r.t. the flat parameter
    vector, by backpropagation.

    dL/dpred = sign(p - clamp(target)) / B, sign(0) = 0, with p = pred (targets
    clamped only) or p = clamp(pred) times the clamp's derivative, 1 for
    |pred| < s and 0 otherwise (clamp_pred).
    Through a softplus layer: dz = dh * sigmoid(z); dW = dz^T h_prev; db = sum dz;
    dh_prev = dz W.

    The loss is not smooth: the sign and the clamp's derivative are decisions taken
    on the prediction.  `decide` (optional, [B]) supplies the predictions they are
    taken on -- e.g. those of the BF16 rounding points, to compare with a BF16
    implementation in its own precision; by default they are taken on y itself.
    """
    layers = unpack(flat, in_dim, width, n_hidden)
    y, (zs, hs) = forward(flat, in_dim, width, n_hidden, H0)
    B = y.shape[0]
    target = np.asarray(target, np.float64)
    tc = np.clip(target, -sigma, sigma)
    loss = clamped_l1(y, target, sigma, clamp_pred)
    yd = y if decide is None else np.asarray(decide, np.float64)
    if clamp_pred:
        dy = np.where(np.abs(yd) < sigma, np.sign(np.clip(yd, -sigma, sigma) - tc), 0.0) / B
    else:
        dy = np.sign(yd - tc) / B
    grads = [None] * len(layers)
    W, b = layers[-1]
    grads[-1] = (dy[None, :] @ hs[-1], np.array([dy.sum()]))
    dh = dy[:, None] @ W                              # [B][width]
    for l in range(len(layers) - 2, -1, -1):
        dz = dh * sigmoid(zs[l])
        W, b = layers[l]
        grads[l] = (dz.T @ hs[l], dz.sum(axis=0))
        dh = dz @ W
    return loss, pack(grads)


class Adam:
    """Adam as in PyTorch's default form: no weight decay, no amsgrad.

    m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
    """

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.p = np.asarray(params, np.float64).copy()
        self.m = np.zeros_like(self.p)
        self.v = np.zeros_like(self.p)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        self.p = self.p - self.lr * mhat / (np.sqrt(vhat) + self.eps)
        return self.p


def screened_verdicts(delta_hat, delta, eps, tau, certified=True):
    """Verdicts of per-point screening with exact fallback, for one motion per row.

    delta_hat, delta: [M][N].  A point is sent to the exact check iff
    delta_hat < tau.  A motion is a collision iff some checked point has
    delta <= eps; in certified mode a motion with no such witness is checked
    exactly over all its points (as the paper's Alg. 1 confirms every motion it
    reports free with the geometric checker).  Returns (verdict [M] uint8,
    n_fallback [M] int64).
    """
    delta_hat = np.asarray(delta_hat)
    delta = np.asarray(delta)
    sent = delta_hat < tau
    witness = np.any(sent & (delta <= eps), axis=1)
    if certified:
        exact = np.any(delta <= eps, axis=1) if delta.shape[1] else np.zeros(delta.shape[0], bool)
        verdict = np.where(witness, True, exact)
    else:
        verdict = witness
    return verdict.astype(np.uint8), sent.sum(axis=1)


def round_bf16(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64.

    BF16 keeps the top 16 bits of an FP32 word; rounding adds half an ulp of the
    kept part (0x7FFF plus the lowest kept bit, for ties to even) before truncating.
    Inputs are first rounded to FP32.
    """
    f = np.ascontiguousarray(np.asarray(a, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward_bf16(flat, in_dim, width, n_hidden, H0):
    """Debugging aid: the network with the BF16 path's rounding points, otherwise FP64.

    The first layer uses FP32-exact weights and unrounded inputs; its activations,
    like those of every hidden layer except the last, are rounded to BF16 before
    they feed a matrix product; the weights of layers 2..L are rounded to BF16; the
    last hidden activations and the output layer stay unrounded, except for a
    single-layer network, whose output layer reads BF16 activations.
    """
    layers = unpack(flat, in_dim, width, n_hidden)
    h = np.asarray(H0, np.float64)
    for l, (W, b) in enumerate(layers[:-1]):
        Wr = W if l == 0 else round_bf16(W)
        h = softplus(h @ Wr.T + b)
        if l + 1 < n_hidden or n_hidden == 1:
            h = round_bf16(h)
    W, b = layers[-1]
    return (h @ W.T + b)[:, 0]
