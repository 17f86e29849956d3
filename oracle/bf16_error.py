"""A-priori error bars of the BF16 network paths against the FP64 networks.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

The BF16 paths of both networks (the softplus MLP of ``oracle.mlp`` and the
paper's residual network of ``oracle.residual``, Sec. IV-A, Fig. 1; the
paper's "16 bit" variant of Sec. V-A, Table II) differ from the FP64
definitions by rounding only.  Every rounding is a *site* s: a value v_s is
replaced by v_s (1 + delta_s) with |delta_s| <= u_s, or, for an FP32 sum, by a
value within a worst-case magnitude m_s of the exact sum.  To first order the
output error is

    y_bf16 - y_64 = sum_s a_s d_s,   a_s = (dy / dv_s) * m_s,   |d_s| <= 1,

with dy/dv_s the sensitivity of the FP64 output to that value (obtained by
back-propagation through the FP64 network).  Rounding errors are modelled as
independent and of mean zero (the standard probabilistic model of rounding
error analysis); Hoeffding's inequality for a sum of independent bounded
terms then gives, per output,

    P( |sum_s a_s d_s| >= lam * sqrt(sum_s a_s^2) ) <= 2 exp(-lam^2 / 2).

The bar used by the tests is

    |y_bf16 - y_64| <= (1 + kappa) lam sqrt(S2) + D,

with S2 = sum_s a_s^2 over every rounding site, D the worst-case error of the
FP32 output layer (a plain bound, not probabilistic), lam = 7 (2 exp(-24.5)
= 4.6e-11 per output) and kappa = 0.1 for the second-order terms the
expansion leaves out: products of two rounding errors (relative size u =
2^-8 of the first-order ones) and the curvature of the activations (softplus''
<= 1/4, so the remainder is at most e/(8 sigma) of the first-order change e,
below 1% for the errors seen here).

Sites and magnitudes (u = 2^-8: BF16 keeps 8 significand bits and rounds to
nearest even; u32 = 2^-24; gamma_n = n u32 / (1 - n u32), the classical bound
of an n-term FP32 sum):

softplus MLP (layer 1 and the output layer in FP32, hidden layers 2..L on BF16
weights and activations with FP32 accumulation):
  - every hidden-layer weight W_l[f][k], l >= 2:   u |W_l[f][k] h_{l-1}[k]| on z_l[f];
  - every FP32 pre-activation sum z_l[f]:         gamma_{K+1} (sum_k |W_l[f][k] h_{l-1}[k]| + |b_l[f]|);
  - every softplus evaluation (hardware exp2/log2): 2^-20 (1 + |z|) on h_l[f];
  - every activation rounded to BF16:              u |h_l[f]|  (layers 1..L-1, and layer 1 when L = 1);
  - output layer: D = gamma_{W+1} (sum_f |w_f h_L[f]| + |b_out|).

residual network (initial layer in FP32 rounded to BF16; each block one FP32
MFMA sum over [h; x_hi; x_lo] with BF16 weights [Wh | Wx | Wx], then ReLU,
folded BatchNorm and the skip in FP32, the result rounded to BF16 except after
the last block):
  - h_0 sum: gamma_{in+1} (|W_0||x| + |b_0|); h_0 rounding: u |h_0|;
  - weights Wh_b[f][k]: u |Wh h|; Wx_b[f][j]: u |Wx x|;
  - block sum z_b[f]: gamma_{K+1} (sum |Wh h| + sum |Wx x| (1 + 2u) + |c|), K = W + 2 in_dim;
  - the input split x ~ x_hi + x_lo (the remainder rounded to BF16): u^2 (1 + u) |x_j|
    per input j, shared by every block (one site, sensitivity summed over the blocks);
  - the FP32 epilogue h + scale relu(z) + shift with scale = gamma / sqrt(var + eps)
    and shift = beta - scale mu folded in FP32: 8 u32 (|h| + |scale relu(z)| + |beta|
    + |scale mu|) per feature;
  - block results rounded to BF16: u |h_b| (every block but the last);
  - output layer as above.
ReLU's derivative is taken as 1 for z > -m, m = 4 u (sum |Wh h| + sum |Wx x| + |c|):
a rounding that moves z across the kink changes relu(z) by at most |dz|, which
the derivative 1 over that margin covers.

A matrix product (numpy ``@``) is used as a library primitive.
"""
from __future__ import annotations

import numpy as np

from . import mlp as om
from . import residual as ores

U_BF16 = 2.0 ** -8
U_FP32 = 2.0 ** -24
LAM = 7.0
KAPPA = 0.1


def gamma(n: int) -> float:
    return n * U_FP32 / (1.0 - n * U_FP32)


def _softplus_site(z):
    return 2.0 ** -20 * (1.0 + np.abs(z))


def mlp_sites(flat, in_dim, width, n_hidden, H0):
    """(y64 [B], S2 [B], D [B]) of the softplus MLP's BF16 path (see module docstring)."""
    u = U_BF16
    layers = om.unpack(flat, in_dim, width, n_hidden)
    X = np.asarray(H0, np.float64)
    zs, hs = [], [X]
    h = X
    for W, b in layers[:-1]:
        z = h @ W.T + b
        h = om.softplus(z)
        zs.append(z)
        hs.append(h)
    w_out, b_out = layers[-1][0][0], layers[-1][1][0]
    y = h @ w_out + b_out
    B = X.shape[0]
    L = n_hidden
    D = gamma(width + 1) * (np.abs(h) @ np.abs(w_out) + abs(b_out))
    S2 = np.zeros(B)
    g_h = np.broadcast_to(w_out, (B, width)).copy()   # dy/dh_L
    for l in range(L, 0, -1):                         # hidden layer l (1-based)
        z, h_l, h_prev = zs[l - 1], hs[l], hs[l - 1]
        W, b = layers[l - 1]
        rounded = (l < L) or (L == 1)
        S2 += np.sum((g_h * _softplus_site(z)) ** 2, axis=1)
        if rounded:
            S2 += u * u * np.sum((g_h * h_l) ** 2, axis=1)
        g_z = g_h * om.sigmoid(z)
        absum = np.abs(h_prev) @ np.abs(W).T + np.abs(b)
        K = W.shape[1]
        S2 += np.sum((g_z * gamma(K + 1) * absum) ** 2, axis=1)
        if l >= 2:
            S2 += u * u * np.sum(g_z ** 2 * ((h_prev ** 2) @ (W ** 2).T), axis=1)
        g_h = g_z @ W
    return y, S2, D


def mlp_bar(flat, in_dim, width, n_hidden, H0, lam=LAM, kappa=KAPPA, chunk=4096):
    """(y64 [B], bar [B]): per-output bound of |y_bf16 - y_64| for the softplus MLP."""
    H0 = np.asarray(H0, np.float64)
    ys, bars = [], []
    for s in range(0, H0.shape[0], chunk):
        y, S2, D = mlp_sites(flat, in_dim, width, n_hidden, H0[s:s + chunk])
        ys.append(y)
        bars.append((1.0 + kappa) * lam * np.sqrt(S2) + D)
    if not ys:
        return np.zeros(0), np.zeros(0)
    return np.concatenate(ys), np.concatenate(bars)


def residual_sites(flat, in_dim, width, n_blocks, X, bn_eps):
    """(y64 [B], S2 [B], D [B]) of the residual network's BF16 path (see module docstring)."""
    u, u32 = U_BF16, U_FP32
    net = ores.unpack(flat, in_dim, width, n_blocks)
    X = np.asarray(X, np.float64)
    B = X.shape[0]
    absX = np.abs(X)
    h = X @ net["W0"].T + net["b0"]
    hs, zs, aux = [h], [], []
    for blk in net["blocks"]:
        zh = h @ blk["Wh"].T
        zx = X @ blk["Wx"].T
        z = zh + zx + blk["c"]
        scale = blk["gamma"] / np.sqrt(blk["var"] + bn_eps)
        a = np.maximum(z, 0.0)
        sh = np.abs(h) @ np.abs(blk["Wh"]).T
        sx = absX @ np.abs(blk["Wx"]).T
        margin = 4.0 * u * (sh + sx + np.abs(blk["c"]))
        aux.append((scale, a, sh, sx, margin))
        h = h + scale * (a - blk["mu"]) + blk["beta"]
        zs.append(z)
        hs.append(h)
    w_out, b_out = net["w_out"], net["b_out"]
    y = h @ w_out + b_out
    D = gamma(width + 1) * (np.abs(h) @ np.abs(w_out) + abs(b_out))
    S2 = np.zeros(B)
    g_h = np.broadcast_to(w_out, (B, width)).copy()        # dy/dh_L
    g_x = np.zeros((B, in_dim))                            # dy/dx through the blocks' Wx terms
    K = width + 2 * in_dim
    for b in range(n_blocks - 1, -1, -1):
        blk = net["blocks"][b]
        scale, a, sh, sx, margin = aux[b]
        h_prev, h_b, z = hs[b], hs[b + 1], zs[b]
        if b + 1 < n_blocks:
            S2 += u * u * np.sum((g_h * h_b) ** 2, axis=1)                       # block result -> BF16
        epi = 8.0 * u32 * (np.abs(h_prev) + np.abs(scale * a) + np.abs(blk["beta"]) + np.abs(scale * blk["mu"]))
        S2 += np.sum((g_h * epi) ** 2, axis=1)                                   # FP32 epilogue
        g_z = g_h * scale * (z > -margin)
        S2 += np.sum((g_z * gamma(K + 1) * (sh + sx * (1 + 2 * u) + np.abs(blk["c"]))) ** 2, axis=1)
        S2 += u * u * np.sum(g_z ** 2 * ((h_prev ** 2) @ (blk["Wh"] ** 2).T), axis=1)
        S2 += u * u * np.sum(g_z ** 2 * ((X ** 2) @ (blk["Wx"] ** 2).T), axis=1)
        g_x += g_z @ blk["Wx"]
        g_h = g_h + g_z @ blk["Wh"]
    # input split (one site per input, shared by all blocks), h_0 rounding and its FP32 sum
    S2 += np.sum((g_x * u * u * (1 + u) * absX) ** 2, axis=1)
    S2 += u * u * np.sum((g_h * hs[0]) ** 2, axis=1)
    S2 += np.sum((g_h * gamma(in_dim + 1) * (absX @ np.abs(net["W0"]).T + np.abs(net["b0"]))) ** 2, axis=1)
    return y, S2, D


def residual_bar(flat, in_dim, width, n_blocks, X, bn_eps, lam=LAM, kappa=KAPPA, chunk=4096):
    """(y64 [B], bar [B]): per-output bound of |y_bf16 - y_64| for the residual network."""
    X = np.asarray(X, np.float64)
    ys, bars = [], []
    for s in range(0, X.shape[0], chunk):
        y, S2, D = residual_sites(flat, in_dim, width, n_blocks, X[s:s + chunk], bn_eps)
        ys.append(y)
        bars.append((1.0 + kappa) * lam * np.sqrt(S2) + D)
    if not ys:
        return np.zeros(0), np.zeros(0)
    return np.concatenate(ys), np.concatenate(bars)


# Median criterion of a BF16 implementation against the emulation of its rounding points
# (``oracle.mlp.forward_bf16``, ``oracle.residual.forward_bf16``).  Both round at the same
# sites; they differ by FP32 against FP64 arithmetic between the roundings (relative size
# about 2^-24 sqrt(K), four orders below the BF16 unit roundoff that scales the bar) and
# by the rare roundings that this difference moves to the neighbouring BF16 value.  The
# median row has none of those, so it sits far below 0.5% of its bar, while every
# plausible misplacement of a rounding point moves the median row by 1% of the bar or
# more (tests/test_oracle_bf16_error.py plants them).
MEDIAN_FRACTION = 0.005


def compare(y, y_em, y64, bar):
    """Check a BF16 result y against the FP64 network (y64) and the rounding emulation
    (y_em), with the per-output bar of ``mlp_bar`` / ``residual_bar``:
      |y - y64| <= bar and |y - y_em| <= bar for every output,
      median |y - y_em| / bar <= MEDIAN_FRACTION.
    Returns (ok, report dict)."""
    y, y_em, y64, bar = (np.asarray(a, np.float64).ravel() for a in (y, y_em, y64, bar))
    e64 = np.abs(y - y64)
    eem = np.abs(y - y_em)
    rep = {"n": int(y.size), "max_err_fp64": float(e64.max()) if y.size else 0.0,
           "median_err_fp64": float(np.median(e64)) if y.size else 0.0,
           "max_err_over_bar": float(np.max(e64 / bar)) if y.size else 0.0,
           "max_emul_over_bar": float(np.max(eem / bar)) if y.size else 0.0,
           "median_emul_over_bar": float(np.median(eem / bar)) if y.size else 0.0,
           "median_bar": float(np.median(bar)) if y.size else 0.0}
    ok = bool(np.all(e64 <= bar) and np.all(eem <= bar)) and rep["median_emul_over_bar"] <= MEDIAN_FRACTION
    return ok, rep
