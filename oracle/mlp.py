"""The learned skip gate (an extension beyond the paper) in float64: a
perceptron in -> H -> H -> 1 with ReLU, trained by mean squared error with
Adam (Kingma and Ba, "Adam: A Method for Stochastic Optimization", 2015).
Test infrastructure only.

Parameter vector layout (shared with the library's C ABI):
  W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1].

Features of a screened edge (in = 2r + 4), built from the same quantities
as Algorithm 3: w/|w| with w = P q_res, u_d = P d_res / |P d_res|,
t_hat = cos(P q_res, P d_res), |q_res|/ub, |d_res|/ub and
|q_proj - d_proj|^2 / ub^2, where ub^2 is the screening bound.  The target
is the true cos(q_res, d_res); the gated estimate is Eq. 2 with
t = f(x) + eps_gate.
"""
from __future__ import annotations

import numpy as np

from .build import split
from .codes import round_bf16
from .estimate import combine, dm_map, parts


def n_params(in_dim: int, H: int) -> int:
    return H * in_dim + H * H + 3 * H + 1


def unpack(w: np.ndarray, in_dim: int, H: int):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + H * in_dim].reshape(H, in_dim); o += H * in_dim
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    W3 = w[o:o + H]; o += H
    b3 = w[o]
    return W1, b1, W2, b2, W3, b3


def init_params(in_dim: int, H: int, seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, in_dim)) * np.sqrt(6.0 / in_dim)
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    W3 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, [0.0]])


def forward(w, X, in_dim: int, H: int, keep: bool = False, bf16_operands: bool = False):
    """Network output.  With ``bf16_operands`` the weights, the inputs and
    both hidden layers are rounded to bfloat16 before each product (biases
    stay exact), the operand precision the library's kernels use; the
    arithmetic itself stays float64."""
    W1, b1, W2, b2, W3, b3 = unpack(w, in_dim, H)
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    r = round_bf16 if bf16_operands else (lambda a: a)
    z1 = r(X) @ r(W1).T + b1
    h1 = r(np.maximum(z1, 0))
    z2 = h1 @ r(W2).T + b2
    h2 = r(np.maximum(z2, 0))
    y = h2 @ r(W3) + b3
    if keep:
        return y, (X, z1, h1, z2, h2)
    return y


def loss_and_grad(w, X, t, in_dim: int, H: int, bf16_operands: bool = False):
    """Mean squared error over the batch and its gradient, by the chain rule
    written out layer by layer.

    With ``bf16_operands`` every factor of every product is a bfloat16 value
    (the precision the library's matrix-core kernels compute in): the
    forward pass as in ``forward``, and in the backward pass the weights and
    the back-propagated errors dz2, dz1 are rounded before they multiply;
    dL/dy itself, the bias gradients (plain sums) and all accumulation stay
    float64."""
    W1, b1, W2, b2, W3, b3 = unpack(w, in_dim, H)
    y, (X, z1, h1, z2, h2) = forward(w, X, in_dim, H, keep=True, bf16_operands=bf16_operands)
    r = round_bf16 if bf16_operands else (lambda a: a)
    B = X.shape[0]
    e = y - np.asarray(t, dtype=np.float64)
    loss = float((e * e).mean())
    dy = 2.0 * e / B                     # dL/dy
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, r(W3)) * (z2 > 0)  # dL/dz2
    gW2 = r(dz2).T @ h1
    gb2 = dz2.sum(0)
    dz1 = (r(dz2) @ r(W2)) * (z1 > 0)    # dL/dz1
    gW1 = r(dz1).T @ r(X)
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def adam_step(w, g, m1, m2, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update with bias correction; returns new (w, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2


def edge_features(q, c, D, P, ub2: float) -> np.ndarray:
    """Gate features of each neighbour row of D (in the parameter layout's
    input order), from the definitions (no factorized tables)."""
    q = np.asarray(q, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    D = np.atleast_2d(np.asarray(D, dtype=np.float64))
    p = parts(q, c, D, P)
    _, _, qr = split(q, c)
    _, _, dr = split(D, c)
    w = P @ qr
    nw = np.sqrt(w @ w)
    wn = w / nw if nw > 0 else np.zeros_like(w)
    Pd = dr @ P.T
    nd = np.sqrt((Pd * Pd).sum(1, keepdims=True))
    U = np.where(nd > 0, Pd / np.where(nd > 0, nd, 1.0), 0.0)
    ub = np.sqrt(ub2)
    inv = 1.0 / ub if ub > 0 else 0.0
    F = np.empty((D.shape[0], 2 * P.shape[0] + 4))
    r = P.shape[0]
    F[:, :r] = wn
    F[:, r:2 * r] = U
    F[:, 2 * r] = p["t_hat"]
    F[:, 2 * r + 1] = p["rq"] * inv
    F[:, 2 * r + 2] = p["rd"] * inv
    F[:, 2 * r + 3] = p["proj"] * inv * inv
    return F


def target_cosine(d2, q_res_norm, d_res_norm, proj):
    """cos(q_res, d_res) recovered from an exact squared distance through
    Eq. 2: q_res.d_res = (|q_proj - d_proj|^2 + |q_res|^2 + |d_res|^2 - d2) / 2."""
    den = 2.0 * q_res_norm * d_res_norm
    num = proj + q_res_norm ** 2 + d_res_norm ** 2 - d2
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def gated_estimate(q, c, D, tables: dict, w, H: int, eps_gate: float, ub2: float,
                   bf16_operands: bool = True, band: float = 0.0) -> np.ndarray:
    """Eq. 2 with t = f(features) + eps_gate (the gated screen).  With
    ``band`` > 0 a cascade: an edge keeps Algorithm 3's estimate unless that
    estimate lies within band * ub2 of the bound ub2, and only those edges
    take the network's."""
    P = tables["P"]
    F = edge_features(q, c, D, P, ub2)
    t = forward(w, F, F.shape[1], H, bf16_operands=bf16_operands) + eps_gate
    p = parts(q, c, D, P)
    est = p["proj"] + p["rq"] ** 2 + p["rd"] ** 2 - 2 * p["rq"] * p["rd"] * t
    if band > 0:
        est_dm = combine(p, dm_map(p["t_hat"], tables))
        est = np.where(np.abs(est_dm - ub2) <= band * ub2, est, est_dm)
    return est
