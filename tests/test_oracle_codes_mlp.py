"""Pins for the oracle's low-precision code rounding and the gate network.
CPU only."""
import numpy as np
import pytest
import torch

from oracle.codes import (E4M3_MAX, e4m3_values, fp8_node_scale, quantize_codes, round_bf16,
                          round_e4m3)
from oracle.mlp import (adam_step, edge_features, forward, init_params, loss_and_grad,
                        n_params, target_cosine)
from oracle.estimate import parts, true_cosine


def test_bf16_matches_library_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000), rng.normal(size=2000) * 1e-3,
                        rng.uniform(-1, 1, 2000)]).astype(np.float32)
    # exact ties: float32 values halfway between bf16 neighbours
    base = rng.normal(size=500).astype(np.float32).view(np.uint32) & 0xFFFF0000
    ties = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, ties])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x.astype(np.float64)), want)


def test_e4m3_code_values_closed_form():
    v = e4m3_values()
    assert v[0x7E] == 448.0 and v[0x08] == 2.0 ** -6 and v[0x01] == 2.0 ** -9
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    fin = v[np.isfinite(v)]
    # every finite code value rounds to itself
    np.testing.assert_array_equal(round_e4m3(fin), fin)
    # midpoints between neighbours round to the one with an even mantissa
    pos = np.unique(fin[fin > 0])
    mids = (pos[:-1] + pos[1:]) / 2
    got = round_e4m3(mids)
    codes = {val: b for b, val in enumerate(v) if np.isfinite(val) and val > 0}
    for m, g in zip(mids, got):
        assert g in (pos[pos < m].max(), pos[pos > m].min())
        assert codes[g] % 2 == 0


def test_e4m3_matches_library_conversion_and_saturates():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20000), rng.normal(size=5000),
                        rng.normal(size=2000) * 1e-2]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_e4m3(x.astype(np.float64)), want)
    assert round_e4m3(np.array([500.0, -1e6, 463.9]))[0] == E4M3_MAX
    assert round_e4m3(np.array([-1e6]))[0] == -E4M3_MAX


def test_quantization_error_within_half_ulp():
    rng = np.random.default_rng(2)
    U = rng.normal(size=(32, 64))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    b = quantize_codes(U, "bf16")
    assert np.all(np.abs(b - U) <= np.abs(U) * 2.0 ** -8 + 1e-300)
    f = quantize_codes(U, "fp8")
    s = fp8_node_scale(U)
    # relative half-ulp of 3 mantissa bits for normals, 2^-10 s below 2^-6 s
    bound = np.maximum(np.abs(U) * 2.0 ** -4, 2.0 ** -10 * s)
    assert np.all(np.abs(f - U) <= bound + 1e-15)
    assert np.max(np.abs(U)) / s == pytest.approx(448.0)


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    in_dim, H = 11, 7
    # random biases keep pre-activations away from the ReLU kink at 0
    w = init_params(in_dim, H, seed=4) + rng.normal(size=n_params(in_dim, H)) * 0.1
    X = rng.normal(size=(17, in_dim))
    t = rng.normal(size=17)
    loss, g = loss_and_grad(w, X, t, in_dim, H)
    assert g.shape == (n_params(in_dim, H),)
    h = 1e-6
    fd = np.empty_like(w)
    for i in range(w.size):
        e = np.zeros_like(w)
        e[i] = h
        fd[i] = (loss_and_grad(w + e, X, t, in_dim, H)[0] - loss_and_grad(w - e, X, t, in_dim, H)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_adam_first_step_is_signed_lr():
    """With zero moments the bias-corrected first Adam step is
    -lr g / (|g| + eps), i.e. -lr sign(g) for |g| >> eps."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    w, m1, m2 = adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(w, -0.01 * g / (np.abs(g) + 1e-8))


def test_features_and_target_are_consistent():
    """The target recovered from the exact distance through Eq. 2 is the
    true residual cosine; t_hat is the low-rank cosine."""
    rng = np.random.default_rng(5)
    q, c = rng.normal(size=12) * 2, rng.normal(size=12) * 2
    D = c + rng.normal(size=(6, 12))
    P, _ = np.linalg.qr(rng.normal(size=(12, 5)))
    P = P.T
    F = edge_features(q, c, D, P, ub2=9.0)
    p = parts(q, c, D, P)
    d2 = ((D - q) ** 2).sum(1)
    tgt = target_cosine(d2, p["rq"], p["rd"], p["proj"])
    np.testing.assert_allclose(tgt, true_cosine(q, c, D), rtol=1e-10)
    np.testing.assert_allclose(F[:, 10], p["t_hat"])
    np.testing.assert_allclose(np.linalg.norm(F[:, :5], axis=1), 1.0)
    np.testing.assert_allclose(F[:, 11], p["rq"] / 3.0)
    assert forward(init_params(14, 8), F, 14, 8).shape == (6,)
