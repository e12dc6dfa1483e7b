"""Hand-worked pins for the oracle's construction (Algorithm 2), estimate
(Algorithm 3) and the learned gate's network, from the cases under
tests/golden/ whose expected values were derived by hand from the
definitions (see each file's derivation).  They are chosen so that the
plausible slips fail: cosines of raw vectors instead of residuals, a
squared or unnormalised cosine, the variance where the standard deviation
belongs, a dropped or sign-flipped correction term, a transposed layer.
CPU only."""
import json
import os

import numpy as np
import pytest

from oracle.build import build, cosine_rows, dm_stats, residual_pairs
from oracle.estimate import combine, dm_map, estimate, parts, true_cosine
from oracle.mlp import forward, loss_and_grad, n_params

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------ Algorithm 2

@pytest.fixture(scope="module")
def alg2():
    return _load("algorithm2_case.json")


def test_algorithm2_residual_cosines(alg2):
    data = np.array(alg2["points"], dtype=np.float64)
    G = np.array(alg2["graph"], dtype=np.int32)
    P = np.array(alg2["basis"], dtype=np.float64)
    t = build(data, G, 2, n_samples=100_000, seed=0, basis=P)
    c, d, dp, _ = t["samples"]
    assert c.tolist() == alg2["centres"]
    np.testing.assert_allclose(t["X"], alg2["X"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(t["Y"], alg2["Y"], rtol=0, atol=1e-12)
    # the same cosines from the pieces: residuals w.r.t. each centre
    R, R2 = residual_pairs(data, c, d, dp)
    np.testing.assert_allclose(cosine_rows(R, R2), alg2["X"], atol=1e-12)
    # the raw-vector reading gives different values on this case
    raw = cosine_rows(data[d], data[dp])
    np.testing.assert_allclose(raw, alg2["raw_vector_X"], atol=1e-12)
    assert np.abs(raw - np.array(alg2["X"])).max() > 0.5


@pytest.mark.parametrize("mode", ["std", "variance"])
def test_algorithm2_matching_statistics(alg2, mode):
    data = np.array(alg2["points"], dtype=np.float64)
    G = np.array(alg2["graph"], dtype=np.int32)
    P = np.array(alg2["basis"], dtype=np.float64)
    t = build(data, G, 2, n_samples=100_000, seed=0, basis=P, sigma_mode=mode)
    for key, v in alg2[mode].items():
        assert t[key] == pytest.approx(v, abs=1e-12), key
    assert t["corr"] == pytest.approx(alg2["corr"], abs=1e-12)
    # dm_stats alone on the hand values of X and Y
    s = dm_stats(np.array(alg2["X"]), np.array(alg2["Y"]), mode)
    for key, v in alg2[mode].items():
        assert s[key] == pytest.approx(v, abs=1e-12), key


def test_algorithm2_std_and_variance_readings_differ(alg2):
    assert abs(alg2["std"]["sigma"] - alg2["variance"]["sigma"]) > 0.2
    assert abs(alg2["std"]["eps"] - alg2["variance"]["eps"]) > 0.05


# ------------------------------------------------------------ Algorithm 3

@pytest.fixture(scope="module")
def alg3():
    return _load("algorithm3_case.json")


def _alg3_tables(case, identity=False):
    t = {"P": np.array(case["basis"], dtype=np.float64)}
    t.update(case["dm"])
    if identity:
        t.update(mu=0.0, sigma=1.0, mu_hat=0.0, sigma_hat=1.0, eps=0.0)
    return t


def test_algorithm3_estimate_with_matching(alg3):
    q, c, D = (np.array(alg3[k], dtype=np.float64) for k in ("query", "centre", "neighbours"))
    tab = _alg3_tables(alg3)
    p = parts(q, c, D, tab["P"])
    np.testing.assert_allclose(p["t_hat"], alg3["t_hat"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(estimate(q, c, D, tab), alg3["est"], rtol=0, atol=1e-12)
    # the matched cosine itself: (t_hat - mu_hat) sigma / sigma_hat + mu + eps
    np.testing.assert_allclose(dm_map(p["t_hat"], tab),
                               [2 / np.sqrt(5) - 0.25, 6 / np.sqrt(10) - 0.25], atol=1e-14)
    np.testing.assert_allclose(estimate(q, c, D, _alg3_tables(alg3, identity=True)),
                               alg3["est_identity_dm"], rtol=0, atol=1e-12)


def test_algorithm3_decomposition_is_exact_with_the_true_cosine(alg3):
    """Eq. 2 with the true residual cosine in place of t returns the exact
    squared distances."""
    q, c, D = (np.array(alg3[k], dtype=np.float64) for k in ("query", "centre", "neighbours"))
    p = parts(q, c, D, np.array(alg3["basis"], dtype=np.float64))
    tc = true_cosine(q, c, D)
    np.testing.assert_allclose(tc, alg3["true_cosine"], atol=1e-14)
    np.testing.assert_allclose(combine(p, tc), alg3["exact_d2"], atol=1e-12)
    np.testing.assert_allclose(((D - q) ** 2).sum(1), alg3["exact_d2"], atol=0)


# ------------------------------------------------------------- the gate

@pytest.fixture(scope="module")
def gate():
    return _load("gate_mlp_case.json")


def _gate_params(case):
    w = case["weights"]
    return np.concatenate([np.ravel(w["W1"]), w["b1"], np.ravel(w["W2"]), w["b2"], w["W3"], [w["b3"]]])


@pytest.mark.parametrize("bf16", [False, True])
def test_gate_forward_hand_values(gate, bf16):
    w = _gate_params(gate)
    assert w.size == n_params(gate["in_dim"], gate["hidden"])
    for row in gate["forward"]:
        y, (X, z1, h1, z2, h2) = forward(w, [row["x"]], gate["in_dim"], gate["hidden"], keep=True,
                                         bf16_operands=bf16)
        assert y[0] == row["y"]
        assert z1[0].tolist() == row["z1"] and h1[0].tolist() == row["h1"]
        assert z2[0].tolist() == row["z2"] and h2[0].tolist() == row["h2"]


@pytest.mark.parametrize("bf16", [False, True])
def test_gate_backward_hand_values(gate, bf16):
    w = _gate_params(gate)
    b = gate["backward"]
    loss, g = loss_and_grad(w, np.array(b["x"], dtype=np.float64), np.array(b["target"]),
                            gate["in_dim"], gate["hidden"], bf16_operands=bf16)
    assert loss == b["loss"]
    gg = b["grad"]
    want = np.concatenate([np.ravel(gg["W1"]), gg["b1"], np.ravel(gg["W2"]), gg["b2"], gg["W3"],
                           [gg["b3"]]])
    assert g.tolist() == want.tolist()
